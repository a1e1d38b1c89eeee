"""FP64 oracle of EvSNet: conv3x3 layers feeding BiLIF units, and its BPTT.

Test infrastructure only (see the package docstring).  All arithmetic is
numpy float64; the caller passes float64 copies of the exact float32 inputs.

Network (per frame t, layer l = 1..L, s_0[t] = x[t]):

    u_l[t] = conv3x3(s_{l-1}[t], W_l)             zero "same" padding, no bias
    h_l[t] = beta * v_l[t-1] + u_l[t]             charge, Sec. 3.3 Eq. (2)
    s_l[t] = +1 if h >= theta, -1 if h <= -theta  bipolar fire, Eq. (3)
    v_l[t] = h_l[t] - theta * s_l[t]              reset by the threshold

Readings of the paper used here: the leak beta = 1 - 1/tau multiplies only
the carried potential; BiLIF fires on the charged potential (the V' of
Eq. (2)); both thresholds are inclusive; the reset subtracts theta * s so a
saturated pixel keeps firing once per frame while |h| >= theta (the
saturation effect of Sec. 3.1); the membrane starts at zero unless an
initial state is given (the internal-state bias of Sec. 3.1).

Backward: the Heaviside in the fire step is replaced by the surrogate of
Eq. (4), read as the total derivative of sigma(h - theta) - sigma(-h - theta):

    psi(h) = sigma'(h - theta) + sigma'(-h - theta)

with one of two smooth steps sigma (argument ``surr``):
    "sigmoid"  sigma(z) = 1 / (1 + exp(-alpha z)),   sigma' = alpha s (1 - s)
    "atan"     the arctangent surrogate the paper trains with (Sec. 3.3, the
               formula itself is not printed; read as the usual arctangent
               step) sigma(z) = 1/2 + arctan(pi/2 alpha z) / pi,
               sigma'(z) = (alpha / 2) / (1 + (pi/2 alpha z)^2)
"""

from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# convolution (cross-correlation, zero padding) and its adjoints
# ----------------------------------------------------------------------------

def conv3x3(s: np.ndarray, w: np.ndarray) -> np.ndarray:
    """u[c,y,x] = sum_{c',i,j} w[c,c',i,j] * s[c', y+i-1, x+j-1]; s outside is 0."""
    cin, H, W = s.shape
    p = np.zeros((cin, H + 2, W + 2))
    p[:, 1:-1, 1:-1] = s
    u = np.zeros((w.shape[0], H, W))
    for i in range(3):
        for j in range(3):
            u += np.tensordot(w[:, :, i, j], p[:, i:i + H, j:j + W], axes=([1], [0]))
    return u


def conv3x3_transpose(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 w.r.t. its input: returns dL/ds given g = dL/du."""
    cout, H, W = g.shape
    p = np.zeros((cout, H + 2, W + 2))
    p[:, 1:-1, 1:-1] = g
    out = np.zeros((w.shape[1], H, W))
    for i in range(3):
        for j in range(3):
            out += np.tensordot(w[:, :, i, j], p[:, 2 - i:2 - i + H, 2 - j:2 - j + W],
                                axes=([0], [0]))
    return out


def conv3x3_weight_grad(g: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 w.r.t. its weights: dW[c,c',i,j] = sum g[c,y,x] s[c',y+i-1,x+j-1]."""
    cin, H, W = s.shape
    p = np.zeros((cin, H + 2, W + 2))
    p[:, 1:-1, 1:-1] = s
    dw = np.zeros((g.shape[0], cin, 3, 3))
    for i in range(3):
        for j in range(3):
            dw[:, :, i, j] = np.tensordot(g, p[:, i:i + H, j:j + W], axes=([1, 2], [1, 2]))
    return dw


# ----------------------------------------------------------------------------
# spiking unit
# ----------------------------------------------------------------------------

def fire(h: np.ndarray, theta: float) -> np.ndarray:
    """Bipolar fire of Eq. (3): sign(h) where |h| >= theta, else 0."""
    return np.where(h >= theta, 1.0, np.where(h <= -theta, -1.0, 0.0))


def sigmoid(z: np.ndarray, alpha: float) -> np.ndarray:
    return 0.5 * (1.0 + np.tanh(0.5 * alpha * z))


def atan_step(z: np.ndarray, alpha: float) -> np.ndarray:
    """Arctangent step 1/2 + arctan(pi/2 alpha z) / pi."""
    return 0.5 + np.arctan(0.5 * np.pi * alpha * z) / np.pi


def step(z: np.ndarray, alpha: float, surr: str = "sigmoid") -> np.ndarray:
    if surr == "sigmoid":
        return sigmoid(z, alpha)
    if surr == "atan":
        return atan_step(z, alpha)
    raise ValueError(surr)


def step_slope(z: np.ndarray, alpha: float, surr: str = "sigmoid") -> np.ndarray:
    """Derivative of step(z)."""
    if surr == "sigmoid":
        a = sigmoid(z, alpha)
        return alpha * a * (1.0 - a)
    if surr == "atan":
        q = 0.5 * np.pi * alpha * z
        return 0.5 * alpha / (1.0 + q * q)
    raise ValueError(surr)


def relaxed_fire(h: np.ndarray, theta: float, alpha: float, surr: str = "sigmoid") -> np.ndarray:
    """Smooth spike sigma(h - theta) - sigma(-h - theta) whose derivative is psi."""
    return step(h - theta, alpha, surr) - step(-h - theta, alpha, surr)


def surrogate(h: np.ndarray, theta: float, alpha: float, surr: str = "sigmoid") -> np.ndarray:
    """psi(h): surrogate dS/dh of Eq. (4) with slope alpha."""
    return step_slope(h - theta, alpha, surr) + step_slope(-h - theta, alpha, surr)


# ----------------------------------------------------------------------------
# BF16 operand quantisation (the precision form rounds x and W, not spikes)
# ----------------------------------------------------------------------------

def bf16_round(a) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float64.

    bfloat16 keeps the upper 16 bits of an IEEE float32; rounding adds half a
    unit of the dropped 16 bits plus the kept lowest bit (ties to even).
    """
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000)
    quiet = np.where((u & 0xFFFF) != 0, np.uint64(0x400000), np.uint64(0))
    r = np.where(special, (u & np.uint64(0xFFFF0000)) | quiet, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# forward
# ----------------------------------------------------------------------------

def forward(x, weights, theta, leak, v_init=None, mode="hard", alpha=4.0,
            reset_unit=None, keep_traces=True, surr="sigmoid"):
    """Run the network over a clip.

    x        [T, C0, H, W]
    weights  list of [C_l, C_{l-1}, 3, 3]
    v_init   None or list of [C_l, H, W] initial membrane potentials
    mode     "hard"    -- Eq. (3) spikes
             "relaxed" -- relaxed_fire for output and reset (smooth; its exact
                          gradient is the surrogate BPTT)
             "hybrid"  -- relaxed output, hard spikes in the reset (its exact
                          gradient is the surrogate BPTT with a detached reset)
    reset_unit  None: v = h - theta*s; a number r: v = h - r*s (Eq. (2) taken
                literally is r = 1)

    Returns dict with "s" (= s_L, [T, C_L, H, W]), "h" and "spk" (per-layer
    traces, lists of [T, C_l, H, W]) and "v" (final states, per layer).
    """
    x = np.asarray(x, dtype=np.float64)
    T, _, H, W = x.shape
    L = len(weights)
    ws = [np.asarray(w, dtype=np.float64) for w in weights]
    r = theta if reset_unit is None else reset_unit
    v = [np.zeros((w.shape[0], H, W)) if v_init is None else np.array(v_init[l], dtype=np.float64)
         for l, w in enumerate(ws)]
    h_tr = [np.zeros((T, w.shape[0], H, W)) for w in ws] if keep_traces else None
    s_tr = [np.zeros((T, w.shape[0], H, W)) for w in ws] if keep_traces else None
    out = np.zeros((T, ws[-1].shape[0], H, W))
    for t in range(T):
        s_in = x[t]
        for l in range(L):
            h = leak * v[l] + conv3x3(s_in, ws[l])
            if mode == "hard":
                s = fire(h, theta)
                rs = s
            elif mode == "relaxed":
                s = relaxed_fire(h, theta, alpha, surr)
                rs = s
            elif mode == "hybrid":
                s = relaxed_fire(h, theta, alpha, surr)
                rs = fire(h, theta)
            else:
                raise ValueError(mode)
            v[l] = h - r * rs
            if keep_traces:
                h_tr[l][t] = h
                s_tr[l][t] = s
            s_in = s
        out[t] = s_in
    return {"s": out, "h": h_tr, "spk": s_tr, "v": v}


# ----------------------------------------------------------------------------
# BPTT backward with segment checkpointing
# ----------------------------------------------------------------------------

def backward(x, weights, theta, leak, grad_s, v_init=None, mode="hard", alpha=4.0,
             detach_reset=False, ckpt_every=None, surr="sigmoid"):
    """Surrogate-gradient BPTT through the whole clip.

    grad_s  [T, C_L, H, W] = dLoss/ds_L[t]
    Returns dict with "dW" (list like weights), "dx" [T, C0, H, W] and
    "dv_init" (list of [C_l, H, W]).

    The adjoint of one BiLIF step, with g_v = dL/dv[t] arriving from t+1:
        g_h = (G - theta * g_v) * psi(h) + g_v     (reset not detached)
        g_h = G * psi(h) + g_v                      (detached reset)
        dL/dv[t-1] = beta * g_h,   dL/du[t] = g_h
    Checkpointing: the membrane of every layer is stored at the start of each
    segment of ``ckpt_every`` frames; each segment's traces are recomputed
    from its checkpoint while the segments are visited in reverse.
    """
    x = np.asarray(x, dtype=np.float64)
    T, C0, H, W = x.shape
    ws = [np.asarray(w, dtype=np.float64) for w in weights]
    L = len(ws)
    k = T if ckpt_every is None else int(ckpt_every)
    # forward pass keeping only the segment-start states
    starts = list(range(0, T, k))
    ckpts = []
    v = [np.zeros((w.shape[0], H, W)) if v_init is None else np.array(v_init[l], dtype=np.float64)
         for l, w in enumerate(ws)]
    for t0 in starts:
        ckpts.append([vl.copy() for vl in v])
        seg = forward(x[t0:t0 + k], ws, theta, leak, v_init=v, mode=mode, alpha=alpha,
                      keep_traces=False, surr=surr)
        v = seg["v"]
    dW = [np.zeros_like(w) for w in ws]
    dx = np.zeros_like(x)
    g_v = [np.zeros((w.shape[0], H, W)) for w in ws]
    for si in reversed(range(len(starts))):
        t0 = starts[si]
        t1 = min(T, t0 + k)
        seg = forward(x[t0:t1], ws, theta, leak, v_init=ckpts[si], mode=mode, alpha=alpha, surr=surr)
        for tt in reversed(range(t1 - t0)):
            t = t0 + tt
            G = np.asarray(grad_s[t], dtype=np.float64)
            for l in reversed(range(L)):
                h = seg["h"][l][tt]
                psi = surrogate(h, theta, alpha, surr)
                if detach_reset:
                    g_h = G * psi + g_v[l]
                else:
                    g_h = (G - theta * g_v[l]) * psi + g_v[l]
                s_in = x[t] if l == 0 else seg["spk"][l - 1][tt]
                dW[l] += conv3x3_weight_grad(g_h, s_in)
                G = conv3x3_transpose(g_h, ws[l])
                g_v[l] = leak * g_h
            dx[t] = G
    return {"dW": dW, "dx": dx, "dv_init": g_v}


def backward_along(x, weights, theta, leak, grad_s, h_traj, alpha=4.0, detach_reset=False,
                   surr="sigmoid"):
    """The BPTT backward of Eq. (4) along a given trajectory of hard spikes.

    h_traj  list over layers of [T, C_l, H, W] charged potentials (e.g. the
            device's own trace).  Everything the backward needs from the
            forward is a function of them: the spikes s_l = fire(h_l) (the
            input of layer l+1 and of its weight gradient) and the surrogate
            psi(h_l).  No forward is run here, so a device whose FP32 sums put
            a potential on the other side of a threshold than FP64 would is
            still checked step by step.  With the oracle's own trajectory
            this is the same computation as ``backward`` with mode "hard".

    Returns dict with "dW", "dx" and "dv_init" as ``backward`` does.
    """
    x = np.asarray(x, dtype=np.float64)
    T, C0, H, W = x.shape
    ws = [np.asarray(w, dtype=np.float64) for w in weights]
    L = len(ws)
    dW = [np.zeros_like(w) for w in ws]
    dx = np.zeros_like(x)
    g_v = [np.zeros((w.shape[0], H, W)) for w in ws]
    for t in reversed(range(T)):
        G = np.asarray(grad_s[t], dtype=np.float64)
        for l in reversed(range(L)):
            h = np.asarray(h_traj[l][t], dtype=np.float64)
            psi = surrogate(h, theta, alpha, surr)
            if detach_reset:
                g_h = G * psi + g_v[l]
            else:
                g_h = (G - theta * g_v[l]) * psi + g_v[l]
            s_in = x[t] if l == 0 else fire(np.asarray(h_traj[l - 1][t], dtype=np.float64), theta)
            dW[l] += conv3x3_weight_grad(g_h, s_in)
            G = conv3x3_transpose(g_h, ws[l])
            g_v[l] = leak * g_h
        dx[t] = G
    return {"dW": dW, "dx": dx, "dv_init": g_v}


# ----------------------------------------------------------------------------
# teacher-forced one-step reference
# ----------------------------------------------------------------------------

def teacher_forced(x, weights, theta, leak, h_dev, v_init=None):
    """One-step references driven by a device trajectory.

    h_dev  list over layers of [T, C_l, H, W] charged potentials produced by
           the device (any precision).  The device's spikes and post-reset
           potentials are derived from them with Eq. (3) and the reset, and
           each step is recomputed in FP64 from the device's own previous
           state and input spikes.  Returns the list of FP64 h references.
    """
    x = np.asarray(x, dtype=np.float64)
    T, _, H, W = x.shape
    ws = [np.asarray(w, dtype=np.float64) for w in weights]
    refs = []
    for l, w in enumerate(ws):
        hd = np.asarray(h_dev[l], dtype=np.float64)
        sd = fire(hd, theta)
        vd = hd - theta * sd
        ref = np.zeros_like(hd)
        for t in range(T):
            if t == 0:
                vprev = np.zeros_like(hd[0]) if v_init is None else np.asarray(v_init[l], dtype=np.float64)
            else:
                vprev = vd[t - 1]
            s_in = x[t] if l == 0 else fire(np.asarray(h_dev[l - 1][t], dtype=np.float64), theta)
            ref[t] = leak * vprev + conv3x3(s_in, w)
        refs.append(ref)
    return refs


def spike_margin(h_ref: np.ndarray, theta: float) -> np.ndarray:
    """Distance of a reference potential to the nearer of the two thresholds."""
    return np.minimum(np.abs(h_ref - theta), np.abs(h_ref + theta))
