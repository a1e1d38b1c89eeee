"""FP64 oracle of the paper's temporal EvSNet -- test infrastructure only.

Sec. 3.3 ("Network architecture", Eq. 5-6): per pixel, the sequence X of
log-luminance differences passes through a 1-D convolutional encoder

    h0 = ReLU(conv_0(X))
    a_i = ReLU(conv_{2i-1}(h_{i-1})),   h_i = ReLU(h_{i-1} + conv_{2i}(a_i)),   i = 1..M

a point-wise convolution projects h_M to one value per frame, and a BiLIF
unit (Eq. 2-3) turns that sequence into spikes S in {-1, 0, 1}.  Sec. 4
fixes the kernel size 7 and M = 3 (seven kernel-7 convolutions, receptive
field 1 + 6 * 7 = 43 frames).

Readings (the paper leaves them open): every Conv1d is a cross-correlation
with "same" zero padding of 3 frames on both sides (centred, non-causal:
the renderer refers to neighbouring frames), each convolution has a bias per
output channel, the hidden width C is a parameter (16 by default), and one
output channel carries both polarities through the sign of the spike.

``quant=True`` mirrors the BF16 kernel: the network input, every weight and
every stored activation (h_i, a_i) is rounded to bfloat16 (through float32,
as the kernel rounds its FP32 sums); sums are exact here (FP64) and biases
stay unrounded.
"""

from __future__ import annotations

import numpy as np

from .evsnet import bf16_round, fire

KSIZE = 7
DEPTH = 3


def conv1d(h: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Cross-correlation with zero padding K//2: h [P][Cin][T], w [Cout][Cin][K], b [Cout] -> [P][Cout][T]."""
    h = np.asarray(h, np.float64)
    P, cin, T = h.shape
    cout, cin2, K = w.shape
    assert cin == cin2
    pad = K // 2
    hp = np.zeros((P, cin, T + 2 * pad))
    hp[:, :, pad:pad + T] = h
    out = np.broadcast_to(np.asarray(b, np.float64)[None, :, None], (P, cout, T)).copy()
    for k in range(K):
        out += np.einsum("oc,pct->pot", np.asarray(w[:, :, k], np.float64), hp[:, :, k:k + T])
    return out


def relu(a):
    return np.maximum(a, 0.0)


def init_params(C: int = 16, seed: int = 0, scale: float = 1.0):
    """He-style random parameters: dict w0 [C][1][7], b0 [C], w[k] [C][C][7] and
    b[k] [C] for k = 1..6, wp [C], bp (scalar)."""
    rng = np.random.default_rng(seed)
    p = {"w0": rng.normal(0, scale * np.sqrt(2.0 / KSIZE), (C, 1, KSIZE)),
         "b0": rng.normal(0, 0.05, C),
         "w": [None] + [rng.normal(0, scale * np.sqrt(1.0 / (C * KSIZE)), (C, C, KSIZE)) for _ in range(2 * DEPTH)],
         "b": [None] + [rng.normal(0, 0.05, C) for _ in range(2 * DEPTH)],
         "wp": rng.normal(0, np.sqrt(2.0 / C), C),
         "bp": float(rng.normal(0, 0.05))}
    return p


def flatten_params(p) -> np.ndarray:
    """The library's weight order: w0, b0, then (w_k, b_k) for k = 1..6, then wp, bp."""
    parts = [p["w0"].reshape(-1), p["b0"]]
    for k in range(1, 2 * DEPTH + 1):
        parts += [p["w"][k].reshape(-1), p["b"][k]]
    parts += [p["wp"], np.array([p["bp"]])]
    return np.concatenate([np.asarray(a, np.float64).reshape(-1) for a in parts])


def encode(x, p, quant: bool = False):
    """x [P][T] -> (u [P][T], layers): the point-wise projection u and the
    activations h0, a1, h1, a2, h2, a3, h3, each [P][C][T]."""
    q = bf16_round if quant else (lambda a: np.asarray(a, np.float64))
    h = q(relu(conv1d(q(x)[:, None, :], q(p["w0"]), p["b0"])))
    layers = [h]
    for i in range(1, DEPTH + 1):
        a = q(relu(conv1d(h, q(p["w"][2 * i - 1]), p["b"][2 * i - 1])))
        h = q(relu(h + conv1d(a, q(p["w"][2 * i]), p["b"][2 * i])))
        layers += [a, h]
    u = np.einsum("c,pct->pt", q(p["wp"]), h) + p["bp"]
    return u, layers


def bilif(u, theta: float, leak: float):
    """BiLIF over time (Eq. 2-3) driven by u [P][T]: returns spikes and the
    charged potentials h_t = leak v_{t-1} + u_t."""
    P, T = u.shape
    v = np.zeros(P)
    s = np.zeros((P, T))
    hs = np.zeros((P, T))
    for t in range(T):
        h = leak * v + u[:, t]
        hs[:, t] = h
        s[:, t] = fire(h, theta)
        v = h - theta * s[:, t]
    return s, hs


def forward(x, p, theta: float, leak: float, quant: bool = False):
    u, layers = encode(x, p, quant)
    s, hs = bilif(u, theta, leak)
    return {"s": s, "h": hs, "u": u, "layers": layers}
