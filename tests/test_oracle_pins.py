"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: they compare it with library
routines (torch conv2d / conv_transpose2d / autograd, scipy lfilter,
wasserstein_distance, quad), closed forms derived from Eq. (2)-(4) and
(7)-(8), worked examples under tests/golden/, brute force, invariants and
finite differences.
"""

import itertools
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.signal
import scipy.stats
import torch
import torch.nn.functional as F

from oracle import emd, evsnet

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(1234)


def rand_net(chs, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [rng.normal(0, scale * math.sqrt(2.0 / (ci * 9)), size=(co, ci, 3, 3))
            for ci, co in zip(chs[:-1], chs[1:])]


def identity_net():
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 1, 1] = 1.0
    return [w]


# ---------------------------------------------------------------- convolution

def test_conv3x3_matches_torch_conv2d():
    s = RNG.normal(size=(3, 7, 9))
    w = RNG.normal(size=(5, 3, 3, 3))
    ref = F.conv2d(torch.from_numpy(s)[None], torch.from_numpy(w), padding=1)[0].numpy()
    np.testing.assert_allclose(evsnet.conv3x3(s, w), ref, rtol=1e-13, atol=1e-13)


def test_conv3x3_adjoints_match_torch_autograd():
    s = torch.from_numpy(RNG.normal(size=(1, 4, 6, 5))).requires_grad_(True)
    w = torch.from_numpy(RNG.normal(size=(3, 4, 3, 3))).requires_grad_(True)
    g = RNG.normal(size=(3, 6, 5))
    u = F.conv2d(s, w, padding=1)
    (u[0] * torch.from_numpy(g)).sum().backward()
    np.testing.assert_allclose(evsnet.conv3x3_transpose(g, w.detach().numpy()),
                               s.grad[0].numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(evsnet.conv3x3_weight_grad(g, s.detach()[0].numpy()),
                               w.grad.numpy(), rtol=1e-12, atol=1e-12)
    ref_t = F.conv_transpose2d(torch.from_numpy(g)[None], w.detach(), padding=1)[0].numpy()
    np.testing.assert_allclose(evsnet.conv3x3_transpose(g, w.detach().numpy()), ref_t,
                               rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- golden files

def _golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([p.strip() for p in line.split(";")])
    return rows


def _floats(s):
    return np.array([float(v) for v in s.split(",")])


@pytest.mark.parametrize("row", _golden("bilif_examples.txt"))
def test_bilif_golden_examples(row):
    kind, theta, beta, inp, expected = row
    inp = _floats(inp)
    x = inp.reshape(-1, 1, 1, 1)
    out = evsnet.forward(x, identity_net(), float(theta), float(beta))
    if kind == "spikes":
        np.testing.assert_array_equal(out["s"].ravel(), _floats(expected))
    else:
        np.testing.assert_allclose(out["h"][0].ravel(), _floats(expected), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("row", _golden("emd_examples.txt"))
def test_emd_golden_examples(row):
    T, S, E, lf, lb = row
    S = _floats(S)
    E = _floats(E)
    assert len(S) == int(T)
    assert emd.emd_forward_dir(S, E) == pytest.approx(float(lf), abs=1e-14)
    assert emd.emd_bidir(S, E) == pytest.approx(float(lb), abs=1e-14)


# ---------------------------------------------------------------- BiLIF pins

def test_p1_zero_input_no_spikes():
    out = evsnet.forward(np.zeros((6, 3, 5, 7)), rand_net((3, 4, 2), 0), 0.5, 0.9)
    assert not out["s"].any()
    assert all(not v.any() for v in out["v"])
    assert all(not h.any() for h in out["h"])


def test_p2_oddness_flips_polarity_exactly():
    x = RNG.normal(size=(8, 3, 6, 6)) * 2.0
    ws = rand_net((3, 4, 4, 2), 1)
    a = evsnet.forward(x, ws, 0.5, 0.9)
    b = evsnet.forward(-x, ws, 0.5, 0.9)
    np.testing.assert_array_equal(b["s"], -a["s"])
    for ha, hb in zip(a["h"], b["h"]):
        np.testing.assert_array_equal(hb, -ha)
    assert np.abs(a["s"]).sum() > 0


def test_p3_leak_closed_form():
    beta, u0 = 0.9, 0.3
    x = np.zeros((20, 1, 1, 1))
    x[0] = u0
    out = evsnet.forward(x, identity_net(), 0.5, beta)
    t = np.arange(20)
    np.testing.assert_allclose(out["h"][0].ravel(), u0 * beta ** t, rtol=1e-13)
    assert not out["s"].any()


@pytest.mark.parametrize("u,theta,beta", [(0.07, 0.5, 0.9), (0.25, 1.0, 0.8), (0.051, 0.5, 0.9)])
def test_p4_first_spike_time_constant_drive(u, theta, beta):
    tstar = math.ceil(math.log(1 - theta * (1 - beta) / u) / math.log(beta)) - 1
    x = np.full((tstar + 3, 1, 1, 1), u)
    s = evsnet.forward(x, identity_net(), theta, beta)["s"].ravel()
    assert s[:tstar].sum() == 0 and s[tstar] == 1


@pytest.mark.parametrize("n,eps", [(1, 0.2), (4, 0.05), (9, 0.3)])
def test_p5_saturation_train(n, eps):
    theta = 0.5
    x = np.zeros((n + 4, 1, 1, 1))
    x[0] = n * theta + eps
    out = evsnet.forward(x, identity_net(), theta, 1.0)
    s = out["s"].ravel()
    np.testing.assert_array_equal(s, np.r_[np.ones(n), np.zeros(4)])
    assert out["v"][0].item() == pytest.approx(eps, abs=1e-12)


def test_p6_charge_conservation_beta_one():
    x = RNG.normal(size=(12, 2, 5, 5))
    ws = rand_net((2, 3), 2, scale=2.0)
    out = evsnet.forward(x, ws, 0.5, 1.0)
    u = np.stack([F.conv2d(torch.from_numpy(x[t])[None], torch.from_numpy(ws[0]), padding=1)[0].numpy()
                  for t in range(12)])
    np.testing.assert_allclose(out["v"][0], u.sum(0) - 0.5 * out["s"].sum(0), atol=1e-12)
    assert np.abs(out["s"]).sum() > 10


def test_p7_no_leak_is_memoryless_ternarisation():
    x = RNG.normal(size=(5, 3, 6, 6))
    ws = rand_net((3, 2), 3)
    s = evsnet.forward(x, ws, 0.5, 0.0)["s"]
    for t in range(5):
        u = F.conv2d(torch.from_numpy(x[t])[None], torch.from_numpy(ws[0]), padding=1)[0].numpy()
        ref = (u >= 0.5).astype(float) - (u <= -0.5).astype(float)
        # beta = 0 still keeps the reset residue, which is multiplied by 0
        np.testing.assert_array_equal(s[t], ref)


def test_p8_no_fire_is_linear_leaky_filter():
    beta = 0.85
    x = RNG.normal(size=(10, 3, 6, 7))
    ws = rand_net((3, 4, 2), 4)
    out = evsnet.forward(x, ws, 1e30, beta)
    u = np.stack([F.conv2d(torch.from_numpy(x[t])[None], torch.from_numpy(ws[0]), padding=1)[0].numpy()
                  for t in range(10)])
    h = scipy.signal.lfilter([1.0], [1.0, -beta], u, axis=0)
    np.testing.assert_allclose(out["h"][0], h, rtol=1e-12, atol=1e-12)
    assert not out["h"][1].any()


def test_p9_chunking_state_carry_is_exact():
    x = RNG.normal(size=(13, 3, 6, 6)) * 2
    ws = rand_net((3, 4, 2), 5)
    full = evsnet.forward(x, ws, 0.5, 0.9)
    a = evsnet.forward(x[:5], ws, 0.5, 0.9)
    b = evsnet.forward(x[5:], ws, 0.5, 0.9, v_init=a["v"])
    np.testing.assert_array_equal(np.concatenate([a["s"], b["s"]]), full["s"])
    for l in range(2):
        np.testing.assert_array_equal(b["v"][l], full["v"][l])


def test_literal_unit_reset_reading_differs():
    """With theta != 1 the literal "-S" reset of Eq. (2) is a different model."""
    x = np.zeros((4, 1, 1, 1))
    x[0] = 1.6
    a = evsnet.forward(x, identity_net(), 0.5, 1.0)["s"].ravel()
    b = evsnet.forward(x, identity_net(), 0.5, 1.0, reset_unit=1.0)["s"].ravel()
    np.testing.assert_array_equal(a, [1, 1, 1, 0])
    np.testing.assert_array_equal(b, [1, 1, 0, 0])


# ---------------------------------------------------------------- surrogate

def test_p16_surrogate_integrates_to_two():
    for alpha, theta in [(4.0, 0.5), (2.0, 1.0), (10.0, 0.3)]:
        val, _ = scipy.integrate.quad(lambda h: float(evsnet.surrogate(np.array(h), theta, alpha)),
                                      -np.inf, np.inf, limit=200)
        assert val == pytest.approx(2.0, rel=1e-8)


def test_surrogate_is_derivative_of_relaxed_spike():
    h = np.linspace(-3, 3, 601)
    eps = 1e-6
    fd = (evsnet.relaxed_fire(h + eps, 0.5, 4.0) - evsnet.relaxed_fire(h - eps, 0.5, 4.0)) / (2 * eps)
    np.testing.assert_allclose(evsnet.surrogate(h, 0.5, 4.0), fd, rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------- BPTT

def _fd_check(mode, detach, chs=(2, 3, 2), T=4, H=5, W=5, seed=7, surr="sigmoid", alpha=4.0):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(T, chs[0], H, W))
    ws = rand_net(chs, seed, scale=1.5)
    v0 = [rng.normal(size=(c, H, W)) * 0.3 for c in chs[1:]]
    G = rng.normal(size=(T, chs[-1], H, W))
    theta, beta = 0.5, 0.9

    def loss(ws_, x_, v_):
        return float((evsnet.forward(x_, ws_, theta, beta, v_init=v_, mode=mode, alpha=alpha,
                                     surr=surr)["s"] * G).sum())

    g = evsnet.backward(x, ws, theta, beta, G, v_init=v0, mode=mode, detach_reset=detach, alpha=alpha,
                        surr=surr)
    eps = 1e-6
    errs = []
    for l in range(len(ws)):
        fd = np.zeros_like(ws[l])
        for idx in np.ndindex(ws[l].shape):
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += eps
            wm[l][idx] -= eps
            fd[idx] = (loss(wp, x, v0) - loss(wm, x, v0)) / (2 * eps)
        errs.append(np.abs(fd - g["dW"][l]).max() / np.abs(fd).max())
    for _ in range(12):
        idx = tuple(int(rng.integers(0, n)) for n in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (loss(ws, xp, v0) - loss(ws, xm, v0)) / (2 * eps)
        errs.append(abs(fd - g["dx"][idx]) / max(1e-3, abs(fd)))
    for l in range(len(ws)):
        idx = (0, 2, 2)
        vp = [v.copy() for v in v0]
        vm = [v.copy() for v in v0]
        vp[l][idx] += eps
        vm[l][idx] -= eps
        fd = (loss(ws, x, vp) - loss(ws, x, vm)) / (2 * eps)
        errs.append(abs(fd - g["dv_init"][l][idx]) / max(1e-3, abs(fd)))
    return max(errs)


def test_p11_bptt_matches_fd_of_relaxed_forward():
    assert _fd_check("relaxed", False) < 1e-6


# ---------------------------------------------------------------- arctangent surrogate (Sec. 3.3)

def test_atan_step_closed_forms():
    """sigma(0) = 1/2, sigma'(0) = alpha/2, sigma(z) + sigma(-z) = 1, limits 0 and 1,
    and sigma(z) = 3/4 where pi/2 alpha z = 1 (arctan 1 = pi/4)."""
    for alpha in (0.5, 2.0, 4.0):
        assert evsnet.step(np.array(0.0), alpha, "atan") == 0.5
        assert evsnet.step_slope(np.array(0.0), alpha, "atan") == pytest.approx(alpha / 2, rel=1e-15)
        z = np.linspace(-5, 5, 101)
        np.testing.assert_allclose(evsnet.step(z, alpha, "atan") + evsnet.step(-z, alpha, "atan"), 1.0,
                                   rtol=0, atol=1e-15)
        assert evsnet.step(np.array(2.0 / (np.pi * alpha)), alpha, "atan") == pytest.approx(0.75, rel=1e-14)
        assert evsnet.step(np.array(1e9), alpha, "atan") == pytest.approx(1.0, abs=1e-8)
        assert evsnet.step(np.array(-1e9), alpha, "atan") == pytest.approx(0.0, abs=1e-8)


def test_atan_surrogate_is_derivative_of_relaxed_spike():
    h = np.linspace(-3, 3, 601)
    eps = 1e-6
    for alpha in (2.0, 4.0):
        fd = (evsnet.relaxed_fire(h + eps, 0.5, alpha, "atan") - evsnet.relaxed_fire(h - eps, 0.5, alpha, "atan")) / (2 * eps)
        np.testing.assert_allclose(evsnet.surrogate(h, 0.5, alpha, "atan"), fd, rtol=1e-7, atol=1e-9)
    # psi is even in h and peaks at the two thresholds
    np.testing.assert_allclose(evsnet.surrogate(h, 0.5, 2.0, "atan"), evsnet.surrogate(-h, 0.5, 2.0, "atan"), rtol=1e-15)
    psi = evsnet.surrogate(h, 0.5, 2.0, "atan")
    assert abs(abs(h[np.argmax(psi)]) - 0.5) < 0.011


def test_atan_bptt_matches_fd_of_relaxed_forward():
    assert _fd_check("relaxed", False, surr="atan", alpha=2.0) < 1e-6


def test_p12_detached_reset_bptt_matches_fd_of_hybrid_forward():
    assert _fd_check("hybrid", True) < 1e-6


def test_p12_reset_variants_differ():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4, 2, 5, 5))
    ws = rand_net((2, 3, 2), 3, scale=1.5)
    G = rng.normal(size=(4, 2, 5, 5))
    a = evsnet.backward(x, ws, 0.5, 0.9, G)["dW"][0]
    b = evsnet.backward(x, ws, 0.5, 0.9, G, detach_reset=True)["dW"][0]
    assert np.abs(a - b).max() > 1e-3


class _Spike(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, theta, alpha):
        ctx.save_for_backward(h)
        ctx.theta, ctx.alpha = theta, alpha
        return (h >= theta).double() - (h <= -theta).double()

    @staticmethod
    def backward(ctx, g):
        (h,) = ctx.saved_tensors
        sig = lambda z: torch.sigmoid(ctx.alpha * z)
        a, b = sig(h - ctx.theta), sig(-h - ctx.theta)
        psi = ctx.alpha * (a * (1 - a) + b * (1 - b))
        return g * psi, None, None


def test_p13_bptt_matches_torch_autograd_and_checkpoint_invariance():
    rng = np.random.default_rng(11)
    T, H, W, chs = 9, 6, 5, (3, 4, 4, 2)
    theta, beta = 0.5, 0.9
    x = rng.normal(size=(T, 3, H, W)) * 2
    ws = rand_net(chs, 11)
    G = rng.normal(size=(T, 2, H, W))
    xt = torch.from_numpy(x).requires_grad_(True)
    wt = [torch.from_numpy(w).requires_grad_(True) for w in ws]
    v = [torch.zeros(c, H, W, dtype=torch.float64) for c in chs[1:]]
    outs = []
    for t in range(T):
        s = xt[t]
        for l in range(3):
            h = beta * v[l] + F.conv2d(s[None], wt[l], padding=1)[0]
            s = _Spike.apply(h, theta, 4.0)
            v[l] = h - theta * s
        outs.append(s)
    (torch.stack(outs) * torch.from_numpy(G)).sum().backward()
    for k in (None, 1, 2, 4, 9):
        g = evsnet.backward(x, ws, theta, beta, G, ckpt_every=k)
        for l in range(3):
            np.testing.assert_allclose(g["dW"][l], wt[l].grad.numpy(), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(g["dx"], xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    g1 = evsnet.backward(x, ws, theta, beta, G, ckpt_every=4)
    g2 = evsnet.backward(x, ws, theta, beta, G, ckpt_every=None)
    for l in range(3):
        np.testing.assert_array_equal(g1["dW"][l], g2["dW"][l])
    # the backward along a given trajectory, fed the autograd run's own
    # charged potentials, gives autograd's gradients (an independent pin of
    # backward_along: no oracle forward is involved)
    ht = [torch.zeros(T, c, H, W, dtype=torch.float64) for c in chs[1:]]
    v = [torch.zeros(c, H, W, dtype=torch.float64) for c in chs[1:]]
    with torch.no_grad():
        for t in range(T):
            s = torch.from_numpy(x[t])
            for l in range(3):
                h = beta * v[l] + F.conv2d(s[None], torch.from_numpy(ws[l]), padding=1)[0]
                ht[l][t] = h
                s = (h >= theta).double() - (h <= -theta).double()
                v[l] = h - theta * s
    ga = evsnet.backward_along(x, ws, theta, beta, G, [h.numpy() for h in ht])
    for l in range(3):
        np.testing.assert_allclose(ga["dW"][l], wt[l].grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ga["dx"], xt.grad.numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("surr,detach", [("sigmoid", False), ("sigmoid", True), ("atan", False)])
def test_backward_along_own_trajectory_equals_bptt(surr, detach):
    """Fed the oracle's own hard-spike trajectory, the backward along a given
    trajectory is the same computation as the checkpointed BPTT: identical
    bits for the weight, input and initial-state gradients."""
    rng = np.random.default_rng(17)
    T, H, W, chs = 8, 7, 6, (3, 5, 4, 2)
    x = rng.normal(size=(T, 3, H, W)) * 2
    ws = rand_net(chs, 17)
    G = rng.normal(size=(T, 2, H, W))
    alpha = 4.0 if surr == "sigmoid" else 2.0
    out = evsnet.forward(x, ws, 0.5, 0.9)
    a = evsnet.backward_along(x, ws, 0.5, 0.9, G, out["h"], alpha=alpha, detach_reset=detach, surr=surr)
    b = evsnet.backward(x, ws, 0.5, 0.9, G, alpha=alpha, detach_reset=detach, surr=surr, ckpt_every=3)
    for l in range(3):
        np.testing.assert_array_equal(a["dW"][l], b["dW"][l])
        np.testing.assert_array_equal(a["dv_init"][l], b["dv_init"][l])
    np.testing.assert_array_equal(a["dx"], b["dx"])


def test_backward_along_follows_the_given_trajectory():
    """A trajectory whose spike differs from the FP64 forward at one neuron
    (as an FP32 device may produce at a near-threshold step) changes the
    gradients exactly as a forward that fired there would: the backward is
    computed along the given potentials, not along a recomputed forward."""
    rng = np.random.default_rng(23)
    T, H, W, chs = 6, 5, 5, (3, 4, 2)
    x = rng.normal(size=(T, 3, H, W)) * 2
    ws = rand_net(chs, 23)
    G = rng.normal(size=(T, 2, H, W))
    out = evsnet.forward(x, ws, 0.5, 0.9)
    h = [a.copy() for a in out["h"]]
    # find a silent hidden neuron and lift its potential onto the threshold
    t, c, y, xx = np.argwhere(np.abs(h[0]) < 0.5)[0]
    h[0][t, c, y, xx] = 0.5
    g = evsnet.backward_along(x, ws, 0.5, 0.9, G, h)
    ref = evsnet.backward_along(x, ws, 0.5, 0.9, G, out["h"])
    # the output layer's weight gradient sees the flipped input spike
    assert np.abs(g["dW"][1] - ref["dW"][1]).max() > 1e-6


# ---------------------------------------------------------------- EMD pins

def test_p14_emd_zero_on_identity_and_shift_and_lone_event():
    T = 11
    S = RNG.integers(0, 3, size=(T, 4))
    assert not emd.emd_bidir(S, S).any()
    for t0 in range(T):
        for d in range(T - t0):
            a = np.zeros(T); a[t0 + d] = 1
            b = np.zeros(T); b[t0] = 1
            assert emd.emd_bidir(a, b) == pytest.approx(d / T, abs=1e-15)
    for t in range(T):
        a = np.zeros(T); a[t] = 1
        assert emd.emd_bidir(a, np.zeros(T)) == pytest.approx((T + 1) / (2 * T), abs=1e-15)
        assert emd.emd_forward_dir(a, np.zeros(T)) == pytest.approx((T - t) / T, abs=1e-15)


def test_p14_emd_equals_scipy_wasserstein_for_equal_counts():
    for _ in range(50):
        T = int(RNG.integers(3, 20))
        S = RNG.integers(0, 4, size=T).astype(float)
        E = RNG.integers(0, 4, size=T).astype(float)
        if S.sum() == 0 or E.sum() == 0:
            continue
        # rescale E's unit masses so both carry the same number of events
        n = int(S.sum())
        Eint = np.zeros(T)
        pos = np.repeat(np.arange(T), E.astype(int))
        for p in RNG.choice(pos, size=n, replace=True):
            Eint[p] += 1
        w1 = scipy.stats.wasserstein_distance(np.arange(T), np.arange(T), S, Eint)
        assert emd.emd_forward_dir(S, Eint) == pytest.approx(n * w1 / T, rel=1e-10, abs=1e-12)
        assert emd.emd_forward_dir(S[::-1], Eint[::-1]) == pytest.approx(n * w1 / T, rel=1e-10, abs=1e-12)


def test_p14_emd_brute_force_matching():
    """Eq. (7) equals the cheapest matching of unit events, for all small cases."""
    for T in range(1, 6):
        for S in itertools.product(range(3), repeat=T):
            ps = np.repeat(np.arange(T), S)
            n = len(ps)
            if n == 0 or n > 4:
                continue
            for E in itertools.product(range(3), repeat=T):
                if sum(E) != n:
                    continue
                pe = np.repeat(np.arange(T), E)
                best = min(sum(abs(a - b) for a, b in zip(ps, perm))
                           for perm in itertools.permutations(pe))
                assert emd.emd_forward_dir(np.array(S, float), np.array(E, float)) * T == pytest.approx(best)
                assert emd.emd_bidir(np.array(S, float), np.array(E, float)) * T == pytest.approx(best)


def test_p14_emd_ternary_sequences_brute_force():
    """Signed spikes: Eq. (7) on every ternary S against every small E (T <= 5)
    equals the L1 mass of its prefix-sum difference, computed by direct loops."""
    for T in range(1, 6):
        for S in itertools.product((-1, 0, 1), repeat=T):
            for E in itertools.product((0, 1), repeat=T):
                tot = 0.0
                for i in range(T):
                    tot += abs(sum(S[:i + 1]) - sum(E[:i + 1]))
                rev = 0.0
                for i in range(T):
                    rev += abs(sum(S[i:]) - sum(E[i:]))
                want = 0.5 * (tot + rev) / T
                assert emd.emd_bidir(np.array(S, float), np.array(E, float)) == pytest.approx(want, abs=1e-14)


def test_emd_grad_matches_fd_on_continuous_spikes():
    T = 9
    S = RNG.normal(size=(T, 2, 3, 3))
    Eon = RNG.integers(0, 2, size=(T, 3, 3)).astype(float)
    Eoff = RNG.integers(0, 2, size=(T, 3, 3)).astype(float)
    for lam in (0.0, 0.3):
        _, g = emd.loss_and_grad(S, Eon, Eoff, lam)
        eps = 1e-7
        for idx in np.ndindex(S.shape):
            Sp, Sm = S.copy(), S.copy()
            Sp[idx] += eps
            Sm[idx] -= eps
            fd = (emd.loss_and_grad(Sp, Eon, Eoff, lam)[0] - emd.loss_and_grad(Sm, Eon, Eoff, lam)[0]) / (2 * eps)
            assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_emd_polarity_split_single_channel():
    """Eq. (9) for a bipolar channel: ON part scored against E_on, OFF part
    (magnitude) against E_off; equivalently the two-channel form on the split."""
    T = 10
    s = RNG.integers(-1, 2, size=(T, 1, 4, 4)).astype(float)
    Eon = RNG.integers(0, 2, size=(T, 4, 4)).astype(float)
    Eoff = RNG.integers(0, 2, size=(T, 4, 4)).astype(float)
    l1, _ = emd.loss_and_grad(s, Eon, Eoff)
    two = np.concatenate([np.maximum(s, 0), np.maximum(-s, 0)], axis=1)
    l2, _ = emd.loss_and_grad(two, Eon, Eoff)
    assert l1 == pytest.approx(l2, abs=1e-12)


def test_emd_count_term():
    T = 6
    S = np.zeros((T, 2, 1, 1)); S[1, 0] = 1; S[3, 1] = -1; S[4, 1] = 1
    Eon = np.zeros((T, 1, 1)); Eoff = np.zeros((T, 1, 1)); Eon[2] = 1
    l0, _ = emd.loss_and_grad(S, Eon, Eoff, 0.0)
    l1, _ = emd.loss_and_grad(S, Eon, Eoff, 2.0)
    # three spikes against one target event: |3 - 1| = 2, weighted by 2
    assert l1 - l0 == pytest.approx(4.0)


# ---------------------------------------------------------------- teacher forcing

def test_teacher_forced_reproduces_exact_trajectory_and_flags_errors():
    rng = np.random.default_rng(21)
    x = rng.normal(size=(7, 3, 6, 6)) * 2
    ws = rand_net((3, 4, 2), 21)
    out = evsnet.forward(x, ws, 0.5, 0.9)
    refs = evsnet.teacher_forced(x, ws, 0.5, 0.9, out["h"])
    for r, h in zip(refs, out["h"]):
        np.testing.assert_allclose(r, h, rtol=1e-13, atol=1e-13)
    # a perturbed step (planted on the CPU) is caught at that step only
    bad = [h.copy() for h in out["h"]]
    bad[1][3, 0, 2, 2] += 1e-3
    refs = evsnet.teacher_forced(x, ws, 0.5, 0.9, bad)
    err = np.abs(refs[1] - bad[1])
    assert err[3, 0, 2, 2] == pytest.approx(1e-3, rel=1e-6)


def test_bf16_round_matches_torch():
    vals = np.concatenate([RNG.normal(size=5000).astype(np.float32) * 10,
                           np.array([1.0, -1.0, 0.0, 1.00390625, 1.01171875, 3.0e38, 1e-40], np.float32)])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(evsnet.bf16_round(vals), ref)


# ---------------------------------------------------------------- Eq. (1) input and contrast-crossing targets

from oracle import prologue  # noqa: E402


def test_luminance_weights_and_gray():
    """Rec. 709 luma weights (Eq. 1) sum to 1: a gray pixel keeps its value;
    each primary alone gives its own weight."""
    img = np.broadcast_to(np.linspace(0, 2, 7)[:, None], (7, 3))
    rgb = np.stack([img] * 3)                                                    # [3, 7, 3]
    np.testing.assert_allclose(prologue.luminance(rgb, 1.0), img, rtol=1e-15)
    for c, w in enumerate(prologue.LUMA):
        e = np.zeros((3, 1, 1))
        e[c] = 1.0
        assert prologue.luminance(e, 255.0)[0, 0] == pytest.approx(255.0 * w, rel=1e-15)


def test_linlog_branches_meet_at_the_knee_and_increase():
    for knee in (5.0, 20.0, 100.0):
        assert prologue.linlog(np.array(knee), knee) == pytest.approx(np.log(knee), rel=1e-15)
        assert prologue.linlog(np.array(knee * (1 - 1e-12)), knee) == pytest.approx(np.log(knee), rel=1e-10)
        L = np.linspace(0, 5 * knee, 2001)
        assert np.all(np.diff(prologue.linlog(L, knee)) > 0)
        assert prologue.linlog(np.array(0.0), knee) == 0.0
    assert prologue.linlog(np.array(np.e ** 4), 20.0) == pytest.approx(4.0, rel=1e-15)
    assert prologue.linlog(np.array(10.0), 20.0) == pytest.approx(np.log(20.0) / 2, rel=1e-15)


def test_logdiff_constant_and_step():
    rng = np.random.default_rng(0)
    frame = rng.uniform(0.01, 1.0, size=(3, 6, 7))
    X = prologue.logdiff(np.stack([frame] * 5))
    assert X.shape == (4, 1, 6, 7) and np.all(X == 0)
    # gray frames above the knee: X = ln(b / a)
    a, b = 0.3, 0.7
    fr = np.stack([np.full((3, 2, 2), a), np.full((3, 2, 2), b)])
    np.testing.assert_allclose(prologue.logdiff(fr), np.log(b / a), rtol=1e-14)
    # below the knee the step is linear: (ln 20 / 20) * 255 * (b - a)
    a, b = 0.01, 0.02
    fr = np.stack([np.full((3, 2, 2), a), np.full((3, 2, 2), b)])
    np.testing.assert_allclose(prologue.logdiff(fr), np.log(20.0) / 20.0 * 255.0 * (b - a), rtol=1e-13)


def _gray_from_log(l):
    """Gray frames whose lin-log luminance (scale 255, knee 20) is l (> ln 20)."""
    v = np.exp(l) / 255.0
    return np.broadcast_to(v[:, None, ...], (v.shape[0], 3) + v.shape[1:]).copy()


def test_contrast_events_log_ramp_closed_form():
    """A log ramp of delta per frame emits floor(t delta / C) ON events up to frame t."""
    T, delta, C = 60, 0.0713, 0.2
    l = 8.0 + delta * np.arange(T)                   # stays above ln(knee) both ways
    E = prologue.contrast_events(_gray_from_log(l[:, None, None] * np.ones((1, 2, 3))), C)
    cum = np.cumsum(E[:, 0, 0, 0].astype(int))
    np.testing.assert_array_equal(cum, np.floor(np.arange(T) * delta / C + 1e-12).astype(int))
    assert np.all(E[:, 1] == 0)
    # the mirrored ramp emits the same counts as OFF events
    E2 = prologue.contrast_events(_gray_from_log((2 * l[0] - l)[:, None, None] * np.ones((1, 2, 3))), C)
    np.testing.assert_array_equal(E2[:, 1], E[:, 0])
    assert np.all(E2[:, 0] == 0)


def test_contrast_events_step_constant_and_balance():
    C = 0.2
    l = np.full(8, np.log(40.0))
    l[3:] += 3.3 * C
    E = prologue.contrast_events(_gray_from_log(l[:, None, None] * np.ones((1, 1, 1))), C)
    np.testing.assert_array_equal(E[:, 0, 0, 0], [0, 0, 0, 3, 0, 0, 0, 0])
    # constant frames: nothing; random clips: the events account for the log change within C
    rng = np.random.default_rng(5)
    fr = rng.uniform(0.05, 1.0, size=(12, 3, 5, 4))
    E = prologue.contrast_events(fr, C).astype(np.float64)
    lg = prologue.linlog(prologue.luminance(fr))
    resid = lg[-1] - lg[0] - C * (E[:, 0] - E[:, 1]).sum(axis=0)
    assert np.all(np.abs(resid) < C + 1e-12)
    assert np.all(prologue.contrast_events(np.stack([fr[0]] * 6), C) == 0)


# ---------------------------------------------------------------- temporal EvSNet (Sec. 3.3, Eq. 5-6)

def test_tnet_conv1d_matches_torch():
    from oracle import tnet
    rng = np.random.default_rng(1)
    h = rng.normal(size=(3, 5, 19))
    w = rng.normal(size=(4, 5, 7))
    b = rng.normal(size=4)
    ref = torch.nn.functional.conv1d(torch.from_numpy(h), torch.from_numpy(w), torch.from_numpy(b), padding=3)
    np.testing.assert_allclose(tnet.conv1d(h, w, b), ref.numpy(), rtol=1e-13, atol=1e-13)


def test_tnet_receptive_field_is_43_frames():
    """With positive input and weights every ReLU passes its argument, the
    net is a cascade of seven kernel-7 convolutions, and a change of X at
    frame t0 moves u exactly on t0-21 .. t0+21 (Sec. 4: W = 43)."""
    from oracle import tnet
    p = tnet.init_params(C=4, seed=3)
    rng = np.random.default_rng(4)
    p["w0"] = np.abs(p["w0"]) + 0.01
    for k in range(1, 7):
        p["w"][k] = np.abs(p["w"][k]) + 0.01
        p["b"][k] = np.abs(p["b"][k])
    p["b0"] = np.abs(p["b0"])
    p["wp"] = np.abs(p["wp"]) + 0.01
    x = rng.uniform(0.1, 1.0, size=(1, 120))
    t0 = 60
    x2 = x.copy()
    x2[0, t0] += 0.5
    du = tnet.encode(x2, p)[0] - tnet.encode(x, p)[0]
    changed = np.nonzero(np.abs(du[0]) > 0)[0]
    assert changed.min() == t0 - 21 and changed.max() == t0 + 21
    assert len(changed) == 43


def test_tnet_inner_convs_zero_reduce_to_one_conv():
    """Zero residual branches: h_i = ReLU(h_{i-1}) = h_{i-1}, so u is the
    point-wise projection of ReLU(conv_0 X), computed here with scipy."""
    import scipy.signal
    from oracle import tnet
    C = 5
    p = tnet.init_params(C=C, seed=5)
    for k in range(1, 7):
        p["w"][k] = np.zeros_like(p["w"][k])
        p["b"][k] = np.zeros_like(p["b"][k])
    x = np.random.default_rng(6).normal(size=(2, 40))
    u, _ = tnet.encode(x, p)
    for n in range(2):
        h0 = np.stack([np.maximum(scipy.signal.correlate(x[n], p["w0"][c, 0], mode="same") + p["b0"][c], 0.0)
                       for c in range(C)])
        np.testing.assert_allclose(u[n], p["wp"] @ h0 + p["bp"], rtol=1e-12, atol=1e-12)
    # zero input, zero biases: nothing fires
    for k in range(1, 7):
        p["b"][k][:] = 0.0
    p["b0"][:] = 0.0
    p["bp"] = 0.0
    out = tnet.forward(np.zeros((3, 30)), p, 0.5, 0.9)
    assert np.all(out["u"] == 0) and np.all(out["s"] == 0)


def test_tnet_centred_padding_time_reversal():
    """With symmetric kernels, centred zero padding makes the encoder commute
    with reversing time (a causal padding would not)."""
    from oracle import tnet
    p = tnet.init_params(C=4, seed=7)
    sym = lambda w: 0.5 * (w + w[..., ::-1])
    p["w0"] = sym(p["w0"])
    for k in range(1, 7):
        p["w"][k] = sym(p["w"][k])
    x = np.random.default_rng(8).normal(size=(3, 50))
    u = tnet.encode(x, p)[0]
    ur = tnet.encode(x[:, ::-1].copy(), p)[0]
    np.testing.assert_allclose(ur[:, ::-1], u, rtol=1e-12, atol=1e-12)
    # and a non-symmetric kernel breaks it
    p["w0"][:, 0, 0] += 0.3
    ur = tnet.encode(x[:, ::-1].copy(), p)[0]
    assert np.abs(ur[:, ::-1] - tnet.encode(x, p)[0]).max() > 1e-3


def test_tnet_delta_net_is_bilif_of_relu_input():
    """conv_0 a centred delta on channel 0, zero residual branches, point-wise
    weight e_0: u = ReLU(X), and the spikes equal the (separately pinned)
    conv3x3 forward of a one-channel centre-tap identity net on ReLU(X)."""
    from oracle import tnet
    C = 3
    p = tnet.init_params(C=C, seed=9)
    p["w0"] = np.zeros((C, 1, 7))
    p["w0"][0, 0, 3] = 1.0
    p["b0"][:] = 0.0
    for k in range(1, 7):
        p["w"][k] = np.zeros_like(p["w"][k])
        p["b"][k][:] = 0.0
    p["wp"] = np.zeros(C)
    p["wp"][0] = 1.0
    p["bp"] = 0.0
    x = np.random.default_rng(10).normal(0.2, 0.6, size=(4, 60))
    out = tnet.forward(x, p, 0.5, 0.9)
    np.testing.assert_array_equal(out["u"], np.maximum(x, 0.0))
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 1, 1] = 1.0
    ref = evsnet.forward(np.maximum(x, 0.0).T[:, None, None, :], [w], 0.5, 0.9)
    np.testing.assert_array_equal(out["s"], ref["s"][:, 0, 0, :].T)


def test_tnet_quant_rounds_through_float32_to_bf16():
    """The BF16 mirror rounds input, weights and stored activations exactly
    as torch's float32 -> bfloat16 conversion does."""
    from oracle import tnet
    p = tnet.init_params(C=3, seed=11)
    x = np.random.default_rng(12).normal(size=(2, 20))
    u, layers = tnet.encode(x, p, quant=True)
    for a in layers:
        t = torch.from_numpy(a.astype(np.float32))
        assert np.array_equal(a, t.to(torch.bfloat16).to(torch.float64).numpy())


def _tnet_golden():
    rows = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "tnet_residual_examples.txt")
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = (s.strip() for s in line.split(";"))
        rows[key] = [float(v) for v in (val.split() if key == "weights" else val.split(","))]
    return rows


def test_tnet_residual_blocks_golden_example():
    """Hand-derived one-channel worked example (tests/golden): delta kernels,
    some negative, chosen so that the ReLU inside each residual block and the
    ReLU after each residual add both clip on some frame.  Dropping either
    ReLU of any block, or applying the outer one before the residual add,
    changes u on at least one frame."""
    from oracle import tnet
    g = _tnet_golden()
    wv = g["weights"]
    delta = lambda w: np.array([0, 0, 0, w, 0, 0, 0], np.float64).reshape(1, 1, 7)
    p = {"w0": delta(wv[0]), "b0": np.array([wv[1]]),
         "w": [None] + [delta(wv[2 * k]) for k in range(1, 7)],
         "b": [None] + [np.array([wv[2 * k + 1]]) for k in range(1, 7)],
         "wp": np.array([wv[14]]), "bp": wv[15]}
    x = np.array(g["x"])[None, :]
    u, layers = tnet.encode(x, p)
    for name, a in zip(("h0", "a1", "h1", "a2", "h2", "a3", "h3"), layers):
        np.testing.assert_array_equal(a[0, 0], g[name], err_msg=name)
    np.testing.assert_array_equal(u[0], g["u"])
