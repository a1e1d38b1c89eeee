"""GPU parity of the BPTT backward (through the C ABI and torch.autograd).

* Hard spikes: weight/input/initial-state gradients against the FP64 oracle
  BPTT on trajectories whose spikes match the oracle's exactly (the test
  checks that first), rel. error <= 1e-4 (FP32 nets) or the BF16 gradient
  gate of tests/_helpers.py (BF16 nets: bf16 adjoints between kernels).
* Relaxed spikes (smooth, FP32): against the oracle's relaxed BPTT and
  against central finite differences of the GPU's own relaxed forward on an
  8x8x4 crop, rel. error <= 1e-2.
* Checkpointing: k = 4 equals k = T to FP32 rounding; repeated calls are
  bitwise identical (fixed-order reductions).
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from oracle import evsnet, emd  # noqa: E402
from tests._helpers import f32, grad_tol, make_inputs, split_layers  # noqa: E402

THETA, LEAK = f32(0.5), f32(0.9)


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-12))


SURR_ALPHA = {"sigmoid": 4.0, "atan": 2.0}


def _setup(evs, channels, prec, T, H, W, N=1, seed=0, scale=1.0, relaxed=False, detach=False, surr="sigmoid"):
    x, ws = make_inputs(channels, T, H, W, N=N, seed=seed, scale=scale)
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec, relaxed=relaxed, detach_reset=detach,
                  surrogate=surr, surr_alpha=SURR_ALPHA[surr])
    wt = [torch.from_numpy(w).cuda() for w in ws]
    packed = evs.pack_weights(net, wt)
    return x, ws, net, packed


@pytest.mark.parametrize("channels,prec,detach,surr", [((3, 8, 2), "fp32", False, "sigmoid"),
                                                       ((3, 16, 16, 2), "fp32", False, "sigmoid"),
                                                       ((3, 16, 16, 2), "fp32", True, "sigmoid"),
                                                       ((3, 16, 16, 2), "fp32", False, "atan"),
                                                       ((3, 32, 2), "bf16", False, "sigmoid"),
                                                       ((3, 32, 2), "fp32", False, "sigmoid"),
                                                       ((3, 16, 16, 2), "bf16", False, "sigmoid"),
                                                       # widths that are not multiples of 4; two
                                                       # 32-wide hidden layers
                                                       ((3, 10, 10, 2), "fp32", False, "sigmoid"),
                                                       ((3, 32, 32, 2), "bf16", False, "sigmoid"),
                                                       ((1, 1), "fp32", False, "sigmoid")])
@pytest.mark.parametrize("k", [4, 100])
def test_backward_matches_oracle(evs, channels, prec, detach, surr, k):
    T, H, W, N = 9, 21, 27, 2
    print(f"case {channels} {prec} detach={detach} surrogate={surr} k={k}", flush=True)
    x, ws, net, packed = _setup(evs, channels, prec, T, H, W, N=N, seed=3, detach=detach, surr=surr)
    xg = x.cuda()
    out = evs.forward(net, packed, xg, trace=True, ckpt_every=k)
    rng = np.random.default_rng(1)
    G = rng.normal(size=(N, T, channels[-1], H, W)).astype(np.float32)
    gws, dx, dv = evs.backward(net, packed, xg, out["ckpt"], k, torch.from_numpy(G).cuda(), want_dx=True,
                               want_dv=True)
    torch.cuda.synchronize()
    if prec == "bf16":
        ows = [evsnet.bf16_round(w) for w in ws]
        xo = evsnet.bf16_round(x.numpy())
    else:
        ows = [w.astype(np.float64) for w in ws]
        xo = x.numpy().astype(np.float64)
    h = out["h"].cpu().numpy()
    dW_ref = [np.zeros_like(w) for w in ows]
    for n in range(N):
        ref = evsnet.forward(xo[n], ows, THETA, LEAK)
        # same trajectory: every layer's spikes agree with the oracle's
        for hl, sr in zip(split_layers(h[n], channels), ref["spk"]):
            assert np.array_equal(evsnet.fire(hl, THETA), sr), "trajectory diverged; reseed"
        g = evsnet.backward(xo[n], ows, THETA, LEAK, G[n], detach_reset=detach, alpha=SURR_ALPHA[surr], surr=surr)
        for l in range(len(ws)):
            dW_ref[l] += g["dW"][l]
        tol = grad_tol(prec)
        rx = _rel(dx[n].cpu().numpy(), g["dx"])
        print(f"  clip {n} dx rel err {rx:.2e}", flush=True)
        assert rx < tol
        dvl = split_layers(dv[n].cpu().numpy()[None], channels)
        for a, b in zip(dvl, g["dv_init"]):
            assert _rel(a[0], b) < tol
    for l in range(len(ws)):
        r = _rel(gws[l].cpu().numpy(), dW_ref[l])
        print(f"  layer {l + 1} dW rel err {r:.2e}", flush=True)
        assert r < grad_tol(prec)


@pytest.mark.parametrize("channels,prec", [((3, 16, 16, 2), "fp32"), ((3, 32, 2), "bf16")])
@pytest.mark.parametrize("N,T,H,W,k", [(1, 1, 1, 1, 1), (2, 3, 2, 37, 2), (1, 5, 19, 1, 5)])
def test_backward_degenerate_shapes(evs, channels, prec, N, T, H, W, k):
    """One pixel and one frame, two rows across several gradient tiles, one
    column: gradients along the device's trajectory against the oracle."""
    print(f"case backward {channels} {prec} N={N} T={T} H={H} W={W} k={k}", flush=True)
    x, ws, net, packed = _setup(evs, channels, prec, T, H, W, N=N, seed=9)
    xg = x.cuda()
    out = evs.forward(net, packed, xg, trace=True, ckpt_every=k)
    G = np.random.default_rng(2).normal(size=(N, T, channels[-1], H, W)).astype(np.float32)
    gws, dx, dv = evs.backward(net, packed, xg, out["ckpt"], k, torch.from_numpy(G).cuda(), want_dx=True,
                               want_dv=True)
    torch.cuda.synchronize()
    if prec == "bf16":
        ows = [evsnet.bf16_round(w) for w in ws]
        xo = evsnet.bf16_round(x.numpy())
    else:
        ows = [w.astype(np.float64) for w in ws]
        xo = x.numpy().astype(np.float64)
    h = out["h"].cpu().numpy()
    dW_ref = [np.zeros_like(w) for w in ows]
    tol = grad_tol(prec)
    for n in range(N):
        g = evsnet.backward_along(xo[n], ows, THETA, LEAK, G[n], split_layers(h[n], channels))
        for l in range(len(ws)):
            dW_ref[l] += g["dW"][l]
        assert _rel(dx[n].cpu().numpy(), g["dx"]) < tol
        dvl = split_layers(dv[n].cpu().numpy()[None], channels)
        for a, b in zip(dvl, g["dv_init"]):
            assert _rel(a[0], b) < tol
    for l in range(len(ws)):
        r = _rel(gws[l].cpu().numpy(), dW_ref[l])
        print(f"  layer {l + 1} dW rel err {r:.2e}", flush=True)
        assert r < tol


def test_checkpoint_interval_and_determinism(evs):
    channels = (3, 16, 16, 2)
    T, H, W = 12, 19, 23
    x, ws, net, packed = _setup(evs, channels, "fp32", T, H, W, seed=5)
    xg = x.cuda()
    G = torch.from_numpy(np.random.default_rng(2).normal(size=(1, T, 2, H, W)).astype(np.float32)).cuda()
    res = {}
    for k in (1, 4, 5, 12):
        out = evs.forward(net, packed, xg, ckpt_every=k)
        res[k] = evs.backward(net, packed, xg, out["ckpt"], k, G, want_dx=True)
    again = evs.backward(net, packed, xg, evs.forward(net, packed, xg, ckpt_every=4)["ckpt"], 4, G, want_dx=True)
    torch.cuda.synchronize()
    for a, b in zip(res[4][0], again[0]):
        assert torch.equal(a, b)
    assert torch.equal(res[4][1], again[1])
    for k in (1, 5, 12):
        for a, b in zip(res[k][0], res[4][0]):
            assert _rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-5
        assert _rel(res[k][1].cpu().numpy(), res[4][1].cpu().numpy()) < 1e-5


@pytest.mark.parametrize("channels,prec", [((3, 16, 16, 2), "fp32"), ((1, 12, 16, 2), "fp32"),
                                           ((3, 16, 16, 2), "bf16")])
def test_weight_gradients_do_not_depend_on_the_input_gradient(evs, channels, prec):
    """Without the input gradient the backward skips writing layer 1's
    adjoints (FP32 nets form the input layer's dW inside the layer-2
    conv-transpose): the weight gradients and the initial-state gradient
    equal, bit for bit, those of a call that also forms grad_x."""
    T, H, W, k = 10, 37, 29, 4
    x, ws, net, packed = _setup(evs, channels, prec, T, H, W, N=2, seed=8)
    xg = x.cuda()
    G = torch.from_numpy(np.random.default_rng(6).normal(size=(2, T, 2, H, W)).astype(np.float32)).cuda()
    out = evs.forward(net, packed, xg, ckpt_every=k)
    a = evs.backward(net, packed, xg, out["ckpt"], k, G, want_dx=True, want_dv=True)
    b = evs.backward(net, packed, xg, out["ckpt"], k, G, want_dv=True)
    torch.cuda.synchronize()
    assert b[1] is None
    for ga, gb in zip(a[0], b[0]):
        assert torch.equal(ga, gb)
    assert torch.equal(a[2], b[2])


@pytest.mark.parametrize("surr", ["sigmoid", "atan"])
def test_relaxed_backward_matches_oracle_and_finite_differences(evs, surr):
    """8x8x4 crop (8x8 pixels, 4 frames): GPU BPTT of the smooth forward
    against the oracle and against central differences of the GPU forward."""
    channels = (3, 16, 16, 2)
    T, H, W = 4, 8, 8
    x, ws, net, packed = _setup(evs, channels, "fp32", T, H, W, seed=9, relaxed=True, surr=surr)
    xg = x.cuda()
    G = np.random.default_rng(4).normal(size=(1, T, 2, H, W)).astype(np.float32)
    Gt = torch.from_numpy(G).cuda()
    out = evs.forward(net, packed, xg, s_fp32=True, ckpt_every=2)
    gws, dx, _ = evs.backward(net, packed, xg, out["ckpt"], 2, Gt, want_dx=True)
    torch.cuda.synchronize()
    ref = evsnet.backward(x[0].numpy(), ws, THETA, LEAK, G[0], mode="relaxed", alpha=SURR_ALPHA[surr], surr=surr)
    for l in range(3):
        assert _rel(gws[l].cpu().numpy(), ref["dW"][l]) < 1e-4
    assert _rel(dx[0].cpu().numpy(), ref["dx"]) < 1e-4

    def loss(wlist):
        p = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in wlist])
        o = evs.forward(net, p, xg, s_fp32=True)
        return float((o["s"].double() * Gt.double()).sum())

    rng = np.random.default_rng(0)
    eps = 2e-3
    errs = []
    for l in range(3):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, n)) for n in ws[l].shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += eps
            wm[l][idx] -= eps
            fd = (loss(wp) - loss(wm)) / (2 * eps)
            gd = float(gws[l].cpu().numpy()[idx])
            errs.append(abs(fd - gd) / max(1.0, abs(fd)))
    print(f"  relaxed FD max err {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-2


def test_autograd_training_step_matches_oracle(evs):
    """EvsFunction + EmdLossFunction: one training step's gradients."""
    from paper_2508_18071_amd import autograd as ag
    import synth
    channels = (3, 16, 16, 2)
    T, H, W = 8, 24, 24
    x, ws, net, packed = _setup(evs, channels, "fp32", T, H, W, seed=11)
    clean = synth.make_clip(synth.WORKLOADS["planes720"], T=T, H=H, W=W, y0=37, x0=51, clean=True)
    from oracle import prologue
    e = torch.from_numpy(prologue.contrast_events(clean.numpy().astype(np.float64)))
    wt = [torch.from_numpy(w).cuda().requires_grad_(True) for w in ws]
    xg = x.cuda()
    s = ag.evsnet(net, xg, wt, ckpt_every=4)
    loss = ag.emd_loss(s, e[None].cuda())
    loss.backward()
    torch.cuda.synchronize()
    ref = evsnet.forward(x[0].numpy(), ws, THETA, LEAK)
    assert np.array_equal(ref["s"], s[0].detach().cpu().numpy())
    l_ref, g_s = emd.loss_and_grad(ref["s"], e[:, 0].numpy(), e[:, 1].numpy())
    assert float(loss.detach()) == pytest.approx(l_ref, rel=1e-6)
    g = evsnet.backward(x[0].numpy(), ws, THETA, LEAK, g_s)
    for l in range(3):
        assert _rel(wt[l].grad.cpu().numpy(), g["dW"][l]) < 1e-4
