"""The BPTT backward at the full training-step size (4 crops x 64 frames x
256x256 of the 720p textured-planes clip, net 3->16->16->2, FP32 and BF16,
checkpoints every 16 frames), in the launch configuration bench.py times.

The full-size run is held to the FP64 oracle's backward along the device's
own trajectory (test_train_size_backward_matches_oracle, about a minute of
host time per precision) and to properties that hold at any size:
* weight and input gradients are bitwise reproducible (fixed-order sums);
* they do not depend on the checkpoint interval (every 16 vs every 64
  frames: rel. 1e-5);
* for hard spikes the backward is linear in the incoming gradient:
  dW(G1 + 2 G2) = dW(G1) + 2 dW(G2) to rel. 1e-5 (FP32; BF16 nets round
  their adjoints to bf16 between kernels, which holds linearity to the BF16
  gradient gate);
* they are finite, and the input-layer gradient is not zero.
"""

import pytest
import torch

from tests._helpers import grad_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import synth
    wl = synth.WORKLOADS["train256"]
    src = synth.WORKLOADS["planes720"]
    xs = [synth.make_clip(src, device="cuda", t0=t0, T=wl.T, y0=y0, x0=x0, H=wl.H, W=wl.W)
          for (t0, y0, x0) in synth.train_crops(wl)]
    x = torch.stack(xs).contiguous()
    torch.cuda.synchronize()
    return wl, x


def _rel(a, b):
    return float((a - b).abs().max() / max(float(b.abs().max()), 1e-30))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_train_size_backward_properties(evs, batch, prec):
    wl, x = batch
    print(f"case train256 4x64x256x256 {prec}", flush=True)
    net = evs.Net(wl.channels, theta=wl.theta, leak=wl.leak, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in wl.weights()])
    g = torch.Generator(device="cuda").manual_seed(7)
    shape = (x.shape[0], x.shape[1], wl.channels[-1], x.shape[3], x.shape[4])
    G1 = torch.randn(shape, device="cuda", generator=g)
    G2 = torch.randn(shape, device="cuda", generator=g)

    def grads(G, k):
        o = evs.forward(net, packed, x, ckpt_every=k)
        gw, dx, _ = evs.backward(net, packed, x, o["ckpt"], k, G, want_dx=True)
        torch.cuda.synchronize()
        return gw, dx

    a_w, a_x = grads(G1, 16)
    b_w, b_x = grads(G1, 16)
    for l in range(len(a_w)):
        assert torch.equal(a_w[l], b_w[l]), f"layer {l + 1} dW not reproducible"
        assert torch.isfinite(a_w[l]).all()
    assert torch.equal(a_x, b_x)
    assert torch.isfinite(a_x).all() and float(a_x.abs().max()) > 0
    c_w, c_x = grads(G1, 64)
    for l in range(len(a_w)):
        r = _rel(c_w[l], a_w[l])
        print(f"  layer {l + 1} dW, checkpoints 64 vs 16: rel {r:.2e}", flush=True)
        assert r < 1e-5
    assert _rel(c_x, a_x) < 1e-5
    d_w, _ = grads(G2, 16)
    e_w, _ = grads(G1 + 2 * G2, 16)
    for l in range(len(a_w)):
        r = _rel(e_w[l], a_w[l] + 2 * d_w[l])
        print(f"  layer {l + 1} dW linearity in grad_s: rel {r:.2e}", flush=True)
        assert r < (1e-5 if prec == "fp32" else grad_tol(prec))


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_train_size_backward_matches_oracle(evs, batch, prec):
    """Oracle parity of the BPTT backward (Sec. 3.3 Eq. 4) at the training
    step's full size, in the launch configuration bench.py times (4 crops x
    64 frames x 256x256, checkpoints every 16 frames, so 4 segments and 256
    tiles per crop whose weight-gradient partials are reduced per layer).

    The oracle runs the backward along the device's own trajectory (the
    charged potentials of every layer from the forward's trace, which the
    segment recomputes reproduce bit for bit): a near-threshold step where an
    FP32 sum lands on the other side of a threshold than FP64 would then does
    not make the two gradients incomparable.  BF16 nets are held to the
    oracle with BF16-rounded x and W (the operands the forward multiplied).
    Gate: dW, dx and the initial-state gradient within 1e-4 relative (FP32)
    or the BF16 gradient gate (bf16 adjoints between kernels)."""
    import numpy as np
    from oracle import evsnet
    from tests._helpers import split_layers

    wl, x = batch
    N, T, _, H, W = x.shape
    k = 16
    print(f"case train256 oracle parity {N}x{T}x{H}x{W} {prec} k={k}", flush=True)
    ws = wl.weights()
    net = evs.Net(wl.channels, theta=wl.theta, leak=wl.leak, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    g = torch.Generator(device="cuda").manual_seed(11)
    G = torch.randn((N, T, wl.channels[-1], H, W), device="cuda", generator=g)
    o = evs.forward(net, packed, x, s_fp32=True, ckpt_every=k, trace=True)
    gw, dx, dv = evs.backward(net, packed, x, o["ckpt"], k, G, want_dx=True, want_dv=True)
    torch.cuda.synchronize()
    h = o["h"].cpu().numpy()
    del o
    xh = x.cpu().numpy()
    Gh = G.cpu().numpy()
    dxh, dvh = dx.cpu().numpy(), dv.cpu().numpy()
    theta, leak = float(np.float32(wl.theta)), float(np.float32(wl.leak))
    if prec == "bf16":
        ows = [evsnet.bf16_round(w) for w in ws]
    else:
        ows = [w.astype(np.float64) for w in ws]
    dW_ref = [np.zeros_like(w) for w in ows]
    for n in range(N):
        xo = evsnet.bf16_round(xh[n]) if prec == "bf16" else xh[n].astype(np.float64)
        ref = evsnet.backward_along(xo, ows, theta, leak, Gh[n], split_layers(h[n], wl.channels))
        for l in range(len(ws)):
            dW_ref[l] += ref["dW"][l]
        rx = _np_rel(dxh[n], ref["dx"])
        dvl = split_layers(dvh[n][None], wl.channels)
        rv = max(_np_rel(a[0], b) for a, b in zip(dvl, ref["dv_init"]))
        print(f"  crop {n}: dx rel {rx:.2e}, dv_init rel {rv:.2e}", flush=True)
        assert rx < grad_tol(prec) and rv < grad_tol(prec)
    for l in range(len(ws)):
        r = _np_rel(gw[l].cpu().numpy(), dW_ref[l])
        print(f"  layer {l + 1} dW rel {r:.2e}", flush=True)
        assert r < grad_tol(prec)


def _np_rel(a, b):
    import numpy as np
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))
