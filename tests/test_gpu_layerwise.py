"""GPU parity of the layer-by-layer path (through the C ABI): networks the
fused kernels do not cover -- more than three layers, hidden layers of
different widths, hidden widths with no fused build -- against the FP64
oracle, with the gates of test_gpu_forward.py and test_gpu_backward.py:

  * forward, teacher-forced per layer: FP32 membrane rel. error <= 1e-5;
    BF16 <= 2e-2 against the unquantised step and <= 1e-5 against the
    BF16-quantised one; spike mismatches <= 1e-4 and only inside the band;
    output spikes equal the fire rule on the device's own potentials;
  * state carry: a clip split in two windows with v_state carried gives the
    same spikes and final state bit for bit, and each checkpoint equals the
    state a shorter run ends with;
  * a trace window equals that window of the full trace;
  * BPTT along the device's trajectory: FP32 <= 1e-4, BF16 the gradient
    gate of tests/_helpers.py.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from oracle import evsnet  # noqa: E402
from tests._helpers import f32, fire32, grad_tol, make_inputs, split_layers, teacher_forced_report  # noqa: E402

THETA, LEAK = f32(0.5), f32(0.9)

CASES = [
    ((3, 8, 16, 2), "fp32"),                       # unequal hidden widths
    ((3, 8, 8, 8, 8, 2), "fp32"),                  # five layers
    ((1, 4, 6, 8, 6, 4, 4, 4, 2), "fp32"),         # eight layers, one input channel
    ((3, 32, 32, 2), "fp32"),                      # two 32-wide layers (no fused FP32 build)
    ((3, 16, 32, 2), "bf16"),
    ((3, 5, 12, 7, 1), "bf16"),                    # widths that are not multiples of 4
]


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


def _net(evs, channels, prec, ws):
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    return net, packed


@pytest.mark.parametrize("channels,prec", CASES)
def test_layerwise_forward_teacher_forced_parity(evs, channels, prec):
    N, T, H, W = 2, 6, 37, 45
    print(f"case layerwise {channels} {prec}", flush=True)
    x, ws = make_inputs(channels, T, H, W, N=N, seed=len(channels) + 7)
    net, packed = _net(evs, channels, prec, ws)
    assert evs.tile_count(net) == 0                 # no fused kernel: the layer-by-layer path
    out = evs.forward(net, packed, x.cuda(), trace=True)
    torch.cuda.synchronize()
    s = out["s"].cpu().numpy().astype(np.float64)
    h = out["h"].cpu().numpy()
    assert int(np.abs(s).sum()) > 0
    for n in range(N):
        hl = split_layers(h[n], channels)
        np.testing.assert_array_equal(s[n], fire32(hl[-1], THETA))
        xn = x[n].numpy()
        if prec == "bf16":
            rep = teacher_forced_report(xn, ws, THETA, LEAK, hl, quant_ws=[evsnet.bf16_round(w) for w in ws],
                                        quant_x=evsnet.bf16_round(xn))
        else:
            rep = teacher_forced_report(xn, ws, THETA, LEAK, hl)
        for l, r in enumerate(rep):
            print(f"  n={n} layer {l + 1}: {r}", flush=True)
            if prec == "bf16":
                assert r["qrel"] <= 1e-5, r
                assert r["rel"] <= 2e-2, r
            else:
                assert r["rel"] <= 1e-5, r
            assert r["outside"] == 0, r
            assert r["mism"] <= max(1, 1e-4 * r["n"]), r


@pytest.mark.parametrize("channels,prec", [((3, 8, 8, 8, 8, 2), "fp32"), ((3, 16, 32, 2), "bf16")])
def test_layerwise_state_carry_checkpoints_and_trace_window(evs, channels, prec):
    N, T, H, W, k = 1, 7, 30, 41, 3
    x, ws = make_inputs(channels, T, H, W, N=N, seed=5)
    net, packed = _net(evs, channels, prec, ws)
    xg = x.cuda()
    v_full = torch.zeros(N, net.sum_c, H, W, device="cuda")
    full = evs.forward(net, packed, xg, v_state=v_full, trace=True, ckpt_every=k)
    v_a = torch.zeros_like(v_full)
    a = evs.forward(net, packed, xg[:, :4].contiguous(), v_state=v_a)
    b = evs.forward(net, packed, xg[:, 4:].contiguous(), v_state=v_a)
    v_k = torch.zeros_like(v_full)
    evs.forward(net, packed, xg[:, :k].contiguous(), v_state=v_k)
    box = (5, 7, 11, 13)
    win = evs.forward(net, packed, xg, trace=True, trace_box=box)
    torch.cuda.synchronize()
    assert torch.equal(torch.cat([a["s"], b["s"]], dim=1), full["s"])
    assert torch.equal(v_a, v_full)
    assert torch.equal(full["ckpt"][:, 0], torch.zeros_like(v_full))
    assert torch.equal(full["ckpt"][:, 1], v_k)
    y0, x0, bh, bw = box
    assert torch.equal(win["h"], full["h"][:, :, :, y0:y0 + bh, x0:x0 + bw])


@pytest.mark.parametrize("channels,prec", [((3, 8, 16, 2), "fp32"), ((3, 8, 8, 8, 8, 2), "fp32"),
                                           ((1, 12, 16, 2), "fp32"),    # one input channel, fused input-layer dW
                                           ((3, 16, 32, 2), "bf16"), ((3, 5, 12, 7, 1), "bf16")])
@pytest.mark.parametrize("k", [4, 100])
def test_layerwise_backward_matches_oracle(evs, channels, prec, k):
    N, T, H, W = 2, 9, 21, 27
    print(f"case layerwise backward {channels} {prec} k={k}", flush=True)
    x, ws = make_inputs(channels, T, H, W, N=N, seed=3)
    net, packed = _net(evs, channels, prec, ws)
    xg = x.cuda()
    out = evs.forward(net, packed, xg, trace=True, ckpt_every=k)
    G = np.random.default_rng(1).normal(size=(N, T, channels[-1], H, W)).astype(np.float32)
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
    tol = grad_tol(prec)
    dW_ref = [np.zeros_like(w) for w in ows]

    def rel(a, b):
        return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-12))

    for n in range(N):
        g = evsnet.backward_along(xo[n], ows, THETA, LEAK, G[n], split_layers(h[n], channels))
        for l in range(len(ws)):
            dW_ref[l] += g["dW"][l]
        r = rel(dx[n].cpu().numpy(), g["dx"])
        print(f"  clip {n} dx rel err {r:.2e}", flush=True)
        assert r < tol
        for a, b in zip(split_layers(dv[n].cpu().numpy()[None], channels), g["dv_init"]):
            assert rel(a[0], b) < tol
    for l in range(len(ws)):
        r = rel(gws[l].cpu().numpy(), dW_ref[l])
        print(f"  layer {l + 1} dW rel err {r:.2e}", flush=True)
        assert r < tol


@pytest.mark.parametrize("surr,alpha", [("sigmoid", 4.0), ("atan", 2.0)])
def test_layerwise_relaxed_backward_matches_oracle_and_finite_differences(evs, surr, alpha):
    """Smooth spikes through four layers (8x8 pixels, 4 frames): BPTT against
    the oracle's relaxed BPTT and against central differences of the GPU's
    own relaxed forward."""
    channels = (3, 6, 10, 6, 2)
    T, H, W = 4, 8, 8
    x, ws = make_inputs(channels, T, H, W, seed=13)
    net = evs.Net(channels, theta=THETA, leak=LEAK, relaxed=True, surrogate=surr, surr_alpha=alpha)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    assert evs.tile_count(net) == 0
    xg = x.cuda()
    G = np.random.default_rng(4).normal(size=(1, T, 2, H, W)).astype(np.float32)
    Gt = torch.from_numpy(G).cuda()
    out = evs.forward(net, packed, xg, s_fp32=True, ckpt_every=2)
    gws, dx, _ = evs.backward(net, packed, xg, out["ckpt"], 2, Gt, want_dx=True)
    torch.cuda.synchronize()
    ref = evsnet.backward(x[0].numpy(), ws, THETA, LEAK, G[0], mode="relaxed", alpha=alpha, surr=surr)

    def rel(a, b):
        return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-12))

    for l in range(len(ws)):
        assert rel(gws[l].cpu().numpy(), ref["dW"][l]) < 1e-4
    assert rel(dx[0].cpu().numpy(), ref["dx"]) < 1e-4

    def loss(wlist):
        p = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in wlist])
        o = evs.forward(net, p, xg, s_fp32=True)
        return float((o["s"].double() * Gt.double()).sum())

    rng = np.random.default_rng(0)
    eps = 2e-3
    errs = []
    for l in range(len(ws)):
        for _ in range(4):
            idx = tuple(int(rng.integers(0, n)) for n in ws[l].shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += eps
            wm[l][idx] -= eps
            errs.append(abs((loss(wp) - loss(wm)) / (2 * eps) - float(gws[l].cpu().numpy()[idx]))
                        / max(1.0, abs((loss(wp) - loss(wm)) / (2 * eps))))
    print(f"  relaxed FD max err {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-2


def test_layerwise_rgb_input_equals_logdiff_then_direct(evs):
    """RGB input on the layer-by-layer path: the Eq. (1) frames formed first,
    spikes and potentials bit for bit those of evs_logdiff followed by the
    direct-input forward."""
    channels = (1, 6, 8, 6, 2)
    N, T, H, W = 1, 5, 29, 35
    rng = np.random.default_rng(21)
    rgb = torch.from_numpy(rng.uniform(0.0, 1.0, size=(N, T + 1, 3, H, W)).astype(np.float32)).cuda()
    _, ws = make_inputs(channels, T, H, W, seed=2)
    net_rgb = evs.Net(channels, theta=THETA, leak=LEAK, input="rgb_logdiff")
    net = evs.Net(channels, theta=THETA, leak=LEAK)
    assert evs.tile_count(net_rgb) == 0
    p_rgb = evs.pack_weights(net_rgb, [torch.from_numpy(w).cuda() for w in ws])
    p = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    a = evs.forward(net_rgb, p_rgb, rgb, trace=True)
    x = evs.logdiff(rgb, net_rgb.lum_scale, net_rgb.knee)
    b = evs.forward(net, p, x, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(a["s"], b["s"])
    assert torch.equal(a["h"], b["h"])
