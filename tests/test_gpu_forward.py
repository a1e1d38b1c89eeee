"""GPU parity of the HIP forward against the FP64 oracle (through the C ABI).

Gates (per layer, teacher-forced one-step checks driven by the device's own
trajectory):
  * FP32: membrane rel. error <= 1e-5 against the FP64 step;
  * BF16: membrane rel. error <= 2e-2 against the unquantised FP64 step and
    <= 1e-5 against the BF16-quantised FP64 step;
  * spikes: mismatch fraction <= 1e-4 and every mismatch inside the band
    |h_ref -+ theta| < 1e-3 (quantised reference for BF16);
  * the emitted output spikes equal the fire rule applied to the device's
    own potentials, bit for bit.
Invariants (zero input, chunking, tile shape, batching) are exact; oddness holds
for spikes and to float32 rounding for potentials.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from oracle import evsnet  # noqa: E402
from tests._helpers import (f32, fire32, make_inputs, split_layers,  # noqa: E402
                            teacher_forced_report)

THETA, LEAK = f32(0.5), f32(0.9)

CASES = [
    # channels, precision, N, T, H, W
    ((3, 8, 2), "fp32", 2, 8, 70, 90),
    ((3, 16, 16, 2), "fp32", 1, 8, 70, 90),
    ((3, 32, 2), "fp32", 1, 6, 53, 75),
    ((3, 32, 2), "bf16", 2, 8, 70, 90),
    ((3, 16, 16, 2), "bf16", 1, 8, 70, 90),
    ((3, 4, 1), "fp32", 1, 6, 40, 33),
    ((1, 16, 2), "fp32", 1, 6, 40, 50),
    ((1, 1), "fp32", 1, 6, 40, 50),
    ((3, 2), "fp32", 1, 6, 37, 70),
    # degenerate and ragged shapes: one pixel and one frame, two rows across
    # several tiles, one column, a frame smaller than a tile (three clips)
    ((3, 16, 16, 2), "fp32", 2, 1, 1, 1),
    ((3, 16, 16, 2), "bf16", 1, 3, 2, 130),
    ((3, 32, 2), "bf16", 1, 2, 45, 1),
    ((3, 32, 2), "fp32", 3, 1, 5, 7),
    ((3, 8, 2), "fp32", 1, 4, 33, 65),
]


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


def _run(evs, channels, prec, x, ws, **kw):
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    wt = [torch.from_numpy(w).cuda() for w in ws]
    packed = evs.pack_weights(net, wt)
    out = evs.forward(net, packed, x.cuda(), trace=True, **kw)
    torch.cuda.synchronize()
    return net, packed, out


@pytest.mark.parametrize("channels,prec,N,T,H,W", CASES)
def test_forward_teacher_forced_parity(evs, channels, prec, N, T, H, W):
    print(f"case channels={channels} prec={prec} N={N} T={T} H={H} W={W}", flush=True)
    x, ws = make_inputs(channels, T, H, W, N=N, seed=len(channels) + H)
    net, _, out = _run(evs, channels, prec, x, ws)
    s = out["s"].cpu().numpy().astype(np.float64)
    h = out["h"].cpu().numpy()
    for n in range(N):
        hl = split_layers(h[n], channels)
        # output spikes are the fire rule on the device's own potentials
        np.testing.assert_array_equal(s[n], fire32(hl[-1], THETA))
        xn = x[n].numpy()
        if prec == "bf16":
            qws = [evsnet.bf16_round(w) for w in ws]
            qx = evsnet.bf16_round(xn)
            rep = teacher_forced_report(xn, ws, THETA, LEAK, hl, quant_ws=qws, quant_x=qx)
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
    # free-running comparison is reported (not gated): chaotic divergence
    # after a near-threshold step is legitimate
    if prec == "fp32":
        ref = evsnet.forward(x[0].numpy(), ws, THETA, LEAK)
        mis = (ref["s"] != s[0]).mean()
        print(f"  free-running output mismatch fraction {mis:.2e}", flush=True)
        if ref["s"].size >= 10000:
            assert mis <= 1e-3


@pytest.mark.parametrize("channels", [(3, 16, 16, 2), (3, 32, 2)])
@pytest.mark.parametrize("scale", [2.0 ** 13, 2.0 ** -16])
def test_fp32_split_input_layer_over_the_input_range(evs, channels, scale):
    """FP32 nets with three input channels split x into two fp16 parts in
    their input layer.  The FP32 gate holds near the top of the accepted
    range (max |x| about 4.3e4, below 65520) and where most values are fp16
    subnormals (max |x| about 8e-5)."""
    print(f"case split range channels={channels} scale={scale}", flush=True)
    x, ws = make_inputs(channels, 4, 45, 61, seed=11, scale=scale)
    _, _, out = _run(evs, channels, "fp32", x, ws)
    hl = split_layers(out["h"][0].cpu().numpy(), channels)
    rep = teacher_forced_report(x[0].numpy(), ws, THETA, LEAK, hl)
    for l, r in enumerate(rep):
        print(f"  layer {l + 1}: {r}", flush=True)
        assert r["rel"] <= 1e-5, r
        assert r["outside"] == 0, r
        assert r["mism"] <= max(1, 1e-4 * r["n"]), r


def test_zero_input_gives_no_spikes(evs):
    x = torch.zeros(1, 5, 3, 40, 50)
    _, ws = make_inputs((3, 16, 16, 2), 1, 4, 4)
    _, _, out = _run(evs, (3, 16, 16, 2), "fp32", x, ws)
    assert int(out["s"].abs().sum()) == 0
    assert float(out["h"].abs().max()) == 0.0


@pytest.mark.parametrize("prec,bound", [("fp32", 1e-6), ("bf16", 1e-5)])
def test_oddness_up_to_accumulator_rounding(evs, prec, bound):
    """Negating the input negates every potential and spike (the oracle's
    oddness pin).  The layers that read spikes run on the bf16 matrix core
    (FP32 nets through fp16 weight parts), whose FP32
    accumulation on gfx950 is not exactly sign-symmetric: potentials agree
    to float32 rounding and spikes may differ only where the potential sits
    at a threshold."""
    x, ws = make_inputs((3, 16, 16, 2), 6, 45, 61)
    _, _, a = _run(evs, (3, 16, 16, 2), prec, x, ws)
    _, _, b = _run(evs, (3, 16, 16, 2), prec, -x, ws)
    d = (b["h"] + a["h"]).abs()
    rel = float(d.max() / a["h"].abs().max())
    print(f"  {prec} oddness: max |h(-x) + h(x)| / max|h| = {rel:.3e}, "
          f"differing potentials {int((d > 0).sum())} of {d.numel()}", flush=True)
    assert rel <= bound
    assert int(a["s"].abs().sum()) > 0
    mism = b["s"] != -a["s"]
    if mism.any():
        hl = a["h"][:, :, -2:][mism]
        assert float((hl.abs() - 0.5).abs().max()) < 1e-4


@pytest.mark.parametrize("channels,prec", [((3, 16, 16, 2), "fp32"), ((3, 32, 2), "bf16"),
                                           ((3, 32, 2), "fp32"), ((3, 8, 2), "fp32")])
def test_tile_shape_independence_is_bitwise(evs, channels, prec):
    x, ws = make_inputs(channels, 5, 67, 101)
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    n = evs.tile_count(net)
    assert n >= 1
    outs = []
    try:
        for t in range(n):
            evs.set_tile(net, t)
            _, _, o = _run(evs, channels, prec, x, ws)
            outs.append(o)
    finally:
        evs.set_tile(net, -1)
    for o in outs[1:]:
        assert torch.equal(o["s"], outs[0]["s"])
        assert torch.equal(o["h"], outs[0]["h"])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_chunked_state_carry_is_bitwise(evs, prec):
    channels = (3, 16, 16, 2)
    x, ws = make_inputs(channels, 9, 50, 70)
    net, packed, full = _run(evs, channels, prec, x, ws)
    v = torch.zeros(1, net.sum_c, 50, 70, device="cuda")
    xa, xb = x[:, :4].contiguous().cuda(), x[:, 4:].contiguous().cuda()
    a = evs.forward(net, packed, xa, v_state=v, trace=True)
    b = evs.forward(net, packed, xb, v_state=v, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.cat([a["s"], b["s"]], 1), full["s"])
    assert torch.equal(torch.cat([a["h"], b["h"]], 1), full["h"])


def test_batch_equals_separate_clips(evs):
    channels = (3, 16, 16, 2)
    x, ws = make_inputs(channels, 5, 40, 60, N=3)
    _, _, both = _run(evs, channels, "fp32", x, ws)
    for n in range(3):
        _, _, one = _run(evs, channels, "fp32", x[n:n + 1].contiguous(), ws)
        assert torch.equal(one["s"][0], both["s"][n])


def test_initial_state_and_checkpoints(evs):
    channels = (3, 16, 16, 2)
    T, H, W = 10, 41, 57
    x, ws = make_inputs(channels, T, H, W)
    net = evs.Net(channels, theta=THETA, leak=LEAK)
    rng = np.random.default_rng(5)
    v0 = rng.normal(0, 0.3, size=(1, net.sum_c, H, W)).astype(np.float32)
    wt = [torch.from_numpy(w).cuda() for w in ws]
    packed = evs.pack_weights(net, wt)
    v = torch.from_numpy(v0).cuda()
    out = evs.forward(net, packed, x.cuda(), v_state=v, trace=True, ckpt_every=4)
    torch.cuda.synchronize()
    h = out["h"][0].cpu().numpy()
    hl = split_layers(h, channels)
    v0l = split_layers(v0[0][None], channels)
    rep = teacher_forced_report(x[0].numpy(), ws, THETA, LEAK, hl, v_init=[a[0] for a in v0l])
    for r in rep:
        assert r["rel"] <= 1e-5 and r["outside"] == 0, r
    ck = out["ckpt"][0].cpu().numpy()
    np.testing.assert_array_equal(ck[0], v0[0])
    # checkpoint k holds v[t0 - 1] = h - theta * s in float32
    for seg, t0 in enumerate(range(0, T, 4)):
        if t0 == 0:
            continue
        hv = h[t0 - 1].astype(np.float32)
        vv = hv - np.float32(THETA) * fire32(hv, THETA).astype(np.float32)
        np.testing.assert_array_equal(ck[seg], vv)
    # final state
    hv = h[T - 1].astype(np.float32)
    np.testing.assert_array_equal(v[0].cpu().numpy(), hv - np.float32(THETA) * fire32(hv, THETA).astype(np.float32))


@pytest.mark.parametrize("surr,alpha", [("sigmoid", 4.0), ("atan", 2.0)])
def test_relaxed_forward_matches_oracle(evs, surr, alpha):
    channels = (3, 16, 16, 2)
    x, ws = make_inputs(channels, 6, 30, 44)
    net = evs.Net(channels, theta=THETA, leak=LEAK, relaxed=True, surrogate=surr, surr_alpha=alpha)
    wt = [torch.from_numpy(w).cuda() for w in ws]
    packed = evs.pack_weights(net, wt)
    out = evs.forward(net, packed, x.cuda(), s_fp32=True, trace=True)
    torch.cuda.synchronize()
    ref = evsnet.forward(x[0].numpy(), ws, THETA, LEAK, mode="relaxed", alpha=alpha, surr=surr)
    s = out["s"][0].cpu().numpy()
    np.testing.assert_allclose(s, ref["s"], atol=2e-4)
    h = split_layers(out["h"][0].cpu().numpy(), channels)
    for hd, hr in zip(h, ref["h"]):
        assert np.abs(hd - hr).max() / np.abs(hr).max() < 1e-4


@pytest.mark.parametrize("channels,prec", [((3, 16, 16, 2), "fp32"), ((3, 32, 2), "bf16")])
def test_inference_kernel_equals_traced_kernel_and_trace_window(evs, channels, prec):
    """The inference build (no traces) and the training/debug build emit the
    same spikes bit for bit; a windowed trace equals that window of the
    full trace."""
    x, ws = make_inputs(channels, 6, 70, 90)
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    xg = x.cuda()
    fast = evs.forward(net, packed, xg)
    full = evs.forward(net, packed, xg, trace=True)
    win = evs.forward(net, packed, xg, trace=True, trace_box=(13, 29, 20, 31))
    torch.cuda.synchronize()
    assert torch.equal(fast["s"], full["s"])
    assert torch.equal(win["s"], full["s"])
    assert torch.equal(win["h"], full["h"][:, :, :, 13:33, 29:60])


@pytest.mark.parametrize("channels,prec", [((3, 16, 16, 2), "fp32"), ((3, 16, 16, 2), "bf16"),
                                           ((3, 32, 2), "bf16"), ((3, 32, 2), "fp32"), ((3, 8, 2), "fp32")])
@pytest.mark.parametrize("T", [4, 7])
def test_every_tile_inference_kernel_equals_traced_kernel(evs, channels, prec, T):
    """The inference build of every compiled tile shape (the kernels the
    autotuner may pick) gives the spikes of the traced build, which the
    teacher-forced parity tests hold to the oracle, bit for bit."""
    H, W = 70, 90
    x, ws = make_inputs(channels, T, H, W, N=2)
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    xg = x.cuda()
    n = evs.tile_count(net)
    bad = []
    try:
        evs.set_tile(net, 0)
        ref = evs.forward(net, packed, xg, trace=True)["s"]
        for t in range(n):
            evs.set_tile(net, t)
            o = evs.forward(net, packed, xg)["s"]
            torch.cuda.synchronize()
            if not torch.equal(o, ref):
                d = (o != ref)
                frames = sorted(set(torch.nonzero(d)[:, 1].tolist()))
                bad.append((evs.tile_name(net, t), int(d.sum()), frames))
    finally:
        evs.set_tile(net, -1)
    print(f"  {channels} {prec} T={T}: {n} tiles, differing: {bad}", flush=True)
    assert not bad


@pytest.mark.parametrize("channels,prec", [((3, 16, 16, 2), "fp32"), ((3, 16, 16, 2), "bf16"),
                                           ((3, 32, 2), "fp32"), ((3, 32, 2), "bf16"), ((3, 8, 2), "fp32"),
                                           ((3, 10, 10, 2), "fp32"), ((3, 32, 32, 2), "bf16")])
def test_prepacked_fragments_equal_built_ones(evs, channels, prec):
    """evs_pack_weights stores the MFMA fragments of the forward kernels
    (built once); a kernel whose packed block is not valid builds its own
    from the FP32 weights.  Both give the same spikes, potentials and
    checkpoints bit for bit (inference, traced and training-step builds)."""
    import ctypes
    from paper_2508_18071_amd import _lib
    print(f"case prepack {channels} {prec}", flush=True)
    T, H, W = 7, 45, 70
    x, ws = make_inputs(channels, T, H, W, seed=5)
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    nfl = sum(ci * co * 9 for ci, co in zip(channels[:-1], channels[1:]))
    off = (nfl * 4 + 255) // 256 * 256
    assert packed.numel() > off, "the packed buffer carries a fragment block"
    plain = packed.clone()
    plain[off:] = 0                                    # no valid header: kernels build their own
    xg = x.cuda()
    outs = []
    for p in (packed, plain):
        a = evs.forward(net, p, xg)
        b = evs.forward(net, p, xg, trace=True)
        c = evs.forward(net, p, xg, s_fp32=True, ckpt_every=3)
        torch.cuda.synchronize()
        outs.append((a["s"], b["s"], b["h"], c["s"], c["ckpt"]))
    for u, v in zip(*outs):
        assert torch.equal(u, v)
