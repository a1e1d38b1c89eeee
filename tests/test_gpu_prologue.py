"""GPU parity of the network input of Eq. (1) and of the contrast-crossing
target generator (through the C ABI) against the FP64 oracle.

* evs_logdiff: X = L_log[k] - L_log[k-1] within FP32 rounding of the logs
  (|err| <= 4e-6 + 1e-6 |X|), on frames whose luminance spans both sides of
  the knee; constant frames give exactly zero.
* evs_contrast_events: the event counts decide integers from floats, so the
  comparison is exact on every pixel whose oracle decisions keep a margin of
  1e-4 from an integer boundary; the remaining pixels (a handful) must still
  account for the log change within C.  Frame 0 is zero everywhere.
* A one-channel net driven by the GPU's X through the forward: parity with
  the oracle on the same input (teacher-forced, FP32 gate).
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import evsnet, prologue  # noqa: E402
from tests._helpers import f32, split_layers, teacher_forced_report  # noqa: E402

THETA, LEAK = f32(0.5), f32(0.9)


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


def _frames(T, H, W, N=1, seed=0, clean=False):
    """Seeded RGB frames of the textured-planes scene under a horizontal
    exposure ramp (x0.05 .. x2), so that the luminance spans both sides of
    the knee of 20 on the 0-255 scale."""
    wl = synth.WORKLOADS["planes720"]
    ramp = np.geomspace(0.05, 2.0, W).astype(np.float32)
    out = []
    for n in range(N):
        x = synth.make_clip(wl, T=T, H=H, W=W, y0=41 + 53 * n, x0=17 + 29 * n, noise_seed=seed + n, clean=clean)
        out.append(x.numpy() * ramp)
    return np.stack(out).astype(np.float32)


@pytest.mark.parametrize("N,T,H,W", [(1, 9, 37, 53), (2, 5, 64, 80), (1, 1, 1, 1)])
def test_logdiff_matches_oracle(evs, N, T, H, W):
    rgb = _frames(T + 1, H, W, N=N, seed=3)
    X = evs.logdiff(torch.from_numpy(rgb).cuda())
    torch.cuda.synchronize()
    assert X.shape == (N, T, 1, H, W)
    Xd = X.cpu().numpy()
    for n in range(N):
        ref = prologue.logdiff(rgb[n].astype(np.float64))
        err = np.abs(Xd[n] - ref)
        assert np.all(err <= 4e-6 + 1e-6 * np.abs(ref)), float((err - 1e-6 * np.abs(ref)).max())
    if H * W > 1:
        lum = prologue.luminance(rgb.astype(np.float64))
        assert (lum < 20).any() and (lum >= 20).any()


def test_logdiff_constant_frames_are_zero(evs):
    rgb = np.repeat(_frames(1, 33, 41, seed=1), 6, axis=1)
    X = evs.logdiff(torch.from_numpy(rgb).cuda())
    torch.cuda.synchronize()
    assert float(X.abs().max()) == 0.0


@pytest.mark.parametrize("N,T,H,W", [(1, 40, 48, 72), (2, 17, 31, 29)])
def test_contrast_events_match_oracle(evs, N, T, H, W):
    C = 0.2
    rgb = _frames(T, H, W, N=N, seed=5, clean=True)
    E = evs.contrast_events(torch.from_numpy(rgb).cuda(), C=C)
    torch.cuda.synchronize()
    Ed = E.cpu().numpy()
    assert np.all(Ed[:, 0] == 0)
    n_amb = 0
    for n in range(N):
        f = rgb[n].astype(np.float64)
        ref = prologue.contrast_events(f, C)
        margin = prologue.contrast_margin(f, C)
        sure = margin > 1e-4
        n_amb += int((~sure).sum())
        np.testing.assert_array_equal(Ed[n][:, :, sure], ref[:, :, sure])
        lg = prologue.linlog(prologue.luminance(f))
        net = (Ed[n][:, 0].astype(np.float64) - Ed[n][:, 1]).sum(axis=0)
        assert np.all(np.abs(lg[-1] - lg[0] - C * net) < C + 1e-4)
    print(f"  contrast events: {int((Ed != 0).sum())} non-zero counts, {n_amb} near-boundary pixels", flush=True)
    assert int((Ed != 0).sum()) > 0
    assert n_amb < 0.01 * N * H * W


def test_one_channel_net_on_gpu_logdiff(evs):
    """RGB -> X (GPU) -> conv3x3 1->16->2 + BiLIF (GPU) vs the oracle forward of
    the same X (teacher-forced FP32 gate)."""
    channels = (1, 16, 2)
    T, H, W = 8, 45, 61
    rgb = _frames(T + 1, H, W, seed=7)
    X = evs.logdiff(torch.from_numpy(rgb).cuda())
    ws = synth.he_weights(channels, 0)
    ws = [w * 6.0 for w in ws]               # X is a small log difference: scale the weights up
    net = evs.Net(channels, theta=THETA, leak=LEAK)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    out = evs.forward(net, packed, X, trace=True)
    torch.cuda.synchronize()
    x64 = X[0].cpu().numpy().astype(np.float64)
    h = split_layers(out["h"][0].cpu().numpy(), channels)
    rep = teacher_forced_report(x64, ws, THETA, LEAK, h)
    print(f"  1-ch net on logdiff: {rep}", flush=True)
    for r in rep:
        assert r["rel"] <= 1e-5
        assert r["outside"] == 0
    ref = evsnet.forward(x64, ws, THETA, LEAK)
    assert int(np.abs(ref["s"]).sum()) > 0


@pytest.mark.parametrize("channels,N,T,H,W", [((1, 2), 2, 7, 45, 61), ((1, 16, 2), 2, 9, 45, 61),
                                              ((1, 16, 2), 1, 5, 64, 83)])
def test_fused_rgb_input_matches_two_pass(evs, channels, N, T, H, W):
    """A net with input="rgb_logdiff" forms X of Eq. (1) while staging the RGB
    frames; spikes, traces and final state are bit-identical to running the
    direct-input net on evs_logdiff's X (inference, debug and relaxed
    kernels), and a clip split in two windows with the state carried gives
    the same spikes (each window re-reads its first RGB frame)."""
    rgb = _frames(T + 1, H, W, N=N, seed=11)
    ws = [w * 6.0 for w in synth.he_weights(channels, 1)]
    rg = torch.from_numpy(rgb).cuda()
    X = evs.logdiff(rg)
    sum_c = sum(channels[1:])
    for relaxed in (False, True):
        nx = evs.Net(channels, theta=THETA, leak=LEAK, relaxed=relaxed)
        nr = evs.Net(channels, theta=THETA, leak=LEAK, relaxed=relaxed, input="rgb_logdiff")
        packed = evs.pack_weights(nx, [torch.from_numpy(w).cuda() for w in ws])
        for debug in ((False, True) if not relaxed else (True,)):
            v1 = torch.zeros(N, sum_c, H, W, device="cuda")
            v2 = torch.zeros(N, sum_c, H, W, device="cuda")
            a = evs.forward(nx, packed, X, v_state=v1, trace=debug, s_fp32=debug)
            b = evs.forward(nr, packed, rg, v_state=v2, trace=debug, s_fp32=debug)
            torch.cuda.synchronize()
            print(f"  fused RGB input {channels} relaxed={relaxed} debug={debug}", flush=True)
            assert torch.equal(a["s"], b["s"])
            assert torch.equal(v1, v2)
            if debug:
                assert torch.equal(a["h"], b["h"])
            assert int((a["s"] != 0).sum()) > 0
        if not relaxed:
            T1 = T // 2
            v = torch.zeros(N, sum_c, H, W, device="cuda")
            s1 = evs.forward(nr, packed, rg[:, : T1 + 1].contiguous(), v_state=v)["s"]
            s2 = evs.forward(nr, packed, rg[:, T1:].contiguous(), v_state=v)["s"]
            torch.cuda.synchronize()
            full = evs.forward(nx, packed, X)["s"]
            torch.cuda.synchronize()
            assert torch.equal(torch.cat([s1, s2], dim=1), full)
