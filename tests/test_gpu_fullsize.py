"""Parity at the full benchmark size, in the launch configuration bench.py
times (1000 frames of 1280x720, default tile, inference kernel).

The inference kernel's spikes are compared bit for bit with the
training/debug kernel's, which also records the charged potentials of every
layer in a few 16x16 windows; those windows are then checked teacher-forced
against the FP64 oracle over all 1000 frames (every step recomputed from the
device's own previous state and input spikes): FP32 rel. error <= 1e-5,
BF16 <= 1e-5 against the BF16-quantised oracle and <= 2e-2 against the
unquantised one, spike mismatches only inside |h -+ theta| < 1e-3.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from oracle import evsnet  # noqa: E402
from tests._helpers import f32  # noqa: E402

THETA, LEAK = f32(0.5), f32(0.9)
BOXES = [(100, 200), (352, 640), (700, 1250)]     # top-left corners of 16x16 windows


@pytest.fixture(scope="module")
def clip720():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import synth
    wl = synth.WORKLOADS["planes720"]
    x = torch.empty(1, 1000, 3, 720, 1280, device="cuda")
    synth.make_clip(wl, device="cuda", T=1000, out=x[0])
    torch.cuda.synchronize()
    return x


def _window_check(x, ws, h, y0, x0, channels, theta, leak, qws=None, quant=False):
    """Teacher-forced one-step check of a 16x16 trace window; returns
    (max rel err vs FP64, max rel err vs quantised FP64, mismatches outside band)."""
    T = h.shape[0]
    H, W = x.shape[2], x.shape[3]
    ya, xa = max(0, y0 - 1), max(0, x0 - 1)
    xc = x[:, :, ya:y0 + 17, xa:x0 + 17].astype(np.float64)
    oy, ox = y0 - ya, x0 - xa
    res = []
    o = 0
    hl = []
    for c in channels[1:]:
        hl.append(h[:, o:o + c].astype(np.float64))
        o += c
    worst, worst_q, outside = 0.0, 0.0, 0
    for l, w in enumerate(ws):
        wq = qws[l] if qws is not None else None
        hd = hl[l]
        sd = evsnet.fire(hd, theta)
        vd = hd - theta * sd
        for t in range(T):
            vprev = vd[t - 1] if t > 0 else np.zeros_like(hd[0])
            if l == 0:
                xin = evsnet.bf16_round(xc[t]) if quant else xc[t]
                full = [evsnet.conv3x3(xc[t], w)[:, oy:oy + 16, ox:ox + 16]]
                if wq is not None:
                    full.append(evsnet.conv3x3(xin, wq)[:, oy:oy + 16, ox:ox + 16])
                sl = (slice(None), slice(0, 16), slice(0, 16))
            else:
                sin = evsnet.fire(hl[l - 1][t], theta)
                full = [evsnet.conv3x3(sin, w)]
                if wq is not None:
                    full.append(evsnet.conv3x3(sin, wq))
                sl = (slice(None), slice(1, 15), slice(1, 15))    # inputs known inside the window only
            ref = leak * vprev + full[0]
            rq = leak * vprev + full[-1]
            a, b, bq = hd[t][sl], ref[sl], rq[sl]
            worst = max(worst, np.abs(a - b).max() / max(np.abs(b).max(), 1e-12))
            worst_q = max(worst_q, np.abs(a - bq).max() / max(np.abs(bq).max(), 1e-12))
            mism = evsnet.fire(a, theta) != evsnet.fire(bq, theta)
            outside += int((mism & (evsnet.spike_margin(bq, theta) >= 1e-3)).sum())
    return worst, worst_q, outside


@pytest.mark.parametrize("channels,prec", [((3, 16, 16, 2), "fp32"), ((3, 16, 16, 2), "bf16"), ((3, 32, 2), "bf16"),
                                          ((3, 32, 2), "fp32")])
def test_fullsize_720p_1000_frames(clip720, channels, prec):
    import paper_2508_18071_amd as evs
    import synth
    print(f"case 720p x 1000 frames {channels} {prec}", flush=True)
    ws = synth.he_weights(channels, 0)
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    fast = evs.forward(net, packed, clip720)["s"]          # bench configuration
    torch.cuda.synchronize()
    qws = [evsnet.bf16_round(w) for w in ws] if prec == "bf16" else None
    for (y0, x0) in BOXES:
        y0, x0 = min(y0, 720 - 16), min(x0, 1280 - 16)
        full = evs.forward(net, packed, clip720, trace=True, trace_box=(y0, x0, 16, 16))
        torch.cuda.synchronize()
        assert torch.equal(full["s"], fast), "inference and traced kernels disagree"
        xw = clip720[0, :, :, max(0, y0 - 1):y0 + 17, max(0, x0 - 1):x0 + 17].cpu().numpy()
        # re-embed so that the window helper sees image coordinates
        h = full["h"][0].cpu().numpy()
        err, errq, outside = _window_check_img(clip720, xw, ws, h, y0, x0, channels, qws, prec == "bf16")
        print(f"  window ({y0},{x0}): rel {err:.2e} quantised-rel {errq:.2e} outside-band {outside}", flush=True)
        if prec == "bf16":
            assert errq <= 1e-5 and err <= 2e-2
        else:
            assert err <= 1e-5
        assert outside == 0
    del fast


def _window_check_img(clip, xw, ws, h, y0, x0, channels, qws, quant):
    # xw is the window plus a 1-pixel halo clipped at the image border;
    # pad it back so that the window sits at offset (1, 1)
    T = xw.shape[0]
    pad = np.zeros((T, 3, 18, 18), np.float32)
    ya, xa = max(0, y0 - 1), max(0, x0 - 1)
    py, px = ya - (y0 - 1), xa - (x0 - 1)
    pad[:, :, py:py + xw.shape[2], px:px + xw.shape[3]] = xw
    return _window_check(pad, ws, h, 1, 1, channels, THETA, LEAK, qws, quant)
