"""GPU checks of the batched persistent launch, hipGraph replay and the
tile autotuner (through the C ABI).

* One persistent launch over clips of uneven shape and length gives the
  same spikes and final membrane state, bit for bit, as one single-clip
  launch per clip.
* A captured sequence of time-window launches (state carried between
  windows) replays several times with eager work in between, and every
  replay equals the eager run bit for bit.
* The autotuner picks a compiled tile and the result does not change the
  spikes.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from tests._helpers import f32, make_inputs  # noqa: E402

THETA, LEAK = f32(0.5), f32(0.9)
SHAPES = [(7, 40, 50), (12, 64, 33), (3, 100, 120), (9, 24, 32), (1, 17, 200)]


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


def _net(evs, channels, prec):
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    _, ws = make_inputs(channels, 1, 4, 4, seed=2)
    return net, evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])


@pytest.mark.parametrize("channels,prec", [((3, 32, 2), "bf16"), ((3, 16, 16, 2), "fp32"), ((3, 8, 2), "fp32")])
def test_batched_equals_single_clip_launches(evs, channels, prec):
    net, packed = _net(evs, channels, prec)
    xs, outs, vs = [], [], []
    for i, (T, H, W) in enumerate(SHAPES):
        x, _ = make_inputs(channels, T, H, W, N=1 + (i % 2), y0=11 * i, x0=29 * i)
        xs.append(x.cuda())
        outs.append(torch.zeros(x.shape[0], T, 2, H, W, dtype=torch.int8, device="cuda"))
        vs.append(torch.zeros(x.shape[0], net.sum_c, H, W, device="cuda"))
    evs.forward_batched(net, packed, xs, outs, v_states=vs)
    torch.cuda.synchronize()
    for x, o, v in zip(xs, outs, vs):
        v1 = torch.zeros_like(v)
        ref = evs.forward(net, packed, x, v_state=v1)
        torch.cuda.synchronize()
        assert torch.equal(ref["s"], o)
        assert torch.equal(v1, v)


def test_graph_of_time_windows_replays_exactly(evs):
    channels, prec = (3, 32, 2), "bf16"
    net, packed = _net(evs, channels, prec)
    clips = [(20, 48, 64), (13, 30, 90)]
    win = 6
    xs = [make_inputs(channels, T, H, W, y0=5 * i)[0].cuda() for i, (T, H, W) in enumerate(clips)]
    outs = [torch.zeros(1, T, 2, H, W, dtype=torch.int8, device="cuda") for T, H, W in clips]
    vs = [torch.zeros(1, net.sum_c, H, W, device="cuda") for _, H, W in clips]
    stream = torch.cuda.Stream()
    ws = torch.empty(1 << 22, dtype=torch.uint8, device="cuda")

    def windows():
        for v in vs:
            v.zero_()
        for t0 in range(0, max(T for T, _, _ in clips), win):
            act = [i for i, (T, _, _) in enumerate(clips) if t0 < T]
            xw = [xs[i][:, t0:t0 + win] for i in act]
            ow = [outs[i][:, t0:t0 + win] for i in act]
            if len(act) == 1:
                evs.forward(net, packed, xw[0], v_state=vs[act[0]], out=ow[0], ws=ws)
            else:
                evs.forward_batched(net, packed, xw, ow, v_states=[vs[i] for i in act], ws=ws)

    # eager reference: every window's x/out slice must be contiguous for the ABI
    assert all(x[:, 0:win].is_contiguous() for x in xs)
    with torch.cuda.stream(stream):
        windows()
    torch.cuda.synchronize()
    ref_o = [o.clone() for o in outs]
    ref_v = [v.clone() for v in vs]
    g = evs.Graph(stream)
    with torch.cuda.stream(stream):
        with g.capture():
            windows()
    for rep in range(3):
        for o in outs:
            o.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref_o):
            assert torch.equal(o, r), f"replay {rep}"
        for v, r in zip(vs, ref_v):
            assert torch.equal(v, r), f"replay {rep}"
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()     # eager work between replays


def test_autotune_picks_a_tile_and_keeps_results(evs):
    channels = (3, 16, 16, 2)
    net, packed = _net(evs, channels, "fp32")
    x, _ = make_inputs(channels, 4, 70, 90)
    x = x.cuda()
    before = evs.forward(net, packed, x)["s"].clone()
    t = evs.autotune(net, 70, 90, T=4)
    assert 0 <= t < evs.tile_count(net)
    after = evs.forward(net, packed, x)["s"]
    torch.cuda.synchronize()
    assert torch.equal(before, after)
