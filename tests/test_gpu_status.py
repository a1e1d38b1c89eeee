"""The caller-owned device status word (include/evs.h, EVS_STATUS_*).

* evs_forward counts the NaN values of x (every pixel, channel and frame,
  the T+1 RGB frames of RGB-input nets, every clip of a batched launch) for
  every network form, on ragged frames whose edge tiles are partial; the
  NaN potentials that mask neurons outside the image are not counted, and
  passing the word changes no output.
* evs_backward counts NaN values of grad_s.
* evs_forward flags inputs beyond the fp16 split of FP32 nets with three
  input channels (|x| >= 65520 or infinite), and only for those nets.
* evs_compact_events flags a list cut at its capacity.
* Counts accumulate over calls and over graph replays; NULL records nothing.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from tests._helpers import f32, make_inputs  # noqa: E402

THETA, LEAK = f32(0.5), f32(0.9)


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


def _plant(x, n_nan, seed):
    """n_nan distinct NaN positions in x [N,T,C,H,W], the four frame corners
    and a row and column of the frame among them."""
    x = x.clone()
    N, T, C, H, W = x.shape
    rng = np.random.default_rng(seed)
    pos = {(0, 0, 0, 0, 0), (N - 1, T - 1, C - 1, H - 1, W - 1), (0, T // 2, 0, 0, W - 1), (N - 1, 0, C - 1, H - 1, 0)}
    while len(pos) < n_nan:
        pos.add(tuple(int(rng.integers(0, d)) for d in (N, T, C, H, W)))
    for p in pos:
        x[p] = float("nan")
    return x, len(pos)


@pytest.mark.parametrize("channels,prec,kw", [
    ((3, 16, 16, 2), "fp32", {}),                 # split FP32 input staging (headline net)
    ((3, 32, 2), "bf16", {}),                     # BF16 register staging
    ((3, 16, 16, 2), "bf16", {}),
    ((3, 32, 2), "fp32", {}),
    ((1, 16, 2), "fp32", {}),                     # DMA staging of one-channel FP32 nets
    ((3, 16, 2), "fp32", {"relaxed": True}),      # relaxed spikes: generic register staging
    ((3, 2), "fp32", {}),                         # single layer
])
def test_forward_counts_nan_inputs_once(evs, channels, prec, kw):
    N, T, H, W = 2, 5, 37, 53
    print(f"case status forward {channels} {prec} {kw}", flush=True)
    x, ws = make_inputs(channels, T, H, W, N=N, seed=1)
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec, **kw)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    st = evs.status_word()
    s_fp32 = bool(kw.get("relaxed"))
    evs.forward(net, packed, x.cuda(), status=st, s_fp32=s_fp32)
    torch.cuda.synchronize()
    assert st.tolist() == [0, 0, 0, 0], "clean input (and the masked neurons outside the image) counted"
    xn, n = _plant(x, 23, seed=len(channels))
    evs.forward(net, packed, xn.cuda(), status=st, s_fp32=s_fp32)
    torch.cuda.synchronize()
    assert st.tolist() == [n, 0, 0, 0]
    # counts accumulate; a NULL word records nothing and changes no output
    o1 = evs.forward(net, packed, xn.cuda(), status=st, s_fp32=s_fp32)["s"]
    o2 = evs.forward(net, packed, xn.cuda(), s_fp32=s_fp32)["s"]
    torch.cuda.synchronize()
    assert st.tolist() == [2 * n, 0, 0, 0]
    if s_fp32:                                    # NaN spikes of the smooth form compare by their bits
        o1, o2 = o1.view(torch.int32), o2.view(torch.int32)
    assert torch.equal(o1, o2)


@pytest.mark.parametrize("channels,prec,value,flagged", [
    ((3, 16, 16, 2), "fp32", 65504.0, False),     # largest fp16 value: inside the split's range
    ((3, 16, 16, 2), "fp32", -65519.0, False),    # rounds to -65504, still inside
    ((3, 16, 16, 2), "fp32", 65520.0, True),      # would round to infinity
    ((3, 32, 2), "fp32", float("-inf"), True),
    ((3, 32, 2), "bf16", 1e9, False),             # BF16 nets do not split x
    ((1, 16, 2), "fp32", 1e9, False),             # one-channel nets use the f32 matrix core
    ((3, 2), "fp32", 1e9, False),                 # no hidden layer: no split
    ((3, 8, 16, 2), "fp32", 1e9, False),          # layer by layer: FP32 multiply-adds, no split
])
def test_forward_flags_inputs_beyond_the_fp16_split(evs, channels, prec, value, flagged):
    print(f"case status range {channels} {prec} {value}", flush=True)
    x, ws = make_inputs(channels, 3, 21, 27, seed=5)
    x[0, 1, -1, 7, 11] = value
    net = evs.Net(channels, theta=THETA, leak=LEAK, precision=prec)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    st = evs.status_word()
    evs.forward(net, packed, x.cuda(), status=st)
    torch.cuda.synchronize()
    assert st.tolist() == [0, 0, evs._lib.EVS_FLAG_X_RANGE if flagged else 0, 0]


def test_forward_rgb_input_counts_every_frame(evs):
    """Nets fed RGB frames (Eq. 1 formed while staging) read T+1 frames of
    three colours: a NaN in any of them, frame 0 and frame T included, is
    counted once."""
    T, H, W = 6, 29, 41
    import synth
    rgb = synth.make_clip(synth.WORKLOADS["planes720"], T=T + 1, H=H, W=W)[None].contiguous()
    ws = synth.he_weights((1, 16, 2), 0)
    net = evs.Net((1, 16, 2), theta=THETA, leak=LEAK, input="rgb_logdiff")
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    st = evs.status_word()
    rgb_n, n = _plant(rgb, 11, seed=5)
    evs.forward(net, packed, rgb_n.cuda(), status=st)
    torch.cuda.synchronize()
    assert st.tolist() == [n, 0, 0, 0]


def test_batched_forward_counts_nan_inputs(evs):
    net = evs.Net((3, 32, 2), theta=THETA, leak=LEAK, precision="bf16")
    xs, outs, total = [], [], 0
    for i, (T, H, W) in enumerate([(6, 40, 70), (3, 33, 45), (5, 64, 64)]):
        x, ws = make_inputs((3, 32, 2), T, H, W, seed=2)
        x, n = _plant(x, 7 + i, seed=10 + i)
        xs.append(x.cuda())
        outs.append(torch.empty(1, T, 2, H, W, dtype=torch.int8, device="cuda"))
        total += n
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    st = evs.status_word()
    evs.forward_batched(net, packed, xs, outs, status=st)
    torch.cuda.synchronize()
    assert st.tolist() == [total, 0, 0, 0]


def test_backward_counts_nan_gradients(evs):
    channels = (3, 16, 16, 2)
    T, H, W = 8, 21, 27
    x, ws = make_inputs(channels, T, H, W, seed=3)
    net = evs.Net(channels, theta=THETA, leak=LEAK)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    xg = x.cuda()
    o = evs.forward(net, packed, xg, ckpt_every=3)
    G = torch.randn(1, T, 2, H, W, device="cuda")
    st = evs.status_word()
    evs.backward(net, packed, xg, o["ckpt"], 3, G, status=st)
    torch.cuda.synchronize()
    assert st.tolist() == [0, 0, 0, 0]
    G[0, 0, 0, 0, 0] = G[0, T - 1, 1, H - 1, W - 1] = G[0, 4, 1, 7, 9] = float("nan")
    evs.backward(net, packed, xg, o["ckpt"], 3, G, status=st)
    torch.cuda.synchronize()
    assert st.tolist() == [0, 3, 0, 0]


def test_compaction_flags_overflow(evs):
    rng = np.random.default_rng(8)
    s = torch.from_numpy(rng.choice(np.array([-1, 0, 1], np.int8), p=[0.2, 0.6, 0.2], size=(3, 2, 40, 50))).cuda()
    n = int(torch.count_nonzero(s))
    st = evs.status_word()
    evs.compact_events(s, capacity=n, status=st)
    torch.cuda.synchronize()
    assert st.tolist() == [0, 0, 0, 0]
    _, cnt = evs.compact_events(s, capacity=n - 1, status=st)
    torch.cuda.synchronize()
    assert int(cnt) == n and st.tolist() == [0, 0, 1, 0]


def test_status_word_under_graph_replay(evs):
    """Recorded in a graph, the forward adds its count on every replay."""
    channels = (3, 16, 16, 2)
    x, ws = make_inputs(channels, 4, 30, 30, seed=4)
    xn, n = _plant(x, 5, seed=4)
    net = evs.Net(channels, theta=THETA, leak=LEAK)
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    xg = xn.cuda()
    out = torch.empty(1, 4, 2, 30, 30, dtype=torch.int8, device="cuda")
    st = evs.status_word()
    stream = torch.cuda.Stream()
    g = evs.Graph(stream)
    with torch.cuda.stream(stream):
        with g.capture():
            evs.forward(net, packed, xg, out=out, status=st, stream=stream)
    torch.cuda.synchronize()
    assert st.tolist() == [0, 0, 0, 0]
    for k in range(1, 4):
        g.replay()
        torch.cuda.synchronize()
        assert st.tolist() == [k * n, 0, 0, 0]
