"""The BPTT backward at the full training-step size (4 crops x 64 frames x
256x256 of the 720p textured-planes clip, net 3->16->16->2, FP32 and BF16,
checkpoints every 16 frames), in the launch configuration bench.py times.

The FP64 oracle cannot run BPTT over 16.8 M pixel-frames in seconds (its
small-size parity is in test_gpu_backward.py), so the full-size run is held
to properties that hold at any size:
* weight and input gradients are bitwise reproducible (fixed-order sums);
* they do not depend on the checkpoint interval (every 16 vs every 64
  frames: rel. 1e-5);
* for hard spikes the backward is linear in the incoming gradient:
  dW(G1 + 2 G2) = dW(G1) + 2 dW(G2) to rel. 1e-5;
* they are finite, and the input-layer gradient is not zero.
"""

import pytest
import torch

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
        assert r < 1e-5
