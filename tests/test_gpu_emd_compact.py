"""GPU parity of the EMD loss and of event compaction (through the C ABI).

EMD: loss and gradient against the FP64 oracle (Eq. 7-11); exact-valued
cases (hard spikes) to 1e-6 relative, continuous spikes to 1e-5.
Compaction: bit-exact event records in (t, c, y, x) order against numpy's
nonzero, including ragged frame sizes, empty input and a too-small buffer.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from oracle import emd  # noqa: E402


@pytest.fixture(scope="module")
def evs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_18071_amd as m
    m.lib()
    return m


def _emd_case(rng, N, T, C, H, W, hard, dens=0.2):
    if hard:
        s = rng.choice([-1.0, 0.0, 1.0], p=[dens / 2, 1 - dens, dens / 2], size=(N, T, C, H, W))
    else:
        s = rng.normal(0, 0.7, size=(N, T, C, H, W))
    e = rng.choice([0, 1, 2], p=[0.85, 0.12, 0.03], size=(N, T, 2, H, W)).astype(np.int8)
    return s.astype(np.float32), e


@pytest.mark.parametrize("C,hard,lam", [(2, True, 0.0), (2, True, 0.25), (1, True, 0.0), (1, True, 0.5),
                                        (2, False, 0.0), (2, False, 0.3), (1, False, 0.0)])
def test_emd_matches_oracle(evs, C, hard, lam):
    rng = np.random.default_rng(10 + C + 3 * hard)
    N, T, H, W = 2, 23, 9, 37
    s, e = _emd_case(rng, N, T, C, H, W, hard)
    loss, g = evs.emd_loss(torch.from_numpy(s).cuda(), torch.from_numpy(e).cuda(), lam)
    torch.cuda.synchronize()
    ref_l, ref_g = 0.0, np.zeros_like(s, dtype=np.float64)
    for n in range(N):
        l, gg = emd.loss_and_grad(s[n], e[n, :, 0], e[n, :, 1], lam)
        ref_l += l
        ref_g[n] = gg
    print(f"  C={C} hard={hard} lam={lam}: loss {float(loss):.6f} vs {ref_l:.6f}", flush=True)
    assert float(loss) == pytest.approx(ref_l, rel=1e-6)
    gd = g.cpu().numpy()
    tol = 1e-6 if hard else 1e-5
    np.testing.assert_allclose(gd, ref_g, rtol=tol, atol=tol)


def test_emd_training_size_and_determinism(evs):
    """The training workload's shape (4 x 64 x 2 x 256 x 256), twice: same bits."""
    rng = np.random.default_rng(7)
    s, e = _emd_case(rng, 4, 64, 2, 256, 256, True, dens=0.1)
    st, et = torch.from_numpy(s).cuda(), torch.from_numpy(e).cuda()
    l1, g1 = evs.emd_loss(st, et, 0.0)
    l2, g2 = evs.emd_loss(st, et, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    ref = sum(emd.loss_and_grad(s[n], e[n, :, 0], e[n, :, 1])[0] for n in range(4))
    assert float(l1) == pytest.approx(ref, rel=1e-6)
    # gradient on sampled pixels
    for (n, y, x) in [(0, 0, 0), (1, 100, 200), (3, 255, 255), (2, 17, 31)]:
        _, gg = emd.loss_and_grad(s[n][:, :, y:y + 1, x:x + 1], e[n, :, 0, y:y + 1, x:x + 1],
                                  e[n, :, 1, y:y + 1, x:x + 1])
        np.testing.assert_allclose(g1[n, :, :, y, x].cpu().numpy(), gg[:, :, 0, 0], rtol=1e-6, atol=1e-7)


def _expected_events(s):
    t, c, y, x = np.nonzero(s)
    v = s[t, c, y, x]
    return (t.astype(np.uint64) | (x.astype(np.uint64) << np.uint64(32)) | (y.astype(np.uint64) << np.uint64(44))
            | (c.astype(np.uint64) << np.uint64(56)) | ((v < 0).astype(np.uint64) << np.uint64(63)))


@pytest.mark.parametrize("T,C,H,W,dens", [(7, 2, 67, 131, 0.1), (3, 1, 128, 128, 0.5), (4, 2, 720, 1280, 0.05),
                                         (2, 2, 5, 3, 0.9), (1, 1, 1, 1, 1.0),
                                         # 1520 chunks: the offset scan's blocks of 1024 counts, two of them
                                         (40, 2, 480, 640, 0.02)])
def test_compaction_exact(evs, T, C, H, W, dens):
    rng = np.random.default_rng(T * 1000 + H)
    s = rng.choice(np.array([-1, 0, 1], np.int8), p=[dens / 2, 1 - dens, dens / 2], size=(T, C, H, W))
    ev, cnt = evs.compact_events(torch.from_numpy(s).cuda())
    torch.cuda.synchronize()
    exp = _expected_events(s)
    n = int(cnt)
    assert n == len(exp)
    got = ev[:n].cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, exp)


def test_compaction_empty_and_overflow(evs):
    s = np.zeros((3, 2, 40, 50), np.int8)
    ev, cnt = evs.compact_events(torch.from_numpy(s).cuda())
    torch.cuda.synchronize()
    assert int(cnt) == 0
    rng = np.random.default_rng(3)
    s = rng.choice(np.array([-1, 0, 1], np.int8), p=[0.2, 0.6, 0.2], size=(3, 2, 40, 50))
    exp = _expected_events(s)
    cap = len(exp) // 3
    ev, cnt = evs.compact_events(torch.from_numpy(s).cuda(), capacity=cap)
    torch.cuda.synchronize()
    assert int(cnt) == len(exp)
    np.testing.assert_array_equal(ev[:cap].cpu().numpy().view(np.uint64), exp[:cap])


def test_compaction_overflow_across_scan_blocks(evs):
    """A capacity that cuts the list inside the second block of chunk counts
    (3420 chunks: four blocks of the offset scan)."""
    rng = np.random.default_rng(11)
    s = rng.choice(np.array([-1, 0, 1], np.int8), p=[0.05, 0.9, 0.05], size=(30, 2, 720, 1280))
    exp = _expected_events(s)
    cap = (len(exp) * 3) // 8
    ev, cnt = evs.compact_events(torch.from_numpy(s).cuda(), capacity=cap)
    torch.cuda.synchronize()
    assert int(cnt) == len(exp)
    np.testing.assert_array_equal(ev[:cap].cpu().numpy().view(np.uint64), exp[:cap])


def test_compaction_of_forward_output(evs):
    """Events of a real forward pass: count equals the number of spikes."""
    from tests._helpers import make_inputs
    x, ws = make_inputs((3, 16, 16, 2), 6, 50, 70)
    net = evs.Net((3, 16, 16, 2))
    packed = evs.pack_weights(net, [torch.from_numpy(w).cuda() for w in ws])
    out = evs.forward(net, packed, x.cuda())
    ev, cnt = evs.compact_events(out["s"][0])
    torch.cuda.synchronize()
    s = out["s"][0].cpu().numpy()
    assert int(cnt) == int(np.count_nonzero(s))
    np.testing.assert_array_equal(ev[:int(cnt)].cpu().numpy().view(np.uint64), _expected_events(s))
