"""The allocation-free EMD loss entry point (evs_emd_loss_noalloc) against
evs_emd_loss with a caller workspace, through the C ABI: two calls in a row
(the second on a smaller input, so the static scratch still holds the first
call's partial sums), loss and gradient bit for bit; sizes beyond the static
scratch are refused on the host."""

import ctypes

import numpy as np
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


def _inputs(N, T, C, H, W, seed):
    rng = np.random.default_rng(seed)
    s = rng.choice(np.array([-1.0, 0.0, 1.0], np.float32), p=[0.2, 0.5, 0.3], size=(N, T, C, H, W))
    e = rng.integers(0, 3, size=(N, T, 2, H, W)).astype(np.int8)
    return torch.from_numpy(s).cuda(), torch.from_numpy(e).cuda()


def _noalloc(evs, s, e, lam):
    N, T, C, H, W = s.shape
    loss = torch.full((1,), float("nan"), device="cuda")
    g = torch.full_like(s, float("nan"))
    st = evs.lib().evs_emd_loss_noalloc(s.data_ptr(), e.data_ptr(), N, T, C, H, W, lam, loss.data_ptr(),
                                        g.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, loss, g


@pytest.mark.parametrize("C", [2, 1])
def test_noalloc_emd_equals_workspace_emd(evs, C):
    for shape, lam, seed in [((3, 40, C, 97, 131), 0.25, 1), ((1, 9, C, 13, 7), 0.0, 2)]:
        print(f"case emd noalloc {shape} lambda={lam}", flush=True)
        s, e = _inputs(*shape, seed)
        ref_loss, ref_g = evs.emd_loss(s, e, lambda_count=lam)
        st, loss, g = _noalloc(evs, s, e, lam)
        torch.cuda.synchronize()
        assert st == 0, evs.lib().evs_last_error()
        assert torch.equal(loss, ref_loss), (float(loss), float(ref_loss))
        assert torch.equal(g, ref_g)


def test_noalloc_emd_rejects_sizes_beyond_its_scratch(evs):
    s = ctypes.c_void_p(256)
    st = evs.lib().evs_emd_loss_noalloc(s, s, 64, 4, 2, 1024, 1024, 0.0, s, None, None)
    assert st == 3
    assert b"static scratch" in evs.lib().evs_last_error()
    st = evs.lib().evs_emd_loss_noalloc(None, s, 1, 4, 2, 8, 8, 0.0, s, None, None)
    assert st == 1
