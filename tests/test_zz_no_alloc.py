"""The allocation-free overlap-list entry point (mlpg_neighbors_static) against the allocating ones.

Called through the C ABI twice in a row -- a 3D lattice, then a smaller 2D
Poisson-disk set -- its offsets and lists must equal those of
mlpg_neighbors_count / mlpg_neighbors_fill bit for bit (integer output), as
well as the oracle's brute-force lists; sizes beyond the static scratch and a
list capacity that is too small are refused.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02205_amd import mlpg
    return mlpg.lib()


def _static(L, x, R, cap):
    n, dim = x.shape
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    tot = C.c_int64(-1)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.mlpg_neighbors_static(dim, n, C.c_void_p(x.data_ptr()), C.c_void_p(R.data_ptr()),
                                 C.c_void_p(off.data_ptr()), C.c_void_p(idx.data_ptr()), cap, C.byref(tot), stream)
    torch.cuda.synchronize()
    return rc, tot.value, off, idx


def _check_case(L, x_np, R_np):
    from paper_2008_02205_amd import mlpg
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    R = torch.from_numpy(np.ascontiguousarray(R_np)).cuda()
    off_ref, total = mlpg.mlpg_neighbors_count(x, R)
    idx_ref = mlpg.mlpg_neighbors_fill(x, R, off_ref, total)
    rc, tot, off, idx = _static(L, x, R, int(total))
    assert rc == 0 and tot == total
    assert torch.equal(off, off_ref)
    assert torch.equal(idx[:total], idx_ref)
    o_or, i_or = oracle.neighbors(x_np, R_np)
    assert np.array_equal(off.cpu().numpy(), o_or) and np.array_equal(idx[:total].cpu().numpy(), i_or)
    return total


def test_static_scratch_lists_equal_the_allocating_entry_points(lib):
    x, dx = W.jittered_lattice((20, 20, 20), (0, 0, 0), (1, 1, 1), 0.2, 31)
    print(f"[case] no-alloc 3D lattice n={x.shape[0]}", flush=True)
    t1 = _check_case(lib, x, np.full(x.shape[0], 2.5 * dx))
    # a second, smaller call on the same scratch (its earlier contents must not leak)
    x2 = W.poisson_disk((0, 0), (2, 1), 0.03, 32)
    print(f"[case] no-alloc 2D Poisson disk n={x2.shape[0]}", flush=True)
    t2 = _check_case(lib, x2, np.full(x2.shape[0], 0.05))
    assert 0 < t2 < t1


def test_static_limits(lib):
    x = torch.rand((100, 2), dtype=torch.float64, device="cuda")
    R = torch.full((100,), 0.2, dtype=torch.float64, device="cuda")
    rc, tot, _, _ = _static(lib, x, R, 10)
    assert rc == -3 and tot > 10          # capacity too small: the count comes back
    rc, tot, off, idx = _static(lib, x, R, tot)
    assert rc == 0
    big = torch.zeros(((1 << 20) + 1, 2), dtype=torch.float64, device="cuda")
    Rb = torch.full(((1 << 20) + 1,), 0.1, dtype=torch.float64, device="cuda")
    rc, _, _, _ = _static(lib, big, Rb, 0)
    assert rc == -1
