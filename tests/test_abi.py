"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/mlpg.h declares, and rejects bad arguments on the host before any launch."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlpg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mlpg_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2008_02205_amd import mlpg
    if not os.path.exists(mlpg.LIB_PATH):
        pytest.skip("libmlpg.so not built")
    return mlpg.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    from paper_2008_02205_amd import mlpg
    assert sorted(mlpg.EXPORTS) == names


def test_host_argument_validation(lib):
    from paper_2008_02205_amd import mlpg
    h = C.c_void_p(None)
    lo = np.zeros(2); hi = np.ones(2)
    rc = lib.mlpg_geometry(C.byref(h), 4, 10, 1, 1, 1, 1, lo.ctypes.data, hi.ctypes.data, 0, None, None, None, None,
                           0, None)
    assert rc == -1 and b"dim" in lib.mlpg_last_error()
    rc = lib.mlpg_geometry(C.byref(h), 2, 0, 1, 1, 1, 1, lo.ctypes.data, hi.ctypes.data, 0, None, None, None, None,
                           0, None)
    assert rc == -1
    rc = lib.mlpg_geometry(C.byref(h), 2, 10, 1, 1, 1, 1, hi.ctypes.data, lo.ctypes.data, 0, None, None, None, None,
                           0, None)
    assert rc == -1 and b"empty domain" in lib.mlpg_last_error()
    assert lib.mlpg_integrate(None, 1, None, 0, None) == -1
    assert lib.mlpg_solve(None, None, None, None, None, None, None, None, None, 0, None) == -1
    assert lib.mlpg_integrate_workspace_bytes(None, 1) == 0
    assert lib.mlpg_assemble_workspace_bytes(None, 16, 0) == 0
    assert lib.mlpg_solve_workspace_bytes(None, None) == 0
    o = mlpg.SolveOpts()
    lib.mlpg_default_opts(C.byref(o))
    assert o.restart_inner == 30 and o.tol_inner == 1e-13
    lib.mlpg_destroy(None)


@pytest.mark.parametrize("dim,M,kind", [(2, 16, 0), (2, 64, 0), (3, 96, 0), (2, 256, 1)])
def test_angular_quadrature_host(lib, dim, M, kind):
    """Host-side rule of the library against the oracle's (numpy Gauss-Legendre)."""
    from paper_2008_02205_amd import mlpg
    om, w = mlpg.mlpg_angular_quadrature(dim, M, kind)
    om_o, w_o = oracle.angular_quadrature(dim, M, "product" if kind == 0 else "beam-dense")
    assert np.abs(om - om_o).max() <= 1e-14
    assert np.abs(w - w_o).max() <= 1e-14
    with pytest.raises(mlpg.MlpgError):
        mlpg.mlpg_angular_quadrature(2, 7)


def _aligned(b):
    return (b + 255) // 256 * 256


@pytest.mark.parametrize("dim,n,nnz", [(2, 16384, 766798), (3, 64000, 28536256), (2, 1, 0)])
def test_geometry_workspace_query_is_the_sum_of_its_buffers(lib, dim, n, nnz):
    """The geometry workspace is host-computable: every buffer the stage carves, 256-byte aligned."""
    from paper_2008_02205_amd import mlpg
    lo, hi = (0.0,) * dim, (1.0,) * dim
    got = mlpg.mlpg_geometry_workspace_bytes(dim, n, nnz, lo, hi)
    h = 2.0 * (1.0 / n) ** (1.0 / dim)
    ncell = int(np.ceil(1.0 / h)) ** dim
    d = dim
    sizes = [64 * d * 8, 64 * d * 8, 64 * 4, n * d * 8, n * 8, (n + 1) * 8, max(1, nnz) * 4, 4 * 8, n * 8, n * 8,
             (n + 1) * 8]
    if dim == 2:
        sizes += [n * 4, n * 32 * 4, n * 32 * 2 * 8]
    else:
        sizes += [n * 4, n * 40 * 4, n * 40 * 4, n * 40 * 16 * 3 * 8]
    sizes += [(n + 1) * 8, (nnz + n) * 4, n * 8, (n + 1) * 8, (n + 1) * 8, n * 4,
              n * 4, n * 8, n * 8, n * 8, ncell * 8, (ncell + 1) * 8, (ncell + 1) * 8, ncell * 8]
    assert got == sum(_aligned(b) for b in sizes)
    assert mlpg.mlpg_geometry_workspace_bytes(dim, n, nnz, hi, lo) == 0
    assert mlpg.mlpg_geometry_workspace_bytes(4, n, nnz, lo, hi) == 0


def test_tuning_table_entries_round_trip_and_are_validated(lib):
    """mlpg_set_tuning stores an entry under its key (replacing an older one) and
    rejects shapes outside the documented ranges; host only."""
    from paper_2008_02205_amd import mlpg
    mlpg.mlpg_set_autotune(2)
    try:
        base = dict(n=777, n_ord=64, streams=6, value_bytes=8, xcd_split=8)
        mlpg.mlpg_set_tuning(dict(base, form=0, waves_per_block=2, items_per_wave=2, us_best=1.5))
        mlpg.mlpg_set_tuning(dict(base, form=1, waves_per_block=8, rounds=3, us_best=2.5))
        t = [e for e in mlpg.mlpg_get_tuning() if e["n"] == 777]
        assert len(t) == 1
        t = t[0]
        assert (t["form"], t["waves_per_block"], t["rounds"], t["threads"]) == (1, 8, 3, 512)
        assert t["us_best"] == 2.5
        mlpg.mlpg_set_tuning(dict(n=777, n_ord=16, streams=3, value_bytes=4, threads=256))
        small = [e for e in mlpg.mlpg_get_tuning() if e["n_ord"] == 16]
        assert small[0]["threads"] == 256 and small[0]["form"] == 0
        wide = dict(n=777, n_ord=96, streams=10, value_bytes=8, xcd_split=1)
        mlpg.mlpg_set_tuning(dict(wide, form=2, waves_per_block=4, items_per_wave=1, ords_per_lane=2))
        t = [e for e in mlpg.mlpg_get_tuning() if e["n_ord"] == 96][0]
        assert (t["form"], t["ords_per_lane"], t["waves_per_block"], t["xcd_split"]) == (2, 2, 4, 1)
        mlpg.mlpg_set_tuning(t)   # an entry read back is accepted as it is
        assert [e for e in mlpg.mlpg_get_tuning() if e["n_ord"] == 96] == [t]
        bad = [dict(base, form=1, waves_per_block=2, rounds=2),           # form 1 needs 4 or 8 waves
               dict(base, form=1, waves_per_block=4, rounds=0),           # rounds >= 1
               dict(base, n_ord=96, form=1, waves_per_block=4, rounds=2),  # form 1 needs <= 64 ordinates
               dict(base, streams=3, form=1, waves_per_block=4, rounds=2),
               dict(base, form=2, waves_per_block=4),
               dict(base, form=2, waves_per_block=4, items_per_wave=1, ords_per_lane=2),   # 64 ordinates: no gain
               dict(wide, form=2, waves_per_block=4, items_per_wave=1, ords_per_lane=4),   # 96 / 4 not fewer items
               dict(wide, form=2, waves_per_block=4, items_per_wave=1, ords_per_lane=3),
               dict(wide, streams=4, form=2, waves_per_block=4, items_per_wave=1, ords_per_lane=2),
               dict(base, form=3, waves_per_block=4, items_per_wave=1),
               dict(base, form=0, waves_per_block=16, items_per_wave=1),
               dict(base, form=0, waves_per_block=4, items_per_wave=1, xcd_split=4),
               dict(base, streams=5, form=0, waves_per_block=4, items_per_wave=1),
               dict(n=777, n_ord=16, streams=3, value_bytes=4, threads=8),
               dict(n=0, n_ord=64, streams=6, value_bytes=8, form=0, waves_per_block=4, items_per_wave=1,
                    xcd_split=8)]
        for b in bad:
            with pytest.raises(mlpg.MlpgError):
                mlpg.mlpg_set_tuning(b)
        assert len([e for e in mlpg.mlpg_get_tuning() if e["n"] == 777]) == 3
    finally:
        mlpg.mlpg_set_autotune(2)
