"""Thin ctypes binding of libmlpg.so (include/mlpg.h), one function per C entry point.

Argument marshalling only: device arrays are torch tensors on the GPU (their
data pointers are passed straight through), host arrays are numpy arrays,
and every call runs on torch's current HIP stream.  All computation happens
in the HIP library; when the library is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlpg.so")

MLPG_FP64, MLPG_MIXED = 0, 1
MLPG_QUAD_PRODUCT, MLPG_QUAD_BEAM_DENSE = 0, 1
MLPG_OP_L, MLPG_OP_T, MLPG_OP_MS, MLPG_OP_SRC = 0, 1, 2, 3
MLPG_ACCEL_NONE, MLPG_ACCEL_DSA = 0, 1
MLPG_PRECOND_JACOBI, MLPG_PRECOND_PATCH = 0, 1
STATUS = {0: "MLPG_OK", -1: "MLPG_ERR_ARG", -2: "MLPG_ERR_HIP", -3: "MLPG_ERR_CAPACITY",
          -4: "MLPG_ERR_NOT_CONVERGED", -5: "MLPG_ERR_GEOMETRY", -6: "MLPG_ERR_WORKSPACE", -7: "MLPG_ERR_STATE"}

EXPORTS = ["mlpg_last_error", "mlpg_angular_quadrature", "mlpg_neighbors_count", "mlpg_neighbors_fill",
           "mlpg_geometry", "mlpg_get_info", "mlpg_get_volumes", "mlpg_cell_capacity", "mlpg_get_cells",
           "mlpg_boundary_points", "mlpg_integrate", "mlpg_get_pattern", "mlpg_get_blocks", "mlpg_assemble",
           "mlpg_apply", "mlpg_default_opts", "mlpg_set_state", "mlpg_get_state", "mlpg_solve",
           "mlpg_point_values", "mlpg_destroy", "mlpg_profile_begin", "mlpg_profile_end", "mlpg_set_progress",
           "mlpg_material_fields", "mlpg_update_points", "mlpg_refined_quadrature",
           "mlpg_material_shells", "mlpg_apply_patch_precond", "mlpg_geometry_workspace_bytes",
           "mlpg_integrate_workspace_bytes", "mlpg_assemble_workspace_bytes", "mlpg_solve_workspace_bytes",
           "mlpg_set_autotune", "mlpg_get_tuning", "mlpg_set_tuning", "mlpg_neighbors_static"]


class MlpgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int), ("n_mat", C.c_int), ("nnz", C.c_int64), ("n_bq", C.c_int64),
                ("oversize_cells", C.c_int64), ("failed_cells", C.c_int64), ("fallback_qps", C.c_int64),
                ("missing_pairs", C.c_int64), ("n_ord", C.c_int), ("n_blocks", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("tol_inner", C.c_double), ("tol_outer", C.c_double), ("restart_inner", C.c_int),
                ("restart_outer", C.c_int), ("max_inner", C.c_int), ("max_outer", C.c_int),
                ("check_every", C.c_int), ("tol_inner_lo", C.c_double), ("max_refine", C.c_int),
                ("accel", C.c_int), ("precond", C.c_int), ("graphs", C.c_int)]


class TuneEntry(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_ord", C.c_int), ("streams", C.c_int), ("value_bytes", C.c_int),
                ("form", C.c_int), ("waves_per_block", C.c_int), ("items_per_wave", C.c_int), ("rounds", C.c_int),
                ("xcd_split", C.c_int), ("threads", C.c_int), ("ords_per_lane", C.c_int), ("us_best", C.c_float),
                ("us_default", C.c_float)]


class SolveInfo(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_solves", C.c_int), ("inner_iters", C.c_int64),
                ("inner_sweeps", C.c_int64), ("outer_res", C.c_double), ("inner_res_max", C.c_double),
                ("converged", C.c_int), ("refinements", C.c_int), ("fp64_completions", C.c_int),
                ("accel_iters", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    """Load libmlpg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2008_02205_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.mlpg_last_error.restype = C.c_char_p
        L.mlpg_last_error.argtypes = []
        L.mlpg_angular_quadrature.argtypes = [i32, i32, i32, vp, vp]
        L.mlpg_neighbors_count.argtypes = [i32, i64, vp, vp, vp, C.POINTER(C.c_int64), vp]
        L.mlpg_neighbors_fill.argtypes = [i32, i64, vp, vp, vp, vp, vp]
        L.mlpg_neighbors_static.argtypes = [i32, i64, vp, vp, vp, vp, i64, C.POINTER(C.c_int64), vp]
        L.mlpg_geometry.argtypes = [C.POINTER(vp), i32, i64, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, C.c_size_t,
                                    vp]
        L.mlpg_geometry_workspace_bytes.restype = C.c_size_t
        L.mlpg_geometry_workspace_bytes.argtypes = [i32, i64, i64, vp, vp]
        L.mlpg_integrate_workspace_bytes.restype = C.c_size_t
        L.mlpg_integrate_workspace_bytes.argtypes = [vp, i32]
        L.mlpg_assemble_workspace_bytes.restype = C.c_size_t
        L.mlpg_assemble_workspace_bytes.argtypes = [vp, i32, i32]
        L.mlpg_solve_workspace_bytes.restype = C.c_size_t
        L.mlpg_solve_workspace_bytes.argtypes = [vp, C.POINTER(SolveOpts)]
        L.mlpg_get_info.argtypes = [vp, C.POINTER(Info)]
        L.mlpg_get_volumes.argtypes = [vp, vp, vp]
        L.mlpg_cell_capacity.argtypes = []
        L.mlpg_get_cells.argtypes = [vp, vp, vp, vp, vp]
        L.mlpg_boundary_points.argtypes = [vp, vp, vp, vp]
        L.mlpg_integrate.argtypes = [vp, i32, vp, C.c_size_t, vp]
        L.mlpg_material_fields.argtypes = [vp, i32, vp, vp]
        L.mlpg_material_shells.argtypes = [vp, i32, vp, vp, vp]
        L.mlpg_update_points.argtypes = [vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.mlpg_refined_quadrature.argtypes = [i32, i32, vp, vp, dbl, i32, vp, vp]
        L.mlpg_get_pattern.argtypes = [vp, vp, vp, vp]
        L.mlpg_get_blocks.argtypes = [vp, vp, vp, vp]
        L.mlpg_assemble.argtypes = [vp, i32, vp, vp, i32, vp, vp, dbl, vp, i32, vp, C.c_size_t, vp]
        L.mlpg_apply.argtypes = [vp, i32, vp, vp, vp]
        L.mlpg_apply_patch_precond.argtypes = [vp, vp, vp, C.POINTER(C.c_int64), vp, C.c_size_t, vp]
        L.mlpg_default_opts.restype = None
        L.mlpg_default_opts.argtypes = [C.POINTER(SolveOpts)]
        L.mlpg_set_state.argtypes = [vp, vp, vp]
        L.mlpg_get_state.argtypes = [vp, vp, vp, vp]
        L.mlpg_solve.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp, C.c_size_t,
                                 vp]
        L.mlpg_point_values.argtypes = [vp, vp, vp, vp]
        L.mlpg_destroy.restype = None
        L.mlpg_destroy.argtypes = [vp]
        L.mlpg_profile_begin.argtypes = []
        L.mlpg_profile_end.argtypes = [vp, vp, vp]
        L.mlpg_set_progress.argtypes = [PROGRESS_FN, vp]
        L.mlpg_set_autotune.argtypes = [i32]
        L.mlpg_get_tuning.argtypes = [i32, C.POINTER(TuneEntry)]
        L.mlpg_set_tuning.argtypes = [C.POINTER(TuneEntry)]
        for name in EXPORTS:
            if name not in ("mlpg_last_error", "mlpg_default_opts", "mlpg_destroy") and \
                    not name.endswith("_workspace_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise MlpgError(rc, lib().mlpg_last_error().decode())


def last_error() -> str:
    """Message of the last failing call on this thread (mlpg_last_error)."""
    return lib().mlpg_last_error().decode()


def _torch():
    import torch
    return torch


def _dev(t) -> Optional[int]:
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensor expected (contiguous, on the GPU)"
    return t.data_ptr()


def _host(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data


def _stream() -> int:
    torch = _torch()
    return torch.cuda.current_stream().cuda_stream


def _empty(shape, dtype=None):
    torch = _torch()
    return torch.empty(shape, dtype=dtype or torch.float64, device="cuda")


# ---------------------------------------------------------------------------

def mlpg_angular_quadrature(dim: int, n_ord: int, kind: int = MLPG_QUAD_PRODUCT):
    om = np.zeros((n_ord, dim))
    w = np.zeros(n_ord)
    _check(lib().mlpg_angular_quadrature(dim, n_ord, kind, _host(om), _host(w)))
    return om, w


def mlpg_neighbors_count(x, R):
    torch = _torch()
    n, dim = x.shape
    off = _empty(n + 1, torch.int64)
    total = C.c_int64(0)
    _check(lib().mlpg_neighbors_count(dim, n, _dev(x), _dev(R), _dev(off), C.byref(total), _stream()))
    return off, int(total.value)


def mlpg_neighbors_fill(x, R, off, total):
    torch = _torch()
    n, dim = x.shape
    idx = _empty(max(total, 1), torch.int32)
    _check(lib().mlpg_neighbors_fill(dim, n, _dev(x), _dev(R), _dev(off), _dev(idx), _stream()))
    return idx[:total]


def _ws(t):
    """(pointer, bytes) of a workspace tensor, or (None, 0) to let the library allocate."""
    if t is None:
        return None, 0
    return C.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def workspace(nbytes: int):
    """A device workspace of nbytes (torch-owned, 256-byte aligned by torch's allocator)."""
    torch = _torch()
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")
    assert t.data_ptr() % 256 == 0
    return t


def mlpg_geometry_workspace_bytes(dim, n, nnz_nbr, dom_lo, dom_hi) -> int:
    lo = np.ascontiguousarray(dom_lo, dtype=np.float64)
    hi = np.ascontiguousarray(dom_hi, dtype=np.float64)
    return int(lib().mlpg_geometry_workspace_bytes(dim, n, nnz_nbr, _host(lo), _host(hi)))


def mlpg_integrate_workspace_bytes(h, rk_order) -> int:
    return int(lib().mlpg_integrate_workspace_bytes(h, rk_order))


def mlpg_assemble_workspace_bytes(h, n_ord, precision) -> int:
    return int(lib().mlpg_assemble_workspace_bytes(h, n_ord, precision))


def mlpg_solve_workspace_bytes(h, opts=None) -> int:
    o = opts or mlpg_default_opts()
    return int(lib().mlpg_solve_workspace_bytes(h, C.byref(o)))


def mlpg_geometry(x, R, nbr_off, nbr_idx, dom_lo, dom_hi, regions=(), ws=None):
    n, dim = x.shape
    lo = np.ascontiguousarray(dom_lo, dtype=np.float64)
    hi = np.ascontiguousarray(dom_hi, dtype=np.float64)
    if regions:
        rlo = np.ascontiguousarray([r[0] for r in regions], dtype=np.float64)
        rhi = np.ascontiguousarray([r[1] for r in regions], dtype=np.float64)
        rmat = np.ascontiguousarray([r[2] for r in regions], dtype=np.int32)
    else:
        rlo = rhi = rmat = None
    h = C.c_void_p(None)
    idx = nbr_idx if nbr_idx.numel() > 0 else _empty(1, _torch().int32)
    wp, wb = _ws(ws)
    _check(lib().mlpg_geometry(C.byref(h), dim, n, _dev(x), _dev(R), _dev(nbr_off), _dev(idx), _host(lo), _host(hi),
                               len(regions), _host(rlo), _host(rhi), _host(rmat), wp, wb, _stream()))
    return h


def mlpg_material_fields(h, fields=()):
    """Smooth material fields ``(a, b, k, phase, material)`` (see the C declaration)."""
    if fields:
        par = np.ascontiguousarray([f[:4] for f in fields], dtype=np.float64)
        mat = np.ascontiguousarray([f[4] for f in fields], dtype=np.int32)
    else:
        par = mat = None
    _check(lib().mlpg_material_fields(h, len(fields), _host(par), _host(mat)))


def mlpg_refined_quadrature(min_level, goal_level, src, center, radius):
    """Alg. 2 refinement of the 2D product rule toward a disk seen from src (see the C declaration)."""
    s = np.ascontiguousarray(src, dtype=np.float64)
    c = np.ascontiguousarray(center, dtype=np.float64)
    n = lib().mlpg_refined_quadrature(min_level, goal_level, _host(s), _host(c), float(radius), 0, None, None)
    if n < 0:
        _check(n)
    om = np.zeros((n, 2))
    w = np.zeros(n)
    got = lib().mlpg_refined_quadrature(min_level, goal_level, _host(s), _host(c), float(radius), n, _host(om),
                                        _host(w))
    if got < 0:
        _check(got)
    return om, w


def mlpg_material_shells(h, shells=()):
    """Shells ``(centre, r_in, r_out, material)`` (see the C declaration)."""
    if shells:
        cen = np.ascontiguousarray([list(sh[0]) for sh in shells], dtype=np.float64)
        rad = np.ascontiguousarray([[sh[1], sh[2]] for sh in shells], dtype=np.float64)
        mat = np.ascontiguousarray([sh[3] for sh in shells], dtype=np.int32)
    else:
        cen = rad = mat = None
    _check(lib().mlpg_material_shells(h, len(shells), _host(cen), _host(rad), _host(mat)))


def mlpg_update_points(h, x, R, nbr_off, nbr_idx, ws=None):
    """New positions and radii for an existing handle (see the C declaration)."""
    idx = nbr_idx if nbr_idx.numel() > 0 else _empty(1, _torch().int32)
    wp, wb = _ws(ws)
    _check(lib().mlpg_update_points(h, _dev(x), _dev(R), _dev(nbr_off), _dev(idx), wp, wb, _stream()))


def mlpg_get_info(h) -> dict:
    info = Info()
    _check(lib().mlpg_get_info(h, C.byref(info)))
    return {k: getattr(info, k) for k, _ in Info._fields_}


def mlpg_get_volumes(h, n):
    V = _empty(n)
    _check(lib().mlpg_get_volumes(h, _dev(V), _stream()))
    return V


def mlpg_cell_capacity() -> int:
    return lib().mlpg_cell_capacity()


def mlpg_get_cells(h, n):
    torch = _torch()
    cap = mlpg_cell_capacity()
    nv = _empty(n, torch.int32)
    verts = _empty((n, cap, 2))
    tags = _empty((n, cap), torch.int32)
    _check(lib().mlpg_get_cells(h, _dev(nv), _dev(verts), _dev(tags), _stream()))
    return nv, verts, tags


def mlpg_boundary_points(h, n_bq, dim):
    torch = _torch()
    y = _empty((max(n_bq, 1), dim))
    face = _empty(max(n_bq, 1), torch.int32)
    _check(lib().mlpg_boundary_points(h, _dev(y), _dev(face), _stream()))
    return y[:n_bq], face[:n_bq]


def mlpg_integrate(h, rk_order: int, ws=None):
    wp, wb = _ws(ws)
    _check(lib().mlpg_integrate(h, rk_order, wp, wb, _stream()))


def mlpg_get_pattern(h, n, nnz):
    torch = _torch()
    row_off = _empty(n + 1, torch.int64)
    col = _empty(nnz, torch.int32)
    _check(lib().mlpg_get_pattern(h, _dev(row_off), _dev(col), _stream()))
    return row_off, col


def mlpg_get_blocks(h, n_blocks, nnz, want_E=True):
    blocks = _empty((n_blocks, nnz))
    E = _empty(nnz) if want_E else None
    _check(lib().mlpg_get_blocks(h, _dev(blocks), _dev(E) if want_E else None, _stream()))
    return blocks, E


def mlpg_assemble(h, omega: np.ndarray, w: np.ndarray, sigma_t, sigma_s, inv_c_dt: float, tau,
                  precision: int = MLPG_FP64, ws=None):
    om = np.ascontiguousarray(omega, dtype=np.float64)
    wq = np.ascontiguousarray(w, dtype=np.float64)
    st = np.ascontiguousarray(np.atleast_1d(sigma_t), dtype=np.float64)
    ss = np.ascontiguousarray(np.atleast_1d(sigma_s), dtype=np.float64)
    wp, wb = _ws(ws)
    _check(lib().mlpg_assemble(h, om.shape[0], _host(om), _host(wq), st.size, _host(st), _host(ss), float(inv_c_dt),
                               _dev(tau), precision, wp, wb, _stream()))


def mlpg_apply(h, which: int, X):
    Y = _empty(X.shape)
    _check(lib().mlpg_apply(h, which, _dev(X), _dev(Y), _stream()))
    return Y


def mlpg_apply_patch_precond(h, X, ws=None):
    """Y = M^-1 X with the patch block-Jacobi preconditioner; returns (Y, patch count)."""
    Y = _empty(X.shape)
    npt = C.c_int64(0)
    wp, wb = _ws(ws)
    _check(lib().mlpg_apply_patch_precond(h, _dev(X), _dev(Y), C.byref(npt), wp, wb, _stream()))
    return Y, npt.value


def mlpg_set_autotune(mode: int):
    """0: keep the built-in launch shape for new problem shapes; 1: measure (default); 2: empty the table."""
    _check(lib().mlpg_set_autotune(int(mode)))


def mlpg_get_tuning() -> list:
    """The launch shapes chosen so far: one dict per (n, n_ord, streams, value size)."""
    cnt = lib().mlpg_get_tuning(0, None)
    if cnt < 0:
        _check(cnt)
    arr = (TuneEntry * max(cnt, 1))()
    lib().mlpg_get_tuning(cnt, arr)
    return [{k: getattr(arr[i], k) for k, _ in TuneEntry._fields_} for i in range(cnt)]


def mlpg_set_tuning(entry: dict):
    """Inserts or replaces one launch-shape entry (a dict as returned by mlpg_get_tuning;
    missing keys default to 0, except us_best and us_default)."""
    e = TuneEntry()
    for k, _ in TuneEntry._fields_:
        setattr(e, k, entry.get(k, 0))
    _check(lib().mlpg_set_tuning(C.byref(e)))


def mlpg_default_opts() -> SolveOpts:
    o = SolveOpts()
    lib().mlpg_default_opts(C.byref(o))
    return o


def mlpg_set_state(h, psi):
    _check(lib().mlpg_set_state(h, _dev(psi), _stream()))


def mlpg_get_state(h, n, n_ord):
    psi = _empty((n, n_ord))
    phi = _empty(n)
    _check(lib().mlpg_get_state(h, _dev(psi), _dev(phi), _stream()))
    return psi, phi


def mlpg_solve(h, q, psi_b=None, opts: Optional[SolveOpts] = None, want_psi: bool = True, raise_on_error=True,
               ws=None):
    n, M = q.shape
    phi = _empty(n)
    phi_pt = _empty(n)
    psi = _empty((n, M)) if want_psi else None
    info = SolveInfo()
    o = opts or mlpg_default_opts()
    wp, wb = _ws(ws)
    rc = lib().mlpg_solve(h, _dev(q), _dev(psi_b), _dev(phi), _dev(phi_pt), _dev(psi), C.byref(o), C.byref(info),
                          wp, wb, _stream())
    if raise_on_error:
        _check(rc)
    d = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
    d["status"] = rc
    return phi, phi_pt, psi, d


def mlpg_point_values(h, coef):
    out = _empty(coef.shape[0])
    _check(lib().mlpg_point_values(h, _dev(coef), _dev(out), _stream()))
    return out


def mlpg_destroy(h):
    if h is not None and h.value:
        lib().mlpg_destroy(h)


PROF_CLASSES = ("spmv_L", "gs_pass_a", "gs_pass_b", "gs_cycle_end")


PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int, C.c_int64, C.c_double)
_progress_keep = None


def mlpg_set_progress(fn=None):
    """fn(level, iters, resid) after every batched Krylov solve (None: off)."""
    global _progress_keep
    cb = PROGRESS_FN(lambda _u, level, iters, resid: fn(level, iters, resid)) if fn else PROGRESS_FN()
    _progress_keep = cb
    _check(lib().mlpg_set_progress(cb, None))


def mlpg_profile_begin():
    _check(lib().mlpg_profile_begin())


def mlpg_profile_end() -> dict:
    ms = np.zeros(len(PROF_CLASSES))
    launches = np.zeros(len(PROF_CLASSES), dtype=np.int64)
    by = np.zeros(len(PROF_CLASSES))
    _check(lib().mlpg_profile_end(_host(ms), _host(launches), _host(by)))
    return {name: {"ms": float(ms[c]), "launches": int(launches[c]), "bytes": float(by[c])}
            for c, name in enumerate(PROF_CLASSES)}
