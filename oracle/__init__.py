"""Plain FP64 CPU oracle of the MLPG discrete-ordinates transport path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares
no code with the HIP library: its own neighbour search, clipping, quadrature
rules (from numpy/scipy Gauss rules), RK evaluation, sparse storage and
Krylov solvers, in ``mlpg_oracle.c`` plus the orchestration below.

Paper: Bassett & Owen, "Meshless discretization of the discrete-ordinates
transport equation with integration based on Voronoi cells" (arXiv 2008.02205).
Parity status of every function is recorded in the tests that pin it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mlpg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class IntegCtx(C.Structure):
    _fields_ = [("dim", C.c_int), ("rk_order", C.c_int), ("n_mat", C.c_int), ("n", C.c_int64),
                ("x", _dp), ("R", _dp), ("V", _dp), ("nb_off", _i64p), ("nb_idx", _i32p),
                ("row_off", _i64p), ("col", _i32p), ("nnz", C.c_int64), ("n_regions", C.c_int),
                ("reg_lo", _dp), ("reg_hi", _dp), ("reg_mat", _i32p), ("blocks", _dp),
                ("fallbacks", C.c_int64), ("missing", C.c_int64), ("n_fields", C.c_int),
                ("field_par", _dp), ("field_mat", _i32p), ("n_shells", C.c_int), ("shell_par", _dp),
                ("shell_mat", _i32p)]


class OpCtx(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_mat", C.c_int), ("n_ord", C.c_int), ("n", C.c_int64),
                ("nnz", C.c_int64), ("row_off", _i64p), ("col", _i32p), ("blocks", _dp),
                ("omega", _dp), ("wq", _dp), ("sig_t", _dp), ("sig_s", _dp), ("a0", C.c_double),
                ("tau", _dp), ("nbq", C.c_int64), ("kmax", C.c_int), ("bq_face", _i32p),
                ("bq_w", _dp), ("bq_nact", _i32p), ("bq_act", _i32p), ("bq_N", _dp),
                ("tol_in", C.c_double), ("tol_out", C.c_double), ("restart_in", C.c_int),
                ("restart_out", C.c_int), ("max_in", C.c_int), ("max_out", C.c_int),
                ("precond", C.c_int), ("x", _dp), ("dom_lo", _dp), ("dom_hi", _dp)]


def _declare(L):
    L.orc_neighbors_count.restype = C.c_int64
    L.orc_neighbors_count.argtypes = [C.c_int, C.c_int64, _dp, _dp, _i64p]
    L.orc_neighbors_fill.restype = None
    L.orc_neighbors_fill.argtypes = [C.c_int, C.c_int64, _dp, _dp, _i64p, _i32p]
    L.orc_cells2d.restype = C.c_int64
    L.orc_cells2d.argtypes = [C.c_int64, _dp, _dp, _i64p, _i32p, _dp, _dp, C.c_int, _i32p, _dp, _i32p,
                              _dp, _dp]
    L.orc_cells3d.restype = C.c_int64
    L.orc_cells3d.argtypes = [C.c_int64, _dp, _dp, _i64p, _i32p, _dp, _dp, C.c_int64, _i64p, C.c_int, C.c_int,
                              _i32p, _i32p, _dp, _i32p, _dp, _dp]
    L.orc_integrate3d.restype = C.c_int64
    L.orc_integrate3d.argtypes = [C.POINTER(IntegCtx), C.c_int, C.c_int, _i32p, _i32p, _dp, _i32p, C.c_int, _dp,
                                  _dp, C.c_int, _dp, _dp, _dp, C.c_int64, C.c_int, _dp, _i32p, _dp, _i32p,
                                  _i32p, _dp, _i64p]
    L.orc_rk_eval.restype = C.c_int
    L.orc_rk_eval.argtypes = [C.c_int, C.c_int, _dp, C.c_int, _i32p, _dp, _dp, _dp, C.c_double, _dp, _dp]
    L.orc_num_blocks.restype = C.c_int
    L.orc_num_blocks.argtypes = [C.c_int, C.c_int]
    L.orc_integrate2d.restype = C.c_int64
    L.orc_integrate2d.argtypes = [C.POINTER(IntegCtx), C.c_int, _i32p, _dp, _i32p, C.c_int, _dp, _dp,
                                  C.c_int, _dp, _dp, _dp, C.c_int64, C.c_int, _dp, _i32p, _dp, _i32p,
                                  _i32p, _dp, _i64p]
    L.orc_step.restype = C.c_int
    L.orc_step.argtypes = [C.POINTER(OpCtx), _dp, _dp, _dp, _dp, _dp, _dp, _i64p, _dp]
    L.orc_step_source_iteration.restype = C.c_int
    L.orc_step_source_iteration.argtypes = [C.POINTER(OpCtx), _dp, _dp, _dp, C.c_int, _dp, _dp]
    L.orc_apply.restype = None
    L.orc_apply.argtypes = [C.POINTER(OpCtx), C.c_int, _dp, _dp]
    L.orc_rhs.restype = None
    L.orc_rhs.argtypes = [C.POINTER(OpCtx), _dp, _dp, _dp, _dp]
    L.orc_point_values.restype = None
    L.orc_point_values.argtypes = [C.c_int64, _i64p, _i32p, _dp, _dp, C.c_int, _dp]
    L.orc_Linv_range.restype = C.c_int64
    L.orc_Linv_range.argtypes = [C.POINTER(OpCtx), _dp, _dp, C.c_int, C.c_int, _dp]
    L.orc_patches_of.restype = C.c_int64
    L.orc_patches_of.argtypes = [C.POINTER(OpCtx), _i64p, _i32p]
    L.orc_patch_precond.restype = None
    L.orc_patch_precond.argtypes = [C.POINTER(OpCtx), C.c_int, _dp, _dp]
    L.orc_num_threads.restype = C.c_int
    L.orc_num_threads.argtypes = []


def _p(a, t=_dp):
    if a is None:
        return C.cast(None, t)
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


# ---------------------------------------------------------------------------
# Quadrature rules (Sec. 3.2, Sec. 5 rule choices; App. A reference elements)
# ---------------------------------------------------------------------------

def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _gj01(n, alpha):
    """Gauss-Jacobi nodes/weights on [0,1] for the weight (1-u)^alpha."""
    from scipy.special import roots_jacobi
    x, w = roots_jacobi(n, alpha, 0.0)
    return 0.5 * (x + 1.0), w / 2.0 ** (alpha + 1)


def segment_rule(n: int = 5):
    """Gauss-Legendre on the reference line [-1, 1] (App. A)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x.copy(), w.copy()


def triangle_rule(n: int = 5):
    """Conical-product rule on {xi >= 0, xi0 + xi1 <= 1}: n*n points, exact to degree 2n-1.

    The collapsed map (u, v) -> (u, (1-u) v) has Jacobian (1-u), absorbed by a
    Gauss-Jacobi rule in u; weights sum to the reference area 1/2."""
    u, wu = _gj01(n, 1.0)
    v, wv = _gl01(n)
    pts = np.array([[ui, (1.0 - ui) * vj] for ui in u for vj in v])
    wts = np.array([a * b for a in wu for b in wv])
    return pts, wts


def tet_rule(n: int = 2):
    """Conical-product rule on the reference tetrahedron: n^3 points, exact to degree 2n-1."""
    u, wu = _gj01(n, 2.0)
    v, wv = _gj01(n, 1.0)
    s, ws = _gl01(n)
    pts, wts = [], []
    for a, ua in enumerate(u):
        for b, vb in enumerate(v):
            for c, sc in enumerate(s):
                pts.append([ua, (1 - ua) * vb, (1 - ua) * (1 - vb) * sc])
                wts.append(wu[a] * wv[b] * ws[c])
    return np.array(pts), np.array(wts)


def refined_quadrature(min_level: int, goal_level: int, src, center, radius: float):
    """Angular refinement of Alg. 2 (Sec. 4.3) on the 2D product rule's azimuthal hierarchy.

    Rule L has 4 * 2^L equal azimuthal sectors per polar level (midpoint
    ordinates, the polar levels of the 2D product rule).  Following Alg. 2:
    start from the goal rule; for every rule from min_level up to the one
    below the goal, add each of its ordinates whose goal ordinates are all
    still present and none of which hits the object, removing those goal
    ordinates; finally add the goal ordinates that remain.  An ordinate hits
    when its azimuth lies within asin(radius / distance) of the direction
    from src to the disk centre (always, when src is inside the disk).
    Returned in the order polar level, then sector start angle.
    """
    xg, wg = np.polynomial.legendre.leggauss(4)
    pos = xg > 0
    xi, wp = xg[pos], wg[pos]
    dx, dy = center[0] - src[0], center[1] - src[1]
    dist = math.hypot(dx, dy)
    inside = dist <= radius
    half = math.asin(radius / dist) if not inside else math.pi
    aim = math.atan2(dy, dx)

    def hits(phi):
        if inside:
            return True
        dphi = (phi - aim + math.pi) % (2.0 * math.pi) - math.pi
        return abs(dphi) <= half

    ng = 4 * 2 ** goal_level
    goal_hit = [hits(2.0 * math.pi * (c + 0.5) / ng) for c in range(ng)]
    picked = []                         # (polar level, rule, sector)
    for p in range(2):
        present = [True] * ng
        for rule in range(min_level, goal_level):
            na = 4 * 2 ** rule
            span = ng // na
            for k in range(na):
                kids = range(k * span, (k + 1) * span)
                if all(present[c] for c in kids) and not any(goal_hit[c] for c in kids):
                    picked.append((p, rule, k))
                    for c in kids:
                        present[c] = False
        picked += [(p, goal_level, c) for c in range(ng) if present[c]]
    picked.sort(key=lambda e: (e[0], e[2] / (4 * 2 ** e[1])))
    om, w = [], []
    for p, rule, k in picked:
        na = 4 * 2 ** rule
        st = math.sqrt(1.0 - xi[p] ** 2)
        ph = (2.0 * (k + 1) - 1.0) * np.pi / na
        om.append([st * math.cos(ph), st * math.sin(ph)])
        w.append(2.0 * wp[p] * 2.0 * np.pi / na)
    return np.array(om), np.array(w)


def angular_quadrature(dim: int, n_ord: int, kind: str = "product"):
    """Ordinates Omega_m and weights w_m with sum w = 4 pi (Sec. 4.1).

    2D "product": two polar levels (positive roots of the 4-point
    Gauss-Legendre rule) times n_ord/2 equally spaced azimuths
    phi_k = (2k-1) pi / N_a; the weight doubles for the folded lower
    hemisphere.  3D "product": 6-point Gauss-Legendre in Omega_z times
    n_ord/6 azimuths.  2D "beam-dense": two polar levels times 128 azimuthal
    sectors, 41 of them uniformly inside |phi| <= 10 degrees and 87 over the
    remaining 340 degrees, ordinates at sector midpoints.
    Order: polar level outer (increasing cosine), azimuth inner (increasing angle).
    """
    if dim == 2 and kind == "product":
        xg, wg = np.polynomial.legendre.leggauss(4)
        pos = xg > 0
        xi, wp = xg[pos], wg[pos]
        na = n_ord // 2
        assert 2 * na == n_ord
        phis = (2.0 * np.arange(1, na + 1) - 1.0) * np.pi / na
        om, w = [], []
        for p in range(2):
            st = math.sqrt(1.0 - xi[p] ** 2)
            for ph in phis:
                om.append([st * math.cos(ph), st * math.sin(ph)])
                w.append(2.0 * wp[p] * 2.0 * np.pi / na)
        return np.array(om), np.array(w)
    if dim == 2 and kind == "beam-dense":
        xg, wg = np.polynomial.legendre.leggauss(4)
        pos = xg > 0
        xi, wp = xg[pos], wg[pos]
        win = math.radians(10.0)
        edges = list(np.linspace(-win, win, 42)) + list(np.linspace(win, 2 * np.pi - win, 88)[1:])
        edges = np.array(edges)
        mids = 0.5 * (edges[:-1] + edges[1:])
        dph = edges[1:] - edges[:-1]
        assert mids.size == n_ord // 2
        om, w = [], []
        for p in range(2):
            st = math.sqrt(1.0 - xi[p] ** 2)
            for ph, d in zip(mids, dph):
                om.append([st * math.cos(ph), st * math.sin(ph)])
                w.append(2.0 * wp[p] * d)
        return np.array(om), np.array(w)
    if dim == 3 and kind == "product":
        xg, wg = np.polynomial.legendre.leggauss(6)
        na = n_ord // 6
        assert 6 * na == n_ord
        phis = (2.0 * np.arange(1, na + 1) - 1.0) * np.pi / na
        om, w = [], []
        for p in range(6):
            st = math.sqrt(1.0 - xg[p] ** 2)
            for ph in phis:
                om.append([st * math.cos(ph), st * math.sin(ph), xg[p]])
                w.append(wg[p] * 2.0 * np.pi / na)
        return np.array(om), np.array(w)
    raise ValueError((dim, kind))


# ---------------------------------------------------------------------------
# Geometry and integration
# ---------------------------------------------------------------------------

def neighbors(x: np.ndarray, R: np.ndarray):
    """Overlap lists |x_i - x_j| <= R_i + R_j, j != i, increasing j (Sec. 3.4)."""
    x = _f64(x); R = _f64(R)
    n, d = x.shape
    off = np.zeros(n + 1, dtype=np.int64)
    tot = lib().orc_neighbors_count(d, n, _p(x), _p(R), _p(off, _i64p))
    idx = np.zeros(max(tot, 1), dtype=np.int32)
    lib().orc_neighbors_fill(d, n, _p(x), _p(R), _p(off, _i64p), _p(idx, _i32p))
    return off, idx[:tot]


def pattern(n: int, off: np.ndarray, idx: np.ndarray):
    """Row i of the sparse pattern: {i} and its overlap neighbours, sorted."""
    rows = []
    counts = np.diff(off) + 1
    row_off = np.zeros(n + 1, dtype=np.int64)
    row_off[1:] = np.cumsum(counts)
    col = np.empty(row_off[-1], dtype=np.int32)
    for i in range(n):
        c = np.concatenate(([i], idx[off[i]:off[i + 1]]))
        c.sort()
        col[row_off[i]:row_off[i + 1]] = c
    del rows
    return row_off, col


@dataclass
class Cells2D:
    nv: np.ndarray
    verts: np.ndarray   # [n][cap][2]
    tags: np.ndarray    # [n][cap]
    V: np.ndarray
    rho: np.ndarray
    failed: int
    cap: int


def cells2d(x, R, off, idx, dom_lo, dom_hi, cap: int = 64) -> Cells2D:
    x = _f64(x); R = _f64(R)
    n = x.shape[0]
    nv = np.zeros(n, dtype=np.int32)
    verts = np.zeros((n, cap, 2))
    tags = np.zeros((n, cap), dtype=np.int32)
    V = np.zeros(n); rho = np.zeros(n)
    lo = _f64(dom_lo); hi = _f64(dom_hi)
    bad = lib().orc_cells2d(n, _p(x), _p(R), _p(off, _i64p), _p(idx, _i32p), _p(lo), _p(hi), cap,
                            _p(nv, _i32p), _p(verts), _p(tags, _i32p), _p(V), _p(rho))
    return Cells2D(nv, verts, tags, V, rho, int(bad), cap)


@dataclass
class Cells3D:
    nf: np.ndarray       # [m] faces per cell
    fnv: np.ndarray      # [m][fcap] vertices per face
    fverts: np.ndarray   # [m][fcap][vcap][3], counter-clockwise seen from outside
    ftags: np.ndarray    # [m][fcap]
    V: np.ndarray
    rho: np.ndarray
    failed: int
    fcap: int
    vcap: int


def cells3d(x, R, off, idx, dom_lo, dom_hi, ids=None, fcap: int = 64, vcap: int = 32) -> Cells3D:
    """3D cells (Sec. 3.1) of the points ``ids`` (all points by default)."""
    x = _f64(x); R = _f64(R)
    n = x.shape[0]
    ids_a = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
    m = n if ids_a is None else ids_a.size
    nf = np.zeros(m, dtype=np.int32)
    fnv = np.zeros((m, fcap), dtype=np.int32)
    fverts = np.zeros((m, fcap, vcap, 3))
    ftags = np.zeros((m, fcap), dtype=np.int32)
    V = np.zeros(m); rho = np.zeros(m)
    bad = lib().orc_cells3d(n, _p(x), _p(R), _p(off, _i64p), _p(idx, _i32p), _p(_f64(dom_lo)), _p(_f64(dom_hi)),
                            m, _p(ids_a, _i64p), fcap, vcap, _p(nf, _i32p), _p(fnv, _i32p), _p(fverts),
                            _p(ftags, _i32p), _p(V), _p(rho))
    return Cells3D(nf, fnv, fverts, ftags, V, rho, int(bad), fcap, vcap)


def num_blocks(dim: int, n_mat: int) -> int:
    return n_mat * (1 + dim) + dim * dim + 2 * dim


def block_names(dim: int, n_mat: int):
    ax = "xyz"
    names = []
    for g in range(n_mat):
        names.append(f"mass{g}")
        names += [f"d{ax[a]}{g}" for a in range(dim)]
    names += [f"k{ax[a]}{ax[b]}" for a in range(dim) for b in range(dim)]
    names += [f"s{f}" for f in range(2 * dim)]
    return names


def rk_eval(x, R, V, y, cand, order, hs):
    """RK values N_j(y) = V_j U_j(y) and gradients for candidates ``cand`` (Sec. 2.2)."""
    x = _f64(x); R = _f64(R); V = _f64(V); y = _f64(y)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    d = x.shape[1]
    N = np.zeros(cand.size); dN = np.zeros((cand.size, d))
    used = lib().orc_rk_eval(d, order, _p(y), cand.size, _p(cand, _i32p), _p(x), _p(R), _p(V), hs,
                             _p(N), _p(dN))
    return N, dN, used


@dataclass
class Geometry:
    dim: int
    x: np.ndarray
    R: np.ndarray
    dom_lo: np.ndarray
    dom_hi: np.ndarray
    nb_off: np.ndarray
    nb_idx: np.ndarray
    cells: object            # Cells2D or Cells3D
    row_off: np.ndarray = None
    col: np.ndarray = None

    @property
    def n(self):
        return self.x.shape[0]

    @property
    def V(self):
        return self.cells.V


def geometry(x, R, dom_lo, dom_hi) -> Geometry:
    x = _f64(x); R = _f64(R)
    off, idx = neighbors(x, R)
    if x.shape[1] == 2:
        cl = cells2d(x, R, off, idx, dom_lo, dom_hi)
    else:
        cl = cells3d(x, R, off, idx, dom_lo, dom_hi)
    g = Geometry(x.shape[1], x, R, _f64(dom_lo), _f64(dom_hi), off, idx, cl)
    g.row_off, g.col = pattern(g.n, off, idx)
    return g


@dataclass
class Integrated:
    geom: Geometry
    rk_order: int
    n_mat: int
    blocks: np.ndarray      # [nblk][nnz]
    E: np.ndarray           # [nnz]
    bq_y: np.ndarray
    bq_face: np.ndarray
    bq_w: np.ndarray
    bq_nact: np.ndarray
    bq_act: np.ndarray
    bq_N: np.ndarray
    kmax: int
    fallbacks: int
    missing: int

    def block(self, name: str) -> np.ndarray:
        return self.blocks[block_names(self.geom.dim, self.n_mat).index(name)]

    @property
    def nbq(self):
        return self.bq_y.shape[0]


def integrate(g: Geometry, rk_order: int, regions=(), n_mat: int = 1, tri_n: int = None, seg_n: int = 5,
              kmax: int = None, tet_n: int = 2, fields=(), shells=()) -> Integrated:
    """Blocks of Alg. 1 over all cells; boundary quadrature points; point-value matrix E.

    Rules: 2D, triangle rule n = 5 (25 points) in the cells and line rule
    seg_n on domain edges; 3D, tetrahedron rule n = 2 (8 points) in the
    cells and triangle rule n = 2 (4 points) on domain faces.

    ``regions``: boxes ``(lo, hi, material)`` (last match wins, material 0
    elsewhere).  ``fields``: smooth material fractions ``(a, b, k, phase,
    material)``; each moves ``a + b prod_alpha cos(k y_alpha + phase)`` of the
    quadrature point's weight from material 0 to ``material`` (the spatially
    varying opacities of Sec. 5.1 are sums of such terms).  ``shells``:
    ``(centre, r_in, r_out, material)``, applied after the boxes (last match
    wins): the points with r_in <= |y - centre| <= r_out take the material."""
    d = g.dim
    if tri_n is None:
        tri_n = 5 if d == 2 else 2
    if kmax is None:
        kmax = 64 if d == 2 else 128
    nnz = int(g.row_off[-1])
    nblk = num_blocks(d, n_mat)
    blocks = np.zeros((nblk, nnz))
    E = np.zeros(nnz)
    reg_lo = np.array([r[0] for r in regions], dtype=np.float64).reshape(-1, d) if regions else np.zeros((1, d))
    reg_hi = np.array([r[1] for r in regions], dtype=np.float64).reshape(-1, d) if regions else np.zeros((1, d))
    reg_mat = np.array([r[2] for r in regions], dtype=np.int32) if regions else np.zeros(1, dtype=np.int32)
    V = _f64(g.V)
    fpar = np.array([f[:4] for f in fields], dtype=np.float64).reshape(-1, 4) if fields else np.zeros((1, 4))
    fmat = np.array([f[4] for f in fields], dtype=np.int32) if fields else np.zeros(1, dtype=np.int32)
    if fields and (fmat.min() < 1 or fmat.max() >= n_mat):
        raise ValueError("a field moves weight to a material in [1, n_mat)")
    if n_mat > 8:
        raise ValueError("at most 8 materials")
    spar = np.array([list(sh[0]) + [sh[1], sh[2]] for sh in shells], dtype=np.float64).reshape(-1, d + 2) \
        if shells else np.zeros((1, d + 2))
    smat = np.array([sh[3] for sh in shells], dtype=np.int32) if shells else np.zeros(1, dtype=np.int32)
    if shells and (smat.min() < 0 or smat.max() >= n_mat):
        raise ValueError("a shell's material must be in [0, n_mat)")
    ic = IntegCtx(d, rk_order, n_mat, g.n, _p(g.x), _p(g.R), _p(V), _p(g.nb_off, _i64p),
                  _p(g.nb_idx, _i32p), _p(g.row_off, _i64p), _p(g.col, _i32p), nnz, len(regions),
                  _p(reg_lo), _p(reg_hi), _p(reg_mat, _i32p), _p(blocks), 0, 0, len(fields),
                  _p(fpar), _p(fmat, _i32p), len(shells), _p(spar), _p(smat, _i32p))
    tp, tw = triangle_rule(tri_n)
    tp = _f64(tp); tw = _f64(tw)
    cl = g.cells
    if d == 2:
        sp, sw = segment_rule(seg_n)
        sp = _f64(sp); sw = _f64(sw)
        # upper bound on boundary points: every domain-tagged edge times the line rule
        nbe = int(np.sum((cl.tags <= -1) & (cl.tags >= -4) & (np.arange(cl.cap)[None, :] < cl.nv[:, None])))
        cap = nbe * seg_n
    else:
        qp, qw = tet_rule(tet_n)
        qp = _f64(qp); qw = _f64(qw)
        live = np.arange(cl.fcap)[None, :] < cl.nf[:, None]
        dom = live & (cl.ftags <= -1) & (cl.ftags >= -6)
        cap = int(np.sum(np.where(dom, np.maximum(cl.fnv - 2, 0), 0))) * tp.shape[0]
    bq_y = np.zeros((max(cap, 1), d)); bq_face = np.zeros(max(cap, 1), dtype=np.int32)
    bq_w = np.zeros(max(cap, 1)); bq_nact = np.zeros(max(cap, 1), dtype=np.int32)
    bq_act = np.zeros((max(cap, 1), kmax), dtype=np.int32); bq_N = np.zeros((max(cap, 1), kmax))
    stats = np.zeros(4, dtype=np.int64)
    if d == 2:
        nbq = lib().orc_integrate2d(C.byref(ic), cl.cap, _p(cl.nv, _i32p), _p(cl.verts), _p(cl.tags, _i32p),
                                    tp.shape[0], _p(tp), _p(tw), sp.shape[0], _p(sp), _p(sw), _p(E), cap, kmax,
                                    _p(bq_y), _p(bq_face, _i32p), _p(bq_w), _p(bq_nact, _i32p),
                                    _p(bq_act, _i32p), _p(bq_N), _p(stats, _i64p))
    else:
        nbq = lib().orc_integrate3d(C.byref(ic), cl.fcap, cl.vcap, _p(cl.nf, _i32p), _p(cl.fnv, _i32p),
                                    _p(cl.fverts), _p(cl.ftags, _i32p), qp.shape[0], _p(qp), _p(qw),
                                    tp.shape[0], _p(tp), _p(tw), _p(E), cap, kmax, _p(bq_y),
                                    _p(bq_face, _i32p), _p(bq_w), _p(bq_nact, _i32p), _p(bq_act, _i32p),
                                    _p(bq_N), _p(stats, _i64p))
    assert nbq <= cap
    if np.any(bq_nact[:nbq] >= kmax):
        raise RuntimeError("boundary point with more active functions than kmax")
    return Integrated(g, rk_order, n_mat, blocks, E, bq_y[:nbq], bq_face[:nbq], bq_w[:nbq],
                      bq_nact[:nbq], bq_act[:nbq], bq_N[:nbq], kmax, int(stats[0]), int(stats[1]))


# ---------------------------------------------------------------------------
# Operators and solves (Sec. 4.1 - 4.2)
# ---------------------------------------------------------------------------

@dataclass
class SolveOpts:
    tol_in: float = 1e-13
    tol_out: float = 1e-12
    restart_in: int = 30
    restart_out: int = 30
    max_in: int = 3000
    max_out: int = 500
    precond: str = "jacobi"     # inner right preconditioner: "jacobi" (point) or "patch" (patch block Jacobi)


class Transport:
    """Per-ordinate operators of Sec. 4.2 on an integrated problem."""

    def __init__(self, it: Integrated, omega, w, sigma_t, sigma_s, inv_c_dt, tau, opts: SolveOpts = None):
        self.it = it
        g = it.geom
        self.omega = _f64(omega)
        self.w = _f64(w)
        self.sig_t = _f64(np.atleast_1d(sigma_t))
        self.sig_s = _f64(np.atleast_1d(sigma_s))
        self.a0 = float(inv_c_dt)
        self.tau = _f64(np.broadcast_to(tau, (g.n,)).copy())
        self.opts = opts or SolveOpts()
        self.M = self.omega.shape[0]
        self._keep = []
        self.ctx = self._ctx()

    def _ctx(self):
        it, g, o = self.it, self.it.geom, self.opts
        bq_face = np.ascontiguousarray(it.bq_face if it.nbq else np.zeros(1, np.int32))
        bq_w = _f64(it.bq_w if it.nbq else np.zeros(1))
        bq_nact = np.ascontiguousarray(it.bq_nact if it.nbq else np.zeros(1, np.int32))
        bq_act = np.ascontiguousarray(it.bq_act if it.nbq else np.zeros((1, it.kmax), np.int32))
        bq_N = _f64(it.bq_N if it.nbq else np.zeros((1, it.kmax)))
        lo = _f64(np.asarray(g.dom_lo, dtype=np.float64).reshape(-1))
        hi = _f64(np.asarray(g.dom_hi, dtype=np.float64).reshape(-1))
        self._keep = [bq_face, bq_w, bq_nact, bq_act, bq_N, lo, hi]
        pc = {"jacobi": 0, "patch": 1}[o.precond]
        return OpCtx(g.dim, it.n_mat, self.M, g.n, int(g.row_off[-1]), _p(g.row_off, _i64p), _p(g.col, _i32p),
                     _p(it.blocks), _p(self.omega), _p(self.w), _p(self.sig_t), _p(self.sig_s), self.a0,
                     _p(self.tau), it.nbq, it.kmax, _p(bq_face, _i32p), _p(bq_w), _p(bq_nact, _i32p),
                     _p(bq_act, _i32p), _p(bq_N), o.tol_in, o.tol_out, o.restart_in, o.restart_out, o.max_in,
                     o.max_out, pc, _p(g.x), _p(lo), _p(hi))

    def patches(self):
        """Patches of the block-Jacobi preconditioner: (start[np+1], points[n])."""
        n = self.it.geom.n
        start = np.zeros(n + 1, dtype=np.int64)
        pts = np.zeros(n, dtype=np.int32)
        np_ = lib().orc_patches_of(C.byref(self.ctx), _p(start, _i64p), _p(pts, _i32p))
        return start[:np_ + 1], pts

    def patch_precond(self, m: int, v: np.ndarray) -> np.ndarray:
        """z = M^-1 v of the patch block-Jacobi preconditioner for ordinate m."""
        z = np.zeros(self.it.geom.n)
        lib().orc_patch_precond(C.byref(self.ctx), int(m), _p(_f64(v)), _p(z))
        return z

    def apply(self, which: str, X: np.ndarray) -> np.ndarray:
        code = {"L": 0, "T": 1, "MS": 2, "MD": 3}[which]
        X = _f64(X)
        if X.ndim == 1:
            X = np.repeat(X[:, None], self.M, axis=1)
        Y = np.zeros((self.it.geom.n, self.M))
        lib().orc_apply(C.byref(self.ctx), code, _p(X), _p(Y))
        return Y

    def rhs(self, psi_prev, q, psib):
        n = self.it.geom.n
        F = np.zeros((n, self.M))
        lib().orc_rhs(C.byref(self.ctx), _p(None if psi_prev is None else _f64(psi_prev)), _p(_f64(q)),
                      _p(None if psib is None else _f64(psib)), _p(F))
        return F

    def inner_solve(self, F, m0=0, m1=None):
        """L_m^-1 F for ordinates m0..m1-1; returns (X, Arnoldi steps summed, max relative residual)."""
        m1 = self.M if m1 is None else m1
        X = np.zeros((self.it.geom.n, self.M))
        rm = np.zeros(1)
        its = lib().orc_Linv_range(C.byref(self.ctx), _p(_f64(F)), _p(X), m0, m1, _p(rm))
        return X, int(its), float(rm[0])

    def step(self, psi_prev, q, psib=None, phi0=None):
        """One backward-Euler step (or the steady solve when 1/(c dt) = 0)."""
        n = self.it.geom.n
        psi = np.zeros((n, self.M)); phi = np.zeros(n)
        st = np.zeros(3, dtype=np.int64); res = np.zeros(2)
        lib().orc_step(C.byref(self.ctx), _p(None if psi_prev is None else _f64(psi_prev)), _p(_f64(q)),
                       _p(None if psib is None else _f64(psib)), _p(None if phi0 is None else _f64(phi0)),
                       _p(psi), _p(phi), _p(st, _i64p), _p(res))
        return psi, phi, {"outer_iters": int(st[0]), "inner_iters": int(st[1]), "inner_solves": int(st[2]),
                          "outer_res": float(res[0]), "inner_res_max": float(res[1])}

    def step_source_iteration(self, psi_prev, q, psib=None, iters=50):
        n = self.it.geom.n
        psi = np.zeros((n, self.M)); phi = np.zeros(n)
        lib().orc_step_source_iteration(C.byref(self.ctx), _p(None if psi_prev is None else _f64(psi_prev)),
                                        _p(_f64(q)), _p(None if psib is None else _f64(psib)), iters,
                                        _p(psi), _p(phi))
        return psi, phi

    def point_values(self, coef: np.ndarray) -> np.ndarray:
        """phi(x_i) = sum_j N_j(x_i) coef_j (Eq. flux-expansion)."""
        g = self.it.geom
        coef = _f64(coef)
        nc = 1 if coef.ndim == 1 else coef.shape[1]
        out = np.zeros((g.n, nc))
        lib().orc_point_values(g.n, _p(g.row_off, _i64p), _p(g.col, _i32p), _p(_f64(self.it.E)), _p(coef), nc,
                               _p(out))
        return out[:, 0] if coef.ndim == 1 else out


def csr_to_dense(row_off, col, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[row_off[i]:row_off[i + 1]]] = val[row_off[i]:row_off[i + 1]]
    return A
