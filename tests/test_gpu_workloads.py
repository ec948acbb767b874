"""Parity at the workloads' own sizes, and on the beam problem's features.

* Stages (neighbour lists, pattern, cells, blocks, point-value matrix) of
  the 128 x 128 manufactured-solution lattice and of the 65k-point
  Poisson-disk beam problem with its two material regions, in full.
* Single operator sweeps at 128 x 128 with 64 ordinates: the launch shapes
  the benchmark times.
* At 128 x 128 the oracle cannot finish the coupled solve in test time, so
  the first-flight solve (sigma_s = 0: Psi = L^-1 F exactly) is checked on
  sampled ordinates, each solved by the oracle on its own.
* The beam problem's physics (void and opaque scattering materials, 256
  locally refined ordinates, inflow beam, backward Euler) at a reduced point
  count, against the oracle's full nested solve.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests._cases import FP64_TOL, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MIXED_TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02205_amd import mlpg
    mlpg.lib()


def _cpu(t):
    return t.detach().cpu().numpy()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _compare_stages(x, R, lo, hi, regions=(), n_mat=1):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    g = oracle.geometry(x, R, lo, hi)
    it = oracle.integrate(g, 1, regions=regions, n_mat=n_mat)
    P = GpuProblem(x, R, lo, hi, regions)
    assert np.array_equal(_cpu(P.nbr_off), g.nb_off)
    assert np.array_equal(_cpu(P.nbr_idx), g.nb_idx)
    V = _cpu(mlpg.mlpg_get_volumes(P.h, P.n))
    # Both sides clip the same polygon with the same cuts; their vertices
    # differ by about one rounding of a coordinate (eps * max|x|), so a
    # cell's area by at most its perimeter (<= 2 pi rho) times that.
    eps = np.finfo(np.float64).eps
    tol_v = 2 * np.pi * g.cells.rho.max() * eps * np.abs(x).max()
    assert np.abs(V - g.V).max() <= tol_v
    assert P.info["oversize_cells"] == int(np.sum(g.cells.rho > R)) == 0
    info = P.integrate(1)
    assert info["missing_pairs"] == 0 and info["fallback_qps"] == it.fallbacks
    assert info["n_mat"] == n_mat
    row_off, col = mlpg.mlpg_get_pattern(P.h, P.n, info["nnz"])
    assert np.array_equal(_cpu(row_off), g.row_off)
    assert np.array_equal(_cpu(col), g.col)
    blocks, E = mlpg.mlpg_get_blocks(P.h, info["n_blocks"], info["nnz"])
    blocks, E = _cpu(blocks), _cpu(E)
    for b, name in enumerate(oracle.block_names(2, n_mat)):
        ref = it.blocks[b]
        scale = np.abs(ref).max()
        assert np.abs(blocks[b] - ref).max() <= 1e-12 * scale, name
    assert np.abs(E - it.E).max() <= 1e-12 * np.abs(it.E).max()
    y, face = P.boundary_points()
    y, face = _cpu(y), _cpu(face)
    assert y.shape[0] == it.nbq
    ka = np.lexsort((it.bq_y[:, 1], it.bq_y[:, 0], it.bq_face))
    kb = np.lexsort((y[:, 1], y[:, 0], face))
    assert np.array_equal(face[kb], it.bq_face[ka])
    assert np.abs(y[kb] - it.bq_y[ka]).max() <= 1e-14
    P.close()
    return g, it


def test_full_size_stages_mms_lattice():
    w = W.config(2)
    _print_case("full-stages", workload=w.name, n=w.counts)
    x, dx = W.points_for(w)
    _compare_stages(x, W.radii_for(w, x, dx), w.lo, w.hi)


def test_full_size_stages_beam_two_materials():
    w = W.config(4)
    _print_case("full-stages", workload=w.name, pd_radius=w.pd_radius)
    x, dx = W.points_for(w)
    print(f"Poisson-disk points: {x.shape[0]}", flush=True)
    g, it = _compare_stages(x, W.radii_for(w, x, dx), w.lo, w.hi, w.regions, 2)
    # the per-material mass blocks add up to the domain area; material 1
    # (x >= 1) holds half of it up to the quadrature of the region's edge
    names = oracle.block_names(2, 2)
    m0, m1 = it.blocks[names.index("mass0")].sum(), it.blocks[names.index("mass1")].sum()
    assert abs(m0 + m1 - 2.0) <= 1e-12 and abs(m1 - 1.0) <= 1e-2


def _mms_problem(sigma_s, precision):
    """The 128 x 128 lattice on the GPU with the library's own ordinates."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w = W.config(2)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    om, wq = mlpg.mlpg_angular_quadrature(2, w.n_ord)
    P = GpuProblem(x, R, w.lo, w.hi)
    P.integrate(w.rk_order)
    P.assemble(om, wq, [w.sigma_t[0]], [sigma_s], w.inv_c_dt, dx, precision=precision)
    return w, x, R, dx, om, wq, P


def test_full_size_operator_sweeps():
    from paper_2008_02205_amd import mlpg
    w_s = 0.5
    w, x, R, dx, om, wq, P = _mms_problem(w_s, mlpg.MLPG_FP64)
    _print_case("full-sweeps", workload=w.name, M=om.shape[0])
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, 1)
    om_o, wq_o = oracle.angular_quadrature(2, w.n_ord)
    tr = oracle.Transport(it, om_o, wq_o, w.sigma_t[0], w_s, w.inv_c_dt, dx)
    X = np.random.default_rng(7).uniform(-1, 1, (g.n, om.shape[0]))
    for name, code in (("L", mlpg.MLPG_OP_L), ("T", mlpg.MLPG_OP_T), ("MS", mlpg.MLPG_OP_MS),
                       ("MD", mlpg.MLPG_OP_SRC)):
        Y = _cpu(mlpg.mlpg_apply(P.h, code, _dev(X)))
        assert rel_l2(Y, tr.apply(name, X)) <= 1e-13, name
    P.close()


@pytest.fixture(scope="module")
def _first_flight_reference():
    """Oracle L_m^-1 F_m for two sampled ordinate ranges of the 128 x 128,
    64-ordinate lattice (first backward-Euler step, manufactured source)."""
    w = W.config(2)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    om, wq = oracle.angular_quadrature(2, w.n_ord)
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, 1)
    tr = oracle.Transport(it, om, wq, w.sigma_t[0], 0.0, w.inv_c_dt, dx)
    psi0 = W.initial_psi(w, x, om)
    q = W.source_values(w, x, om, w.dt)
    F = tr.rhs(psi0, q, None)
    ref = {}
    for m0, m1 in ((0, 3), (w.n_ord - 3, w.n_ord)):
        X, _, res = tr.inner_solve(F, m0, m1)
        assert res <= 1e-13
        for m in range(m0, m1):
            ref[m] = X[:, m].copy()
    return ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_first_flight_sampled_ordinates(precision, _first_flight_reference):
    from paper_2008_02205_amd import mlpg
    ref = _first_flight_reference
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    w, x, R, dx, om, wq, P = _mms_problem(0.0, prec)
    _print_case("full-first-flight", workload=w.name, precision=precision)
    P.set_state(_dev(W.initial_psi(w, x, om)))
    phi, pv, psi, info = P.step(_dev(W.source_values(w, x, om, w.dt)))
    psi = _cpu(psi)
    assert info["converged"] == 1 and info["outer_iters"] <= 1
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for m, xm in ref.items():
        e = rel_l2(psi[:, m], xm)
        print(f"ordinate {m}: rel L2 {e:.2e}", flush=True)
        assert e <= tol, m
    # Phi is the quadrature sum of the recovered Psi (any size)
    assert rel_l2(_cpu(phi), psi @ wq) <= 1e-13
    P.close()


BEAM_PD_RADIUS = 0.08   # about 210 Poisson-disk points on [0,2] x [0,1]
BEAM_STEPS = 1


@pytest.fixture(scope="module")
def _beam_reference():
    w = W.config(4)
    x = W.poisson_disk(w.lo, w.hi, BEAM_PD_RADIUS, w.seed)
    dx = math.sqrt(float(np.prod(np.subtract(w.hi, w.lo))) / x.shape[0])
    R = W.radii_for(w, x, dx)
    om, wq = oracle.angular_quadrature(2, w.n_ord, w.ord_kind)
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, 1, regions=w.regions, n_mat=2)
    tr = oracle.Transport(it, om, wq, w.sigma_t, w.sigma_s, w.inv_c_dt, dx)
    psi = W.initial_psi(w, x, om)
    phi = psi @ wq
    out = []
    for s in range(1, BEAM_STEPS + 1):
        q = W.source_values(w, x, om, s * w.dt)
        pb = W.inflow_values(w, it.bq_y, om)
        psi, phi, info = tr.step(psi, q, pb, phi)
        out.append((psi.copy(), phi.copy(), tr.point_values(phi)))
    return w, x, R, dx, om, wq, out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_beam_void_opaque_reduced(precision, _beam_reference):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w, x, R, dx, om, wq, ref = _beam_reference
    _print_case("beam", n=x.shape[0], M=om.shape[0], precision=precision)
    # the library's locally refined rule: azimuths near pi carry a few ulps
    om_g, wq_g = mlpg.mlpg_angular_quadrature(2, w.n_ord, mlpg.MLPG_QUAD_BEAM_DENSE)
    assert np.abs(om_g - om).max() <= 1e-14 and np.abs(wq_g - wq).max() <= 1e-14
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    P = GpuProblem(x, R, w.lo, w.hi, w.regions)
    P.integrate(1)
    P.assemble(om_g, wq_g, list(w.sigma_t), list(w.sigma_s), w.inv_c_dt, dx, precision=prec)
    assert P.info["n_mat"] == 2
    P.set_state(_dev(W.initial_psi(w, x, om_g)))
    y, _ = P.boundary_points()
    pb = _dev(W.inflow_values(w, _cpu(y), om_g))
    assert float(pb.sum()) > 0
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for s, (psi_o, phi_o, pv_o) in enumerate(ref, start=1):
        phi, pv, psi, info = P.step(_dev(W.source_values(w, x, om_g, s * w.dt)), pb)
        assert info["converged"] == 1
        e = (rel_l2(_cpu(phi), phi_o), rel_l2(_cpu(pv), pv_o), rel_l2(_cpu(psi), psi_o))
        print(f"beam {precision}: phi {e[0]:.2e} point {e[1]:.2e} psi {e[2]:.2e} outer {info['outer_iters']}",
              flush=True)
        assert max(e) <= tol
    P.close()


def test_full_size_3d_gaussian_workload_stages():
    """The 3D workload at its own size (40^3 jittered lattice, quadratic RK, R = 2.5 h):
    neighbour lists and pattern bit for bit, sampled cells against the oracle one by one,
    and the block identities that hold at any size."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w = W.config(3)
    _print_case("full-stages-3d", workload=w.name, n=w.counts)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    off, idx = oracle.neighbors(x, R)
    P = GpuProblem(x, R, w.lo, w.hi)
    assert np.array_equal(_cpu(P.nbr_off), off)
    assert np.array_equal(_cpu(P.nbr_idx), idx)
    V = _cpu(mlpg.mlpg_get_volumes(P.h, P.n))
    assert abs(V.sum() - 1.0) <= 1e-12
    assert P.info["oversize_cells"] == 0 and P.info["failed_cells"] == 0
    ids = np.random.default_rng(5).choice(x.shape[0], 300, replace=False)
    cl = oracle.cells3d(x, R, off, idx, w.lo, w.hi, ids=ids)
    assert cl.failed == 0
    eps = np.finfo(np.float64).eps
    assert np.abs(V[ids] - cl.V).max() <= 64 * eps * cl.V.max()
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = P.integrate(w.rk_order)
    torch.cuda.synchronize()
    print(f"3D integration of {x.shape[0]} cells: {time.perf_counter() - t0:.2f} s, nnz {info['nnz']}, "
          f"fallbacks {info['fallback_qps']}", flush=True)
    assert info["missing_pairs"] == 0
    row_off, col = mlpg.mlpg_get_pattern(P.h, P.n, info["nnz"])
    row_off, col = _cpu(row_off), _cpu(col)
    ro, co = oracle.pattern(P.n, off, idx)
    assert np.array_equal(row_off, ro) and np.array_equal(col, co)
    blocks, _ = mlpg.mlpg_get_blocks(P.h, info["n_blocks"], info["nnz"], want_E=False)
    names = oracle.block_names(3, 1)
    blk = lambda nm: _cpu(blocks[names.index(nm)])
    n = P.n
    mass = blk("mass0")
    assert abs(mass.sum() - 1.0) <= 1e-10
    rows = np.repeat(np.arange(n), np.diff(row_off))
    for a, nm in enumerate(("dx0", "dy0", "dz0")):
        D = blk(nm)
        assert np.abs(np.bincount(col, D, n)).max() <= 1e-9
        lhs = np.bincount(col, D * x[rows, a], n)
        assert np.abs(lhs - np.bincount(col, mass, n)).max() <= 1e-9
    for f in range(6):
        assert abs(blk(f"s{f}").sum() - 1.0) <= 1e-10
    P.close()


def test_3d_sweeps_at_the_workload_launch_shape():
    """The 3D workload's sweep configuration (R = 2.5h, ~450 nonzeros per interior row, 10 streams, 96
    ordinates: one full and one half-empty 64-lane chunk per row) against the oracle's operators, at 8^3
    points.  Linear RK keeps the blocks equal to rounding (the stream layout does not depend on the
    order; quadratic-RK blocks are compared in the stage tests)."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w = W.config(3, 8)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    _print_case("3d-sweeps", workload=w.name, n=x.shape[0], M=w.n_ord)
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, 1)
    om, wq = oracle.angular_quadrature(3, w.n_ord)
    tr = oracle.Transport(it, om, wq, w.sigma_t[0], w.sigma_s[0], 0.0, dx)
    P = GpuProblem(x, R, w.lo, w.hi)
    P.integrate(1)
    P.assemble(*mlpg.mlpg_angular_quadrature(3, w.n_ord), [w.sigma_t[0]], [w.sigma_s[0]], 0.0, dx)
    X = np.random.default_rng(11).uniform(-1, 1, (g.n, w.n_ord))
    for name, code in (("L", mlpg.MLPG_OP_L), ("T", mlpg.MLPG_OP_T), ("MS", mlpg.MLPG_OP_MS),
                       ("MD", mlpg.MLPG_OP_SRC)):
        Y = _cpu(mlpg.mlpg_apply(P.h, code, _dev(X)))
        e = rel_l2(Y, tr.apply(name, X))
        print(f"{name}: {e:.2e}", flush=True)
        assert e <= 1e-13, name
    P.close()
