"""Parity of the three-dimensional HIP path with the FP64 oracle.

Stages (neighbour lists and pattern bit for bit, cell volumes, blocks, the
point-value matrix and the boundary points), single operator sweeps and the
coupled solves (steady, backward Euler, inflow) on jittered and exact
lattices of the unit cube, with linear and quadratic RK.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._cases import FP64_TOL, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MIXED_TOL = 1e-8
LO, HI = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)


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


def _lattice3(n, jitter=0.2, seed=7, rfac=2.5):
    x, dx = W.jittered_lattice((n, n, n), LO, HI, jitter, seed)
    return x, np.full(x.shape[0], rfac * dx), dx


def _gpu_problem(x, R, regions=()):
    from paper_2008_02205_amd.problem import GpuProblem
    return GpuProblem(x, R, LO, HI, regions)


def _quad(M):
    from paper_2008_02205_amd import mlpg
    return mlpg.mlpg_angular_quadrature(3, M)


@pytest.mark.parametrize("n,jitter,order", [(4, 0.0, 1), (5, 0.2, 0), (5, 0.2, 1), (6, 0.2, 1), (6, 0.2, 2)])
def test_stages_3d(n, jitter, order):
    from paper_2008_02205_amd import mlpg
    _print_case("stages3d", n=n, jitter=jitter, order=order)
    x, R, dx = _lattice3(n, jitter)
    g = oracle.geometry(x, R, LO, HI)
    it = oracle.integrate(g, order)
    P = _gpu_problem(x, R)
    assert np.array_equal(_cpu(P.nbr_off), g.nb_off)
    assert np.array_equal(_cpu(P.nbr_idx), g.nb_idx)
    V = _cpu(mlpg.mlpg_get_volumes(P.h, P.n))
    # same clipping arithmetic on both sides; the volume sums differ in order
    eps = np.finfo(np.float64).eps
    assert np.abs(V - g.V).max() <= 64 * eps * g.V.max()
    assert P.info["oversize_cells"] == int(np.sum(g.cells.rho > R)) == 0
    info = P.integrate(order)
    assert info["missing_pairs"] == 0
    row_off, col = mlpg.mlpg_get_pattern(P.h, P.n, info["nnz"])
    assert np.array_equal(_cpu(row_off), g.row_off)
    assert np.array_equal(_cpu(col), g.col)
    blocks, E = mlpg.mlpg_get_blocks(P.h, info["n_blocks"], info["nnz"])
    blocks, E = _cpu(blocks), _cpu(E)
    names = oracle.block_names(3, 1)
    if order < 2:
        assert info["fallback_qps"] == it.fallbacks
        for b, name in enumerate(names):
            ref = it.blocks[b]
            assert np.abs(blocks[b] - ref).max() <= 1e-12 * np.abs(ref).max(), name
        assert np.abs(E - it.E).max() <= 1e-12 * np.abs(it.E).max()
    else:
        # Quadratic moment matrices near corners reach condition numbers near
        # 1e6, so summation-order differences show at ~1e-10, and a pivot at
        # the fallback threshold may drop an order on one side only.
        print(f"fallbacks gpu {info['fallback_qps']} oracle {it.fallbacks}", flush=True)
        assert abs(info["fallback_qps"] - it.fallbacks) <= 2
        bad = 0
        for b, name in enumerate(names):
            d = np.abs(blocks[b] - it.blocks[b]) / np.abs(it.blocks[b]).max()
            print(f"{name}: max rel diff {d.max():.2e}", flush=True)
            bad += int(np.sum(d > 1e-9))
        assert bad <= 0.01 * blocks.size
        if info["fallback_qps"] == it.fallbacks:
            assert bad == 0
    y, face = P.boundary_points()
    y, face = _cpu(y), _cpu(face)
    assert y.shape[0] == it.nbq
    _match_point_sets(y, face, it.bq_y, it.bq_face)
    P.close()


def _match_point_sets(y, face, yo, fo, tol=1e-13):
    """The two boundary-point sets are equal up to rounding: a one-to-one
    nearest-neighbour matching within tol, on the same face."""
    from scipy.spatial import cKDTree
    tree = cKDTree(np.column_stack([yo, fo * 10.0]))
    d, k = tree.query(np.column_stack([y, face * 10.0]))
    bad = np.nonzero(d > tol)[0]
    for b in bad[:8]:
        print(f"unmatched boundary point {y[b]} face {face[b]}; nearest oracle {yo[k[b]]} face {fo[k[b]]} "
              f"at {d[b]:.2e}", flush=True)
    assert bad.size == 0
    assert np.unique(k).size == k.size


def test_operator_sweeps_3d():
    from paper_2008_02205_amd import mlpg
    _print_case("sweeps3d", n=5, M=12)
    x, R, dx = _lattice3(5)
    g = oracle.geometry(x, R, LO, HI)
    it = oracle.integrate(g, 1)
    om, w = oracle.angular_quadrature(3, 12)
    tr = oracle.Transport(it, om, w, 1.3, 0.6, 7.0, dx)
    P = _gpu_problem(x, R)
    P.integrate(1)
    P.assemble(*_quad(12), [1.3], [0.6], 7.0, dx)
    X = np.random.default_rng(4).uniform(-1, 1, (g.n, 12))
    for name, code in (("L", mlpg.MLPG_OP_L), ("T", mlpg.MLPG_OP_T), ("MS", mlpg.MLPG_OP_MS),
                       ("MD", mlpg.MLPG_OP_SRC)):
        assert rel_l2(_cpu(mlpg.mlpg_apply(P.h, code, _dev(X))), tr.apply(name, X)) <= 1e-13, name
    P.close()


def _solve_both_3d(n, M, order, sig_t, sig_s, inv_c_dt, steps, q_fn, psib_fn=None, psi0_fn=None, jitter=0.2,
                   rfac=2.5, precision=None, omega=None, w=None, max_inner=None):
    from paper_2008_02205_amd import mlpg
    x, R, dx = _lattice3(n, jitter, rfac=rfac)
    g = oracle.geometry(x, R, LO, HI)
    it = oracle.integrate(g, order)
    if omega is None:
        om_o, w_o = oracle.angular_quadrature(3, M)
        om_g, w_g = _quad(M)
    else:
        om_o, w_o = om_g, w_g = omega, w
    tr = oracle.Transport(it, om_o, w_o, sig_t, sig_s, inv_c_dt, dx)
    P = _gpu_problem(x, R)
    P.integrate(order)
    P.assemble(om_g, w_g, [sig_t], [sig_s], inv_c_dt, dx,
               precision=mlpg.MLPG_FP64 if precision is None else precision)
    y_g, _ = P.boundary_points()
    psi_o = psi0_fn(x, om_o) if psi0_fn else None
    phi_o = psi_o @ w_o if psi_o is not None else None
    if psi0_fn:
        P.set_state(_dev(psi0_fn(x, om_g)))
    out = []
    for s in range(1, steps + 1):
        t = s * (1.0 / inv_c_dt if inv_c_dt > 0 else 0.0)
        pb_o = psib_fn(it.bq_y, om_o, t) if psib_fn else None
        psi_o, phi_o, info_o = tr.step(psi_o, q_fn(x, om_o, t), pb_o, phi_o)
        pb_g = _dev(psib_fn(_cpu(y_g), om_g, t)) if psib_fn else None
        opts = None
        if max_inner:
            opts = mlpg.mlpg_default_opts()
            opts.max_inner = max_inner
        phi_g, pv_g, psi_g, info_g = P.step(_dev(q_fn(x, om_g, t)), pb_g, opts)
        e = (rel_l2(_cpu(phi_g), phi_o), rel_l2(_cpu(pv_g), tr.point_values(phi_o)), rel_l2(_cpu(psi_g), psi_o))
        print(f"step {s}: phi {e[0]:.2e} point {e[1]:.2e} psi {e[2]:.2e} outer {info_g['outer_iters']} "
              f"(oracle {info_o['outer_iters']})", flush=True)
        out.append((e, info_g))
    P.close()
    return out


def _gauss(x, om, t):
    return np.repeat(W.gaussian_source(x, (0.5, 0.5, 0.5), 0.15)[:, None], om.shape[0], axis=1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_steady_gaussian_source_3d(precision):
    """The Gaussian-source scattering problem at reduced size (linear RK)."""
    from paper_2008_02205_amd import mlpg
    _print_case("steady3d", n=5, M=24, precision=precision)
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for e, info in _solve_both_3d(5, 24, 1, 1.0, 0.9, 0.0, 1, _gauss, precision=prec):
        assert info["converged"] == 1 and max(e) <= tol


def test_quadratic_rk_scattering_3d():
    """Quadratic RK with R = 2.5 h (the 3D workload's discretisation) at 5^3, 12 ordinates."""
    _print_case("quadratic3d", n=5, M=12)
    # restarted GMRES(30) with point Jacobi needs 700-2300 steps per ordinate
    # here, and the tail depends on rounding; the GPU gets room beyond 3000
    for e, info in _solve_both_3d(5, 12, 2, 1.0, 0.9, 0.0, 1, _gauss, max_inner=10000):
        assert info["converged"] == 1
        # the FP64 bar (measured about 4e-11: quadratic-RK blocks agree to about
        # 1e-10 of their largest entry, and the fields inherit that)
        assert max(e) <= FP64_TOL


def test_backward_euler_and_inflow_3d():
    """Two backward-Euler steps with an oblique plane-wave inflow in a pure absorber."""
    _print_case("be-inflow3d", n=5, M=1)
    om = np.array([[0.8, 0.36, 0.48]]); w = np.array([4 * np.pi])
    res = _solve_both_3d(5, 1, 1, 2.0, 0.0, 10.0, 2, lambda x, o, t: np.zeros((x.shape[0], 1)),
                         psib_fn=lambda y, o, t: W.absorber_psi(y, 0.8, 2.0)[:, None],
                         psi0_fn=lambda x, o: np.zeros((x.shape[0], 1)), omega=om, w=w)
    for e, info in res:
        assert info["converged"] == 1 and max(e) <= FP64_TOL
