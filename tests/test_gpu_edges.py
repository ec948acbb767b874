"""Edge cases of the HIP path against the FP64 oracle.

Ordinate counts at the sweep's launch-shape boundaries (the row-group
kernel's largest, the wave kernel's partial first wave, a second and a
third 64-ordinate chunk holding two ordinates), and the smallest problems
the method admits: one point (its cell is the whole domain and the linear
RK falls back to order 0), a 2 x 2 and a 3 x 3 lattice in 2D, one and
eight points in 3D.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._cases import FP64_TOL, lattice_case, rel_l2

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


def _problem(x, R, lo, hi, M, sig_t, sig_s, inv_c_dt, tau, precision="fp64"):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    P = GpuProblem(x, R, lo, hi)
    P.integrate(1)
    P.assemble(*mlpg.mlpg_angular_quadrature(x.shape[1], M), [sig_t], [sig_s], inv_c_dt, tau,
               precision=mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED)
    return P


@pytest.mark.parametrize("M", [2, 46, 48, 66, 130])
def test_sweeps_across_launch_shapes(M):
    print(f"[case] sweeps n=12 M={M}", flush=True)
    from paper_2008_02205_amd import mlpg
    x, R, dx = lattice_case(12)
    g = oracle.geometry(x, R, (0, 0), (1, 1))
    it = oracle.integrate(g, 1)
    om, w = oracle.angular_quadrature(2, M)
    tr = oracle.Transport(it, om, w, 1.3, 0.6, 7.0, dx)
    P = _problem(x, R, (0, 0), (1, 1), M, 1.3, 0.6, 7.0, dx)
    X = np.random.default_rng(9).uniform(-1, 1, (g.n, M))
    for name, code in (("L", mlpg.MLPG_OP_L), ("T", mlpg.MLPG_OP_T), ("MS", mlpg.MLPG_OP_MS),
                       ("MD", mlpg.MLPG_OP_SRC)):
        e = rel_l2(_cpu(mlpg.mlpg_apply(P.h, code, torch.from_numpy(X).cuda())), tr.apply(name, X))
        print(f"{name}: {e:.1e}", flush=True)
        assert e <= 1e-13, name
    P.close()


def _steady_both(x, R, lo, hi, M, dx, precision):
    dim = x.shape[1]
    g = oracle.geometry(x, R, lo, hi)
    it = oracle.integrate(g, 1)
    om, w = oracle.angular_quadrature(dim, M)
    tr = oracle.Transport(it, om, w, 1.0, 0.5, 0.0, dx)
    q = np.ones((g.n, M))
    psi_o, phi_o, _ = tr.step(None, q, None, None)
    P = _problem(x, R, lo, hi, M, 1.0, 0.5, 0.0, dx, precision)
    phi_g, pv_g, psi_g, info = P.step(torch.from_numpy(q).cuda(), None)
    fb = P.info["fallback_qps"]
    P.close()
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    e = (rel_l2(_cpu(phi_g), phi_o), rel_l2(_cpu(pv_g), tr.point_values(phi_o)), rel_l2(_cpu(psi_g), psi_o))
    print(f"{precision}: phi {e[0]:.1e} phi(x_i) {e[1]:.1e} psi {e[2]:.1e} fallback qps {fb}", flush=True)
    assert info["converged"] == 1
    assert max(e) <= tol
    return fb


@pytest.mark.parametrize("n,precision", [(1, "fp64"), (2, "fp64"), (2, "mixed"), (3, "fp64")])
def test_smallest_problems_2d(n, precision):
    print(f"[case] smallest 2D n={n}x{n} M=8 {precision}", flush=True)
    x, R, dx = lattice_case(n)
    fb = _steady_both(x, R, (0, 0), (1, 1), 8, dx, precision)
    if n == 1:
        assert fb > 0   # one point: every quadrature point falls back to order 0


@pytest.mark.parametrize("n", [1, 2])
def test_smallest_problems_3d(n):
    print(f"[case] smallest 3D n={n}^3 M=24", flush=True)
    x, dx = W.jittered_lattice((n, n, n), (0, 0, 0), (1, 1, 1), 0.2, 7)
    R = np.full(x.shape[0], 2.5 * dx)
    _steady_both(x, R, (0, 0, 0), (1, 1, 1), 24, dx, "fp64")
