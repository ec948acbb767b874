"""Points that move every time step: neighbours, cells, integration and assembly inside the time loop.

The HIP path (mlpg_update_points, then mlpg_integrate and mlpg_assemble on the
same handle, the per-point state kept) against the FP64 oracle doing the same
sequence from scratch each step, and the degenerate move to the same points.
"""
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


def _run_gpu(w, xs, R, dx, om, wq, precision, steps):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    P = GpuProblem(xs[0], R, w.lo, w.hi)
    P.integrate(1)
    P.assemble(om, wq, [1.0], [0.5], 1.0 / w.dt, dx, precision=prec)
    P.set_state(_dev(W.mms_sin_psi(xs[0], om, 0.0)))
    out = []
    for s in range(1, steps + 1):
        info = P.move(xs[s], R)
        assert info["oversize_cells"] == 0
        P.integrate(1)
        P.assemble(om, wq, [1.0], [0.5], 1.0 / w.dt, dx, precision=prec)
        phi, pv, psi, inf = P.step(_dev(W.mms_sin_source(xs[s], om, s * w.dt, 1.0, 0.5)))
        assert inf["converged"] == 1
        out.append((_cpu(phi), _cpu(pv), _cpu(psi)))
    P.close()
    return out


def _run_oracle(w, xs, R, dx, om, wq, steps):
    psi = W.mms_sin_psi(xs[0], om, 0.0)
    phi = psi @ wq
    out = []
    for s in range(1, steps + 1):
        g = oracle.geometry(xs[s], R, w.lo, w.hi)
        it = oracle.integrate(g, 1)
        tr = oracle.Transport(it, om, wq, 1.0, 0.5, 1.0 / w.dt, dx)
        psi, phi, _ = tr.step(psi, W.mms_sin_source(xs[s], om, s * w.dt, 1.0, 0.5), None, phi)
        out.append((phi, tr.point_values(phi), psi))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_moving_points_backward_euler(precision):
    """Three backward-Euler steps of the manufactured problem on a 12^2 lattice sheared by the cellular flow."""
    from paper_2008_02205_amd import mlpg
    print(f"[case] moving points n=12 M=8 steps=3 {precision}", flush=True)
    w = W.config(8, 12)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    xs = [x]
    for _ in range(3):
        xs.append(W.advect_points(w, xs[-1], 4 * w.dt))   # a larger stride so that the pattern changes
    assert any(not np.array_equal(oracle.neighbors(xs[0], R)[1], oracle.neighbors(xs[s], R)[1])
               for s in (1, 2, 3))
    om_o, w_o = oracle.angular_quadrature(2, 8)
    om_g, w_g = mlpg.mlpg_angular_quadrature(2, 8)
    ref = _run_oracle(w, xs, R, dx, om_o, w_o, 3)
    got = _run_gpu(w, xs, R, dx, om_g, w_g, precision, 3)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for s, (a, b) in enumerate(zip(got, ref)):
        e = [rel_l2(u, v) for u, v in zip(a, b)]
        print(f"step {s + 1}: phi {e[0]:.2e} point {e[1]:.2e} psi {e[2]:.2e}", flush=True)
        assert max(e) <= tol


def test_move_to_the_same_points_changes_nothing():
    """Rebuilding at unchanged positions reproduces the run without a rebuild."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    print("[case] move to the same points n=10 M=8", flush=True)
    w = W.config(8, 10)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    om, wq = mlpg.mlpg_angular_quadrature(2, 8)
    res = []
    for rebuild in (False, True):
        P = GpuProblem(x, R, w.lo, w.hi)
        P.integrate(1)
        P.assemble(om, wq, [1.0], [0.5], 1.0 / w.dt, dx)
        P.set_state(_dev(W.mms_sin_psi(x, om, 0.0)))
        for s in (1, 2):
            if rebuild:
                P.move(x, R)
                P.integrate(1)
                P.assemble(om, wq, [1.0], [0.5], 1.0 / w.dt, dx)
            phi, pv, psi, inf = P.step(_dev(W.mms_sin_source(x, om, s * w.dt, 1.0, 0.5)))
        res.append(_cpu(psi))
        P.close()
    # the integration sums with atomics, so a rebuild may differ in the last bits
    assert rel_l2(res[1], res[0]) <= 1e-12
