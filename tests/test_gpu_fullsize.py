"""Coupled solves against the oracle at the workloads' own sizes.

* The headline workload (128 x 128 jittered lattice, 64 ordinates, sigma_t = 1,
  sigma_s = 0.5, manufactured source, backward Euler with 1/(c dt) = 100):
  backward-Euler steps 1 and 2 in full -- inner GMRES on every ordinate, the
  outer GMRES on Phi, the recovery of Psi -- FP64 within 1e-10 and mixed within
  1e-8 relative L2 on Phi, phi(x_i) and Psi (Sec. 4.1-4.2).
* The beam workload's physics (void and opaque scattering materials, 256
  locally refined ordinates, the inflow beam, backward Euler with
  1/(c dt) = 20) at about 3,200 Poisson-disk points: steps 1 and 2, FP64 and
  mixed.

The oracle solves each reference once per module (about 15 s per step of the
headline workload on 8 host threads).
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
STEPS = 2
BEAM_PD_RADIUS = 0.02   # 3,167 Poisson-disk points on [0,2] x [0,1]


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


@pytest.fixture(scope="module")
def _mms_reference():
    """Oracle backward-Euler steps 1..STEPS of the 128 x 128, 64-ordinate workload."""
    w = W.config(2)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    om, wq = oracle.angular_quadrature(2, w.n_ord)
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, w.rk_order)
    tr = oracle.Transport(it, om, wq, w.sigma_t[0], w.sigma_s[0], w.inv_c_dt, dx)
    psi = W.initial_psi(w, x, om)
    phi = psi @ wq
    out = []
    for s in range(1, STEPS + 1):
        psi, phi, info = tr.step(psi, W.source_values(w, x, om, s * w.dt), None, phi)
        assert info["inner_res_max"] <= 1e-13 and info["outer_res"] <= 1e-12
        print(f"oracle step {s}: outer {info['outer_iters']} inner {info['inner_iters']}", flush=True)
        out.append((psi.copy(), phi.copy(), tr.point_values(phi)))
    return w, x, R, dx, out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_headline_workload_coupled_steps(precision, _mms_reference):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w, x, R, dx, ref = _mms_reference
    _print_case("full-coupled", workload=w.name, n=x.shape[0], M=w.n_ord, precision=precision)
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    om, wq = mlpg.mlpg_angular_quadrature(2, w.n_ord)
    P = GpuProblem(x, R, w.lo, w.hi)
    P.integrate(w.rk_order)
    P.assemble(om, wq, [w.sigma_t[0]], [w.sigma_s[0]], w.inv_c_dt, dx, precision=prec)
    P.set_state(_dev(W.initial_psi(w, x, om)))
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for s, (psi_o, phi_o, pv_o) in enumerate(ref, start=1):
        phi, pv, psi, info = P.step(_dev(W.source_values(w, x, om, s * w.dt)))
        assert info["converged"] == 1
        e = (rel_l2(_cpu(phi), phi_o), rel_l2(_cpu(pv), pv_o), rel_l2(_cpu(psi), psi_o))
        print(f"step {s} {precision}: Phi {e[0]:.2e} phi(x_i) {e[1]:.2e} Psi {e[2]:.2e} outer {info['outer_iters']} "
              f"refinements {info['refinements']} fp64 completions {info['fp64_completions']}", flush=True)
        assert max(e) <= tol, (s, e)
    P.close()


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
    pb = W.inflow_values(w, it.bq_y, om)
    out = []
    for s in range(1, STEPS + 1):
        psi, phi, info = tr.step(psi, W.source_values(w, x, om, s * w.dt), pb, phi)
        assert info["inner_res_max"] <= 1e-13 and info["outer_res"] <= 1e-12
        print(f"oracle beam step {s}: outer {info['outer_iters']} inner {info['inner_iters']}", flush=True)
        out.append((psi.copy(), phi.copy(), tr.point_values(phi)))
    return w, x, R, dx, out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_beam_workload_steps_3k_points(precision, _beam_reference):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w, x, R, dx, ref = _beam_reference
    _print_case("beam-3k", n=x.shape[0], M=w.n_ord, precision=precision)
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    om, wq = mlpg.mlpg_angular_quadrature(2, w.n_ord, mlpg.MLPG_QUAD_BEAM_DENSE)
    P = GpuProblem(x, R, w.lo, w.hi, w.regions)
    P.integrate(1)
    P.assemble(om, wq, list(w.sigma_t), list(w.sigma_s), w.inv_c_dt, dx, precision=prec)
    P.set_state(_dev(W.initial_psi(w, x, om)))
    y, _ = P.boundary_points()
    pb = _dev(W.inflow_values(w, _cpu(y), om))
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for s, (psi_o, phi_o, pv_o) in enumerate(ref, start=1):
        phi, pv, psi, info = P.step(_dev(W.source_values(w, x, om, s * w.dt)), pb)
        assert info["converged"] == 1
        e = (rel_l2(_cpu(phi), phi_o), rel_l2(_cpu(pv), pv_o), rel_l2(_cpu(psi), psi_o))
        print(f"beam step {s} {precision}: Phi {e[0]:.2e} phi(x_i) {e[1]:.2e} Psi {e[2]:.2e} "
              f"outer {info['outer_iters']}", flush=True)
        assert max(e) <= tol, (s, e)
    P.close()
