"""Parity of spatially varying materials (material fields) and of the paper's manufactured problems.

The HIP path (material fields evaluated at every volume quadrature point in
the integration kernels) against the FP64 oracle: blocks in 2D and 3D,
steady and backward-Euler solves of the sinusoidal and outgoing-wave
manufactured problems of Sec. 5.1, and the second-order spatial convergence
the paper reports, continued on the GPU to lattices the oracle does not reach.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests._cases import FP64_TOL, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MIXED_TOL = 1e-8
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_orders.json")))


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


def _points(n, d, jitter, seed=13):
    lo, hi = (-1.0,) * d, (1.0,) * d
    x, dx = W.jittered_lattice((n,) * d, lo, hi, jitter, seed)
    return x, np.full(x.shape[0], (2.0 if d == 2 else 2.5) * dx), dx, lo, hi


@pytest.mark.parametrize("d,n", [(2, 10), (3, 4)])
def test_field_blocks(d, n):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    _print_case("field-blocks", d=d, n=n)
    x, R, dx, lo, hi = _points(n, d, 0.2)
    g = oracle.geometry(x, R, lo, hi)
    it = oracle.integrate(g, 1, n_mat=3, fields=W.MMS_COS_FIELDS)
    P = GpuProblem(x, R, lo, hi, fields=W.MMS_COS_FIELDS)
    info = P.integrate(1)
    assert info["n_mat"] == 3 and info["missing_pairs"] == 0
    blocks, E = mlpg.mlpg_get_blocks(P.h, info["n_blocks"], info["nnz"])
    blocks = _cpu(blocks)
    for b, name in enumerate(oracle.block_names(d, 3)):
        ref = it.blocks[b]
        assert np.abs(blocks[b] - ref).max() <= 1e-12 * np.abs(ref).max(), name
    # clearing the fields restores the single-material blocks
    mlpg.mlpg_material_fields(P.h, ())
    info = P.integrate(1)
    it1 = oracle.integrate(g, 1, n_mat=3)
    blocks = _cpu(mlpg.mlpg_get_blocks(P.h, info["n_blocks"], info["nnz"])[0])
    assert np.abs(blocks[0] - it1.blocks[0]).max() <= 1e-12 * np.abs(it1.blocks[0]).max()
    assert np.all(blocks[1 + d:3 * (1 + d)] == 0.0)
    P.close()


def _solve_pair(kind, n, M, steps=0, dt=0.0, precision="fp64"):
    """GPU and oracle solves of a Sec. 5.1 problem; returns per-step errors (phi, point values, psi)."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w = W.config(6 if kind == "cos" else 7, n)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    inv_c_dt = 0.0 if steps == 0 else 1.0 / dt
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, 1, n_mat=len(w.sigma_t), fields=w.fields)
    om_o, w_o = oracle.angular_quadrature(2, M)
    om_g, w_g = mlpg.mlpg_angular_quadrature(2, M)
    tr = oracle.Transport(it, om_o, w_o, w.sigma_t, w.sigma_s, inv_c_dt, dx)
    P = GpuProblem(x, R, w.lo, w.hi, fields=w.fields)
    P.integrate(1)
    P.assemble(om_g, w_g, list(w.sigma_t), list(w.sigma_s), inv_c_dt, dx,
               precision=mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED)
    y_g, _ = P.boundary_points()
    y_g = _cpu(y_g)
    src = W.mms_cos_source if kind == "cos" else W.mms_wave_source
    psi_f = W.mms_cos_psi if kind == "cos" else W.mms_wave_psi
    psi_o = phi_o = None
    if steps:
        psi_o = np.repeat(psi_f(x, w.t0)[:, None], M, axis=1)
        phi_o = psi_o @ w_o
        P.set_state(_dev(np.repeat(psi_f(x, w.t0)[:, None], M, axis=1)))
    out = []
    for s in range(max(steps, 1)):
        t = w.t0 + (s + 1) * dt
        inv_c = 1.0 if steps else 0.0
        pb_o = np.repeat(psi_f(it.bq_y, t)[:, None], M, axis=1)
        psi_o, phi_o, info_o = tr.step(psi_o, src(x, om_o, t, inv_c), pb_o, phi_o)
        pb_g = _dev(np.repeat(psi_f(y_g, t)[:, None], M, axis=1))
        phi_g, pv_g, psi_g, info_g = P.step(_dev(src(x, om_g, t, inv_c)), pb_g)
        pv_o = tr.point_values(phi_o)
        e = (rel_l2(_cpu(phi_g), phi_o), rel_l2(_cpu(pv_g), pv_o), rel_l2(_cpu(psi_g), psi_o))
        print(f"step {s + 1}: phi {e[0]:.2e} point {e[1]:.2e} psi {e[2]:.2e} outer {info_g['outer_iters']} "
              f"(oracle {info_o['outer_iters']})", flush=True)
        out.append((e, info_g))
    P.close()
    return out


@pytest.mark.parametrize("kind,precision", [("cos", "fp64"), ("cos", "mixed"), ("wave", "fp64")])
def test_paper_mms_steady(kind, precision):
    _print_case("paper-mms-steady", kind=kind, precision=precision)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for e, info in _solve_pair(kind, 12, 8, precision=precision):
        assert info["converged"] == 1 and max(e) <= tol


@pytest.mark.parametrize("kind", ["cos", "wave"])
def test_paper_mms_backward_euler(kind):
    """Two backward-Euler steps from the exact state, time-dependent source and inflow."""
    _print_case("paper-mms-be", kind=kind)
    for e, info in _solve_pair(kind, 10, 8, steps=2, dt=0.1):
        assert info["converged"] == 1 and max(e) <= FP64_TOL


@pytest.mark.parametrize("kind", ["cos", "wave"])
def test_paper_mms_second_order_on_gpu(kind):
    """Sec. 5.1: second order in space, on uniform lattices up to 128^2."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    errs, hs = [], []
    for n in (16, 32, 64, 128):
        _print_case("paper-mms-order", kind=kind, n=n)
        w = W.config(6 if kind == "cos" else 7, n)
        x, dx = W.points_for(w)
        om, wq = mlpg.mlpg_angular_quadrature(2, 8)
        P = GpuProblem(x, W.radii_for(w, x, dx), w.lo, w.hi, fields=w.fields)
        P.integrate(1)
        P.assemble(om, wq, list(w.sigma_t), list(w.sigma_s), 0.0, dx)
        y, _ = P.boundary_points()
        pb = _dev(W.inflow_values(w, _cpu(y), om))
        phi, pv, _, info = P.step(_dev(W.source_values(w, x, om, w.t0)), pb, want_psi=False)
        assert info["converged"] == 1
        ex = 4.0 * np.pi * W.paper_mms_psi(w, x, w.t0)
        errs.append(float(np.abs(_cpu(pv) - ex).sum() / ex.sum()))
        hs.append(dx)
        print(f"n={n} rel error {errs[-1]:.3e}", flush=True)
        P.close()
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert abs(slope - GOLD["mms_spatial_order_linear_rk"]) <= GOLD["order_tolerance"], (errs, slope)
