"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Integer and index work (neighbour lists, pattern) must match bit for bit.
Floating point: per-stage values within 1e-12 relative (FP64 atomics sum in
a nondeterministic order, so rounding differs), single operator sweeps
within 1e-13, and every solved field (Phi, phi(x_i), Psi) within 1e-10
relative L2, the FP64 bar of the method's specification.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._cases import FP64_TOL, absorber_dir, lattice_case, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02205_amd import mlpg
    mlpg.lib()


def _gpu_problem(x, R, lo, hi, regions=()):
    from paper_2008_02205_amd.problem import GpuProblem
    return GpuProblem(x, R, lo, hi, regions)


def _cpu(t):
    return t.detach().cpu().numpy()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu_quadrature(M, kind="product"):
    """The library's own angular quadrature (the oracle builds its own)."""
    from paper_2008_02205_amd import mlpg
    code = {"product": mlpg.MLPG_QUAD_PRODUCT, "beam-dense": mlpg.MLPG_QUAD_BEAM_DENSE}[kind]
    return mlpg.mlpg_angular_quadrature(2, M, code)


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("n", [7, 16, 33])
def test_neighbors_pattern_cells_blocks(n):
    _print_case("stages", n=n)
    x, R, dx = lattice_case(n)
    g = oracle.geometry(x, R, (0, 0), (1, 1))
    it = oracle.integrate(g, 1)
    P = _gpu_problem(x, R, (0, 0), (1, 1))
    assert np.array_equal(_cpu(P.nbr_off), g.nb_off)
    assert np.array_equal(_cpu(P.nbr_idx), g.nb_idx)
    from paper_2008_02205_amd import mlpg
    V = _cpu(mlpg.mlpg_get_volumes(P.h, P.n))
    assert np.abs(V - g.V).max() <= 1e-13 * g.V.max()
    assert P.info["oversize_cells"] == int(np.sum(g.cells.rho > R))
    P.integrate(1)
    info = P.info
    assert info["missing_pairs"] == 0 and info["fallback_qps"] == it.fallbacks
    row_off, col = mlpg.mlpg_get_pattern(P.h, P.n, info["nnz"])
    assert np.array_equal(_cpu(row_off), g.row_off)
    assert np.array_equal(_cpu(col), g.col)
    blocks, E = mlpg.mlpg_get_blocks(P.h, info["n_blocks"], info["nnz"])
    blocks, E = _cpu(blocks), _cpu(E)
    names = oracle.block_names(2, 1)
    for b, name in enumerate(names):
        ref = it.blocks[b]
        scale = np.abs(ref).max()
        assert np.abs(blocks[b] - ref).max() <= 1e-12 * scale, name
    assert np.abs(E - it.E).max() <= 1e-12 * np.abs(it.E).max()
    # boundary quadrature points: same set (order may differ)
    y, face = P.boundary_points()
    y, face = _cpu(y), _cpu(face)
    assert y.shape[0] == it.nbq
    ka = np.lexsort((it.bq_y[:, 1], it.bq_y[:, 0], it.bq_face))
    kb = np.lexsort((y[:, 1], y[:, 0], face))
    assert np.array_equal(face[kb], it.bq_face[ka])
    assert np.abs(y[kb] - it.bq_y[ka]).max() <= 1e-14
    P.close()


@pytest.mark.parametrize("order", [0, 2])
def test_blocks_other_rk_orders(order):
    _print_case("rk-order", order=order)
    x, R, dx = lattice_case(12, rfac=2.5)
    g = oracle.geometry(x, R, (0, 0), (1, 1))
    it = oracle.integrate(g, order)
    P = _gpu_problem(x, R, (0, 0), (1, 1))
    P.integrate(order)
    from paper_2008_02205_amd import mlpg
    blocks, E = mlpg.mlpg_get_blocks(P.h, P.info["n_blocks"], P.info["nnz"])
    blocks = _cpu(blocks)
    # Both sides drop an order at a quadrature point when a Cholesky pivot of
    # the moment matrix falls below 1e-6 of its largest diagonal entry; a tie
    # would need a pivot within rounding of that bound.  Here both take the
    # same decisions (equal counts), and then every entry must agree.
    assert P.info["fallback_qps"] == it.fallbacks
    # quadratic moment matrices reach condition numbers near 1e6, which turns
    # summation-order differences into ~1e-10 relative differences
    tol = 1e-12 if order < 2 else 1e-9
    for b in range(blocks.shape[0]):
        d = np.abs(blocks[b] - it.blocks[b]) / np.abs(it.blocks[b]).max()
        print(f"block {b}: max rel diff {d.max():.2e}", flush=True)
        assert d.max() <= tol, b
    n = P.n
    cols = g.col
    rows = np.repeat(np.arange(n), np.diff(g.row_off))
    itol = 1e-12 if order < 2 else 1e-9
    assert abs(blocks[0].sum() - 1.0) <= itol
    for a in range(2):
        assert np.abs(np.bincount(cols, blocks[1 + a], n)).max() <= itol
        if order >= 1:   # linear reproduction: sum_i D^a[i,j] x_i^a = sum_i Mass[i,j]
            lhs = np.bincount(cols, blocks[1 + a] * x[rows, a], n)
            assert np.abs(lhs - np.bincount(cols, blocks[0], n)).max() <= itol
    P.close()


@pytest.mark.parametrize("M,kind", [(2, "product"), (16, "product"), (64, "product"), (256, "beam-dense")])
def test_angular_quadrature_matches(M, kind):
    om, w = _gpu_quadrature(M, kind)
    om_o, w_o = oracle.angular_quadrature(2, M, kind)
    # a few ulps of azimuths up to pi
    assert np.abs(om - om_o).max() <= 8 * np.finfo(np.float64).eps and np.abs(w - w_o).max() <= 1e-14


def test_single_operator_sweeps():
    _print_case("spmv", n=20, M=16)
    x, R, dx = lattice_case(20)
    g = oracle.geometry(x, R, (0, 0), (1, 1))
    it = oracle.integrate(g, 1)
    om, w = oracle.angular_quadrature(2, 16)
    tr = oracle.Transport(it, om, w, 1.3, 0.6, 7.0, dx)
    P = _gpu_problem(x, R, (0, 0), (1, 1))
    P.integrate(1)
    P.assemble(*_gpu_quadrature(16), [1.3], [0.6], 7.0, dx)
    from paper_2008_02205_amd import mlpg
    X = np.random.default_rng(4).uniform(-1, 1, (g.n, 16))
    Xd = torch.from_numpy(X).cuda()
    for name, code in (("L", mlpg.MLPG_OP_L), ("T", mlpg.MLPG_OP_T), ("MS", mlpg.MLPG_OP_MS),
                       ("MD", mlpg.MLPG_OP_SRC)):
        Y = _cpu(mlpg.mlpg_apply(P.h, code, Xd))
        ref = tr.apply(name, X)
        assert rel_l2(Y, ref) <= 1e-13, name
    P.close()


def _solve_both(n, M, sig_t, sig_s, inv_c_dt, steps, q_fn, psib_fn=None, psi0_fn=None, jitter=0.2,
                ord_kind="product", omega=None, w=None):
    x, R, dx = lattice_case(n, jitter=jitter)
    g = oracle.geometry(x, R, (0, 0), (1, 1))
    it = oracle.integrate(g, 1)
    if omega is None:
        omega, w = oracle.angular_quadrature(2, M, ord_kind)
        om_g, w_g = _gpu_quadrature(M, ord_kind)
    else:   # a user-given ordinate set is an input of both sides
        om_g, w_g = omega, w
    tr = oracle.Transport(it, omega, w, sig_t, sig_s, inv_c_dt, dx)
    P = _gpu_problem(x, R, (0, 0), (1, 1))
    P.integrate(1)
    P.assemble(om_g, w_g, [sig_t], [sig_s], inv_c_dt, dx)
    y_g, f_g = P.boundary_points()
    psi_o = psi0_fn(x, omega) if psi0_fn else None
    phi_o = psi_o @ w if psi_o is not None else None
    if psi0_fn:
        P.set_state(torch.from_numpy(np.ascontiguousarray(psi0_fn(x, om_g))).cuda())
    out = []
    for s in range(1, steps + 1):
        t = s * (1.0 / inv_c_dt if inv_c_dt > 0 else 0.0)
        pb_o = psib_fn(it.bq_y, omega, t) if psib_fn else None
        psi_o, phi_o, info_o = tr.step(psi_o, q_fn(x, omega, t), pb_o, phi_o)
        pb_g = torch.from_numpy(np.ascontiguousarray(psib_fn(_cpu(y_g), om_g, t))).cuda() if psib_fn else None
        phi_g, pv_g, psi_g, info_g = P.step(torch.from_numpy(np.ascontiguousarray(q_fn(x, om_g, t))).cuda(), pb_g)
        out.append((phi_o, tr.point_values(phi_o), psi_o, _cpu(phi_g), _cpu(pv_g), _cpu(psi_g), info_o, info_g))
    P.close()
    return out


def _assert_fields(res):
    for (phi_o, pv_o, psi_o, phi_g, pv_g, psi_g, info_o, info_g) in res:
        assert info_g["converged"] == 1
        assert rel_l2(phi_g, phi_o) <= FP64_TOL
        assert rel_l2(pv_g, pv_o) <= FP64_TOL
        assert rel_l2(psi_g, psi_o) <= FP64_TOL


@pytest.mark.parametrize("n,M", [(9, 16), (16, 16), (32, 16)])
def test_steady_uniform_source_solve(n, M):
    """cfg-1 family: steady, sigma_t = 1, sigma_s = 0.5, q = 1, vacuum (32 x 32 is the full size)."""
    _print_case("steady", n=n, M=M)
    res = _solve_both(n, M, 1.0, 0.5, 0.0, 1, lambda x, om, t: np.ones((x.shape[0], om.shape[0])))
    _assert_fields(res)


def test_backward_euler_mms_steps():
    """cfg-2 family at reduced size: 64 ordinates, manufactured source, backward Euler."""
    _print_case("mms-be", n=16, M=64)
    res = _solve_both(16, 64, 1.0, 0.5, 100.0, 2, lambda x, om, t: W.mms_sin_source(x, om, t, 1.0, 0.5),
                      psi0_fn=lambda x, om: W.mms_sin_psi(x, om, 0.0))
    _assert_fields(res)


def test_absorber_with_inflow_single_ordinate():
    """One oblique ordinate, pure absorber, inflow psi_b = exp(-sigma x / mu) on inflow faces."""
    _print_case("absorber", n=17, M=1)
    mu, eta = absorber_dir()
    om = np.array([[mu, eta]]); w = np.array([4 * np.pi])
    res = _solve_both(17, 1, 2.0, 0.0, 0.0, 1, lambda x, o, t: np.zeros((x.shape[0], 1)),
                      psib_fn=lambda y, o, t: W.absorber_psi(y, mu, 2.0)[:, None], omega=om, w=w)
    _assert_fields(res)
    assert res[0][7]["outer_iters"] <= 1


def test_unjittered_lattice_and_ragged_sizes():
    """Exact lattice (degenerate co-circular vertices) with an ordinate count that leaves partial waves."""
    _print_case("lattice-ragged", n=11, M=6)
    res = _solve_both(11, 6, 1.0, 0.3, 3.0, 1, lambda x, om, t: np.ones((x.shape[0], om.shape[0])), jitter=0.0)
    _assert_fields(res)


def test_state_roundtrip_and_errors():
    from paper_2008_02205_amd import mlpg
    x, R, dx = lattice_case(8)
    P = _gpu_problem(x, R, (0, 0), (1, 1))
    with pytest.raises(mlpg.MlpgError) as e:
        mlpg.mlpg_solve(P.h, torch.zeros((P.n, 4), dtype=torch.float64, device="cuda"))
    assert e.value.code == -7
    with pytest.raises(mlpg.MlpgError):
        mlpg.mlpg_integrate(P.h, 3)
    P.integrate(1)
    om, w = _gpu_quadrature(4)
    P.assemble(om, w, [1.0], [0.2], 0.0, dx)
    psi = torch.rand((P.n, 4), dtype=torch.float64, device="cuda")
    P.set_state(psi)
    psi2, phi2 = mlpg.mlpg_get_state(P.h, P.n, 4)
    assert torch.equal(psi, psi2)
    assert torch.allclose(phi2, psi @ torch.from_numpy(w).cuda(), rtol=1e-14, atol=0)
    # an inner solve at its iteration limit ends the step at once: MLPG_ERR_NOT_CONVERGED
    # after the first batched inner solve, no outer iteration, info filled in
    o = mlpg.mlpg_default_opts()
    o.max_inner = 1
    phi, pv, ps, info = mlpg.mlpg_solve(P.h, torch.ones((P.n, 4), dtype=torch.float64, device="cuda"), None, o,
                                        raise_on_error=False)
    assert info["status"] == -4 and info["converged"] == 0
    assert info["inner_solves"] == 1 and info["outer_iters"] == 0 and info["inner_iters"] <= 4
    assert "max_inner" in mlpg.last_error()
    # the state is left as it was
    psi3, _ = mlpg.mlpg_get_state(P.h, P.n, 4)
    assert torch.equal(psi, psi3)
    # the outer limit alone: outputs of the last iterate, NOT_CONVERGED
    o = mlpg.mlpg_default_opts()
    o.max_outer = 1
    o.tol_outer = 1e-300
    phi, pv, ps, info = mlpg.mlpg_solve(P.h, torch.ones((P.n, 4), dtype=torch.float64, device="cuda"), None, o,
                                        raise_on_error=False)
    assert info["status"] == -4 and info["converged"] == 0 and info["outer_iters"] == 1
    assert bool(torch.isfinite(phi).all())
    P.close()


def test_malformed_overlap_lists_are_rejected():
    """Caller-supplied lists are validated before any kernel reads them."""
    from paper_2008_02205_amd import mlpg
    x, R, dx = lattice_case(6)
    off, idx = oracle.neighbors(x, R)
    n = x.shape[0]
    cases = {}
    bad = idx.copy(); bad[3] = n + 5; cases["index out of range"] = (off, bad)
    bad = idx.copy(); bad[off[2]] = 2; cases["self index"] = (off, bad)
    bad = idx.copy(); bad[off[4]], bad[off[4] + 1] = bad[off[4] + 1], bad[off[4]]; cases["unsorted"] = (off, bad)
    boff = off.copy(); boff[5] = boff[6] + 1; cases["decreasing offsets"] = (boff, idx)
    boff = off.copy(); boff[0] = 1; cases["offsets not from 0"] = (boff, idx)
    for name, (o_, i_) in cases.items():
        with pytest.raises(mlpg.MlpgError) as e:
            mlpg.mlpg_geometry(_dev(x), _dev(R), _dev(o_), _dev(i_), (0, 0), (1, 1))
        assert e.value.code == -1, name
        assert "malformed overlap lists" in str(e.value), name
    # a list with a neighbour missing on both sides passes the check but loses
    # co-active pairs: the integration refuses it
    i, j = 10, int(idx[off[10]])
    keep = np.ones(idx.size, dtype=bool)
    keep[off[i]] = False
    keep[off[j] + int(np.searchsorted(idx[off[j]:off[j + 1]], i))] = False
    cnt = np.diff(off) - np.bincount(np.repeat(np.arange(n), np.diff(off))[~keep], minlength=n)
    off2 = np.concatenate(([0], np.cumsum(cnt))).astype(np.int64)
    h = mlpg.mlpg_geometry(_dev(x), _dev(R), _dev(off2), _dev(idx[keep]), (0, 0), (1, 1))
    with pytest.raises(mlpg.MlpgError) as e:
        mlpg.mlpg_integrate(h, 1)
    assert e.value.code == -1 and "missing from the overlap lists" in str(e.value)
    mlpg.mlpg_destroy(h)


def _solve_mixed_vs_oracle(n, M, sig_t, sig_s, inv_c_dt, steps, q_fn, psi0_fn=None):
    from paper_2008_02205_amd import mlpg
    x, R, dx = lattice_case(n)
    g = oracle.geometry(x, R, (0, 0), (1, 1))
    it = oracle.integrate(g, 1)
    omega, w = oracle.angular_quadrature(2, M)
    om_g, w_g = _gpu_quadrature(M)
    tr = oracle.Transport(it, omega, w, sig_t, sig_s, inv_c_dt, dx)
    P = _gpu_problem(x, R, (0, 0), (1, 1))
    P.integrate(1)
    P.assemble(om_g, w_g, [sig_t], [sig_s], inv_c_dt, dx, precision=mlpg.MLPG_MIXED)
    psi_o = psi0_fn(x, omega) if psi0_fn else None
    phi_o = psi_o @ w if psi_o is not None else None
    if psi0_fn:
        P.set_state(torch.from_numpy(np.ascontiguousarray(psi0_fn(x, om_g))).cuda())
    out = []
    for s in range(1, steps + 1):
        t = s * (1.0 / inv_c_dt if inv_c_dt > 0 else 0.0)
        psi_o, phi_o, _ = tr.step(psi_o, q_fn(x, omega, t), None, phi_o)
        phi_g, pv_g, psi_g, info = P.step(torch.from_numpy(np.ascontiguousarray(q_fn(x, om_g, t))).cuda())
        out.append((rel_l2(_cpu(phi_g), phi_o), rel_l2(_cpu(pv_g), tr.point_values(phi_o)),
                    rel_l2(_cpu(psi_g), psi_o), info))
    P.close()
    return out


MIXED_TOL = 1e-8   # relative L2 bar of the mixed path after FP64 refinement


@pytest.mark.parametrize("n,M", [(16, 16), (32, 16)])
def test_mixed_precision_steady(n, M):
    """FP32 SpMV/basis inside FP64 refinement matches the FP64 oracle (cfg-1 family)."""
    _print_case("mixed-steady", n=n, M=M)
    for ephi, epv, epsi, info in _solve_mixed_vs_oracle(
            n, M, 1.0, 0.5, 0.0, 1, lambda x, om, t: np.ones((x.shape[0], om.shape[0]))):
        print(f"mixed steady: phi {ephi:.2e} psi {epsi:.2e} refinements {info['refinements']}", flush=True)
        assert info["converged"] == 1 and info["refinements"] > 0
        assert ephi <= MIXED_TOL and epv <= MIXED_TOL and epsi <= MIXED_TOL


def test_mixed_precision_backward_euler():
    _print_case("mixed-be", n=16, M=64)
    for ephi, epv, epsi, info in _solve_mixed_vs_oracle(
            16, 64, 1.0, 0.5, 100.0, 2, lambda x, om, t: W.mms_sin_source(x, om, t, 1.0, 0.5),
            psi0_fn=lambda x, om: W.mms_sin_psi(x, om, 0.0)):
        print(f"mixed BE: phi {ephi:.2e} psi {epsi:.2e} refinements {info['refinements']}", flush=True)
        assert info["converged"] == 1
        assert ephi <= MIXED_TOL and epv <= MIXED_TOL and epsi <= MIXED_TOL
