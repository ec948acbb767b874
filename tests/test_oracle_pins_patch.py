"""Pins of the oracle's patch block-Jacobi preconditioner of the inner solves.

Sec. 4.2 preconditions every transport operator L_m (the paper with ILUT);
the preconditioner changes iteration counts, never the converged solution.
Pinned here against what fixes it independently:

* the patches of a jittered cell-centred lattice are exactly its 2 x 2
  (2 x 2 x 2 in 3D) blocks of lattice cells, found from each point's lattice
  cell (the jitter stays inside it), in grid order;
* a grid cell with more points than the cap splits into consecutive chunks;
* z = M^-1 v solves L_m[P, P] z_P = v_P on every patch against the dense
  operator assembled column by column from the oracle's own sweeps (a
  library solve of each block);
* a solve with the patch preconditioner equals the point-Jacobi one and the
  dense direct solve of the coupled system;
* on a coarse Poisson-disk set whose operator has rows with negative
  diagonal entries, point-Jacobi GMRES(30) stalls while the patch
  preconditioner converges.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _transport(n, dim=2, M=4, jitter=0.2, sig_t=1.0, sig_s=0.5, a0=0.0, precond="patch", rfac=2.0):
    lo, hi = (0.0,) * dim, (1.0,) * dim
    x, dx = W.jittered_lattice((n,) * dim, lo, hi, jitter, 13)
    R = np.full(x.shape[0], rfac * dx)
    g = oracle.geometry(x, R, lo, hi)
    it = oracle.integrate(g, 1)
    om, wq = oracle.angular_quadrature(dim, M)
    tr = oracle.Transport(it, om, wq, sig_t, sig_s, a0, dx, oracle.SolveOpts(precond=precond))
    return x, dx, g, it, om, wq, tr


def _expected_lattice_patches(x, dx, dim):
    k = np.floor(x / dx).astype(int) // 2          # the 2^dim block of lattice cells
    nb = int(k.max()) + 1
    key = np.zeros(x.shape[0], dtype=np.int64)
    for a in range(dim):
        key = key * nb + k[:, a]
    order = np.lexsort((np.arange(x.shape[0]), key))
    groups = [order[key[order] == v] for v in np.unique(key)]
    return groups


@pytest.mark.parametrize("n,dim", [(8, 2), (7, 2), (4, 3)])
def test_lattice_patches_are_blocks_of_lattice_cells(n, dim):
    x, dx, g, it, om, wq, tr = _transport(n, dim=dim, M=4 if dim == 2 else 6)
    start, pts = tr.patches()
    got = [pts[start[p]:start[p + 1]] for p in range(len(start) - 1)]
    want = _expected_lattice_patches(x, dx, dim)
    assert len(got) == len(want)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    if n % 2 == 0:
        assert all(len(a) == 2 ** dim for a in got)
    assert np.array_equal(np.sort(pts), np.arange(x.shape[0]))


def test_crowded_cell_splits_into_chunks_of_sixteen():
    """40 points in one grid cell and one elsewhere: chunks 16, 16, 8 in increasing index."""
    rs = np.random.default_rng(3)
    n = 41
    # grid side 2 sqrt(1/41) ~ 0.31: the corner cell [0, 0.31)^2 takes the cluster
    x = np.vstack([rs.uniform(0.01, 0.2, (40, 2)), [[0.9, 0.9]]])
    perm = rs.permutation(n)
    x = x[perm]
    R = np.full(n, 0.3)
    g = oracle.geometry(x, R, (0, 0), (1, 1))
    it = oracle.integrate(g, 0)
    om, wq = oracle.angular_quadrature(2, 2)
    tr = oracle.Transport(it, om, wq, 1.0, 0.0, 0.0, 0.1, oracle.SolveOpts(precond="patch"))
    start, pts = tr.patches()
    sizes = np.diff(start)
    assert list(sizes) == [16, 16, 8, 1]
    cluster = np.sort(np.where(perm < 40)[0])
    assert np.array_equal(pts[:40], cluster)
    assert pts[40] == np.where(perm == 40)[0][0]


def _dense_L(tr, n):
    M = tr.M
    Ls = np.zeros((M, n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Ls[:, :, j] = tr.apply("L", e).T
    return Ls


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 3)])
def test_patch_solve_inverts_each_diagonal_block(dim, n):
    x, dx, g, it, om, wq, tr = _transport(n, dim=dim, M=4 if dim == 2 else 6, a0=5.0)
    Ls = _dense_L(tr, g.n)
    start, pts = tr.patches()
    v = np.random.default_rng(9).uniform(-1, 1, g.n)
    for m in range(tr.M):
        z = tr.patch_precond(m, v)
        for p in range(len(start) - 1):
            P = pts[start[p]:start[p + 1]]
            B = Ls[m][np.ix_(P, P)]
            assert np.allclose(z[P], np.linalg.solve(B, v[P]), rtol=1e-12, atol=1e-14 * np.abs(z).max())


def test_patch_and_point_jacobi_reach_the_same_solution():
    x, dx, g, it, om, wq, trp = _transport(12, M=8, sig_s=0.9)
    trj = oracle.Transport(it, om, wq, 1.0, 0.9, 0.0, dx, oracle.SolveOpts(precond="jacobi"))
    q = np.ones((g.n, 8))
    psi_p, phi_p, ip = trp.step(None, q)
    psi_j, phi_j, ij = trj.step(None, q)
    assert ip["inner_res_max"] <= 1e-13 and ij["inner_res_max"] <= 1e-13
    assert np.linalg.norm(phi_p - phi_j) <= 1e-11 * np.linalg.norm(phi_j)
    assert np.linalg.norm(psi_p - psi_j) <= 1e-11 * np.linalg.norm(psi_j)
    # fewer Arnoldi steps per inner solve
    assert ip["inner_iters"] < ij["inner_iters"]


def test_patch_preconditioned_step_matches_dense_direct_solve():
    x, dx, g, it, om, wq, tr = _transport(6, M=4, sig_s=0.8, a0=10.0)
    n, M = g.n, 4
    Ls = _dense_L(tr, n)
    MSs = np.zeros((M, n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        MSs[:, :, j] = tr.apply("MS", e).T
    A = np.zeros((n * M, n * M))
    for m in range(M):
        A[m * n:(m + 1) * n, m * n:(m + 1) * n] += Ls[m]
        for mp in range(M):
            A[m * n:(m + 1) * n, mp * n:(mp + 1) * n] -= MSs[m] * wq[mp]
    rs = np.random.default_rng(2)
    psi_prev = rs.uniform(0, 1, (n, M))
    q = rs.uniform(0, 1, (n, M))
    F = tr.rhs(psi_prev, q, None)
    sol = np.linalg.solve(A, F.T.reshape(-1)).reshape(M, n).T
    psi, phi, info = tr.step(psi_prev, q, None)
    assert np.linalg.norm(psi - sol) <= 1e-10 * np.linalg.norm(sol)


@pytest.mark.slow
def test_patch_converges_where_point_jacobi_stalls():
    """Coarse Poisson-disk beam problem (211 points, 256 ordinates): after six backward-Euler
    steps, ordinate 104's operator has negative diagonal entries and point-Jacobi GMRES(30) stalls
    on the next right-hand side; the patch preconditioner solves it."""
    w = W.config(4)
    x = W.poisson_disk(w.lo, w.hi, 0.08, w.seed)
    dx = math.sqrt(2.0 / x.shape[0])
    R = W.radii_for(w, x, dx)
    om, wq = oracle.angular_quadrature(2, w.n_ord, w.ord_kind)
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, 1, regions=w.regions, n_mat=2)
    trp = oracle.Transport(it, om, wq, w.sigma_t, w.sigma_s, w.inv_c_dt, dx, oracle.SolveOpts(precond="patch"))
    trj = oracle.Transport(it, om, wq, w.sigma_t, w.sigma_s, w.inv_c_dt, dx, oracle.SolveOpts(precond="jacobi"))
    psi = W.initial_psi(w, x, om)
    phi = psi @ wq
    pb = W.inflow_values(w, it.bq_y, om)
    for s in range(1, 7):
        psi, phi, info = trp.step(psi, W.source_values(w, x, om, s * w.dt), pb, phi)
        assert info["inner_res_max"] <= 1e-13
    F = trp.rhs(psi, W.source_values(w, x, om, 7 * w.dt), pb)
    _, its_j, res_j = trj.inner_solve(F, 104, 105)
    _, its_p, res_p = trp.inner_solve(F, 104, 105)
    assert res_j > 0.1 and its_j == 3000
    assert res_p <= 1e-13 and its_p < 3000
