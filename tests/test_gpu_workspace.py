"""Caller-owned stage workspaces on the GPU.

For every stage (geometry, integration, assembly, solve; FP64 and mixed, with
and without the patch preconditioner and the diffusion-synthetic
acceleration): a workspace of exactly the queried size works, a smaller one
fails with MLPG_ERR_WORKSPACE before anything is enqueued, and nothing is
written past the queried size (a sentinel tail stays intact) -- so the query
is the bytes the stage uses.  The solution computed in torch-owned
workspaces equals the one in library-allocated ones.  The state moves with
the assembly workspace.  Device memory outside the workspaces stays flat
across a whole problem.
"""
import numpy as np
import pytest

import oracle
from tests._cases import lattice_case, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SENTINEL = 0xA5
TAIL = 4096


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02205_amd import mlpg
    mlpg.lib()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _padded(nbytes):
    """A workspace of nbytes followed by a sentinel tail; returns (full buffer, exact view)."""
    from paper_2008_02205_amd import mlpg
    full = mlpg.workspace(nbytes + TAIL)
    full.fill_(SENTINEL)
    return full, full[:nbytes]


def _tail_intact(full, nbytes):
    torch.cuda.synchronize()
    return bool((full[nbytes:] == SENTINEL).all())


def _written(view):
    torch.cuda.synchronize()
    return bool((view != SENTINEL).any())


@pytest.mark.parametrize("precision,precond,accel", [("fp64", "jacobi", False), ("mixed", "patch", False),
                                                     ("fp64", "patch", True)])
def test_stage_queries_are_the_bytes_used(precision, precond, accel):
    from paper_2008_02205_amd import mlpg
    print(f"[case] workspace precision={precision} precond={precond} accel={accel}", flush=True)
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    x, R, dx = lattice_case(14)
    n = x.shape[0]
    xd, Rd = _dev(x), _dev(R)
    off, total = mlpg.mlpg_neighbors_count(xd, Rd)
    idx = mlpg.mlpg_neighbors_fill(xd, Rd, off, total)
    lo, hi = (0.0, 0.0), (1.0, 1.0)
    # geometry
    g_need = mlpg.mlpg_geometry_workspace_bytes(2, n, total, lo, hi)
    small = mlpg.workspace(g_need - 256)
    with pytest.raises(mlpg.MlpgError) as e:
        mlpg.mlpg_geometry(xd, Rd, off, idx, lo, hi, ws=small)
    assert e.value.code == -6 and "needs" in str(e.value)
    g_full, g_ws = _padded(g_need)
    h = mlpg.mlpg_geometry(xd, Rd, off, idx, lo, hi, ws=g_ws)
    assert _written(g_ws) and _tail_intact(g_full, g_need)
    # integration
    i_need = mlpg.mlpg_integrate_workspace_bytes(h, 1)
    with pytest.raises(mlpg.MlpgError) as e:
        mlpg.mlpg_integrate(h, 1, ws=mlpg.workspace(i_need - 256))
    assert e.value.code == -6
    i_full, i_ws = _padded(i_need)
    mlpg.mlpg_integrate(h, 1, ws=i_ws)
    assert _written(i_ws) and _tail_intact(i_full, i_need)
    # assembly
    M = 16
    om, wq = mlpg.mlpg_angular_quadrature(2, M)
    tau = torch.full((n,), dx, dtype=torch.float64, device="cuda")
    a_need = mlpg.mlpg_assemble_workspace_bytes(h, M, prec)
    with pytest.raises(mlpg.MlpgError) as e:
        mlpg.mlpg_assemble(h, om, wq, [1.0], [0.9], 0.0, tau, prec, ws=mlpg.workspace(a_need - 256))
    assert e.value.code == -6
    a_full, a_ws = _padded(a_need)
    mlpg.mlpg_assemble(h, om, wq, [1.0], [0.9], 0.0, tau, prec, ws=a_ws)
    assert _written(a_ws) and _tail_intact(a_full, a_need)
    # solve
    o = mlpg.mlpg_default_opts()
    o.precond = mlpg.MLPG_PRECOND_PATCH if precond == "patch" else mlpg.MLPG_PRECOND_JACOBI
    if accel:
        o.accel = mlpg.MLPG_ACCEL_DSA
    s_need = mlpg.mlpg_solve_workspace_bytes(h, o)
    q = torch.ones((n, M), dtype=torch.float64, device="cuda")
    with pytest.raises(mlpg.MlpgError) as e:
        mlpg.mlpg_solve(h, q, None, o, ws=mlpg.workspace(s_need - 256))
    assert e.value.code == -6
    s_full, s_ws = _padded(s_need)
    phi, pv, psi, info = mlpg.mlpg_solve(h, q, None, o, ws=s_ws)
    assert info["converged"] == 1
    assert _written(s_ws) and _tail_intact(s_full, s_need)
    # every other workspace still untouched past its size after the solve
    assert _tail_intact(g_full, g_need) and _tail_intact(i_full, i_need) and _tail_intact(a_full, a_need)
    # the same problem with library-allocated workspaces
    h2 = mlpg.mlpg_geometry(xd, Rd, off, idx, lo, hi)
    mlpg.mlpg_integrate(h2, 1)
    mlpg.mlpg_assemble(h2, om, wq, [1.0], [0.9], 0.0, tau, prec)
    phi2, pv2, psi2, info2 = mlpg.mlpg_solve(h2, q, None, o)
    assert rel_l2(phi.cpu().numpy(), phi2.cpu().numpy()) <= 1e-12
    assert rel_l2(psi.cpu().numpy(), psi2.cpu().numpy()) <= 1e-12
    mlpg.mlpg_destroy(h)
    mlpg.mlpg_destroy(h2)


def test_state_follows_the_assembly_workspace():
    """Re-assembling into a new workspace carries Psi, Phi over; into the same one keeps them in place."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    x, R, dx = lattice_case(10)
    P = GpuProblem(x, R, (0, 0), (1, 1))
    P.integrate(1)
    om, wq = mlpg.mlpg_angular_quadrature(2, 8)
    P.assemble(om, wq, [1.0], [0.5], 10.0, dx)
    psi = torch.rand((P.n, 8), dtype=torch.float64, device="cuda")
    P.set_state(psi)
    old = P.ws["assemble"]
    tau = torch.full((P.n,), dx, dtype=torch.float64, device="cuda")
    # same workspace, new cross sections: state in place
    mlpg.mlpg_assemble(P.h, om, wq, [2.0], [0.5], 10.0, tau, mlpg.MLPG_FP64, ws=old)
    assert torch.equal(mlpg.mlpg_get_state(P.h, P.n, 8)[0], psi)
    # a different workspace: copied from the previous one
    new = mlpg.workspace(old.numel() + 512)
    mlpg.mlpg_assemble(P.h, om, wq, [2.0], [0.5], 10.0, tau, mlpg.MLPG_FP64, ws=new)
    P.ws["assemble"] = new
    old.fill_(0)
    assert torch.equal(mlpg.mlpg_get_state(P.h, P.n, 8)[0], psi)
    # a new ordinate count starts from zero
    om2, wq2 = mlpg.mlpg_angular_quadrature(2, 16)
    P.assemble(om2, wq2, [1.0], [0.5], 10.0, dx)
    assert float(mlpg.mlpg_get_state(P.h, P.n, 16)[0].abs().max()) == 0.0
    P.close()


def test_device_memory_is_the_workspaces():
    """Over a whole problem (geometry to a solve) the device memory in use beyond torch's own
    allocations does not grow: every byte the library touches comes from the workspaces."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    x, R, dx = lattice_case(24)
    om, wq = mlpg.mlpg_angular_quadrature(2, 32)

    def outside():
        torch.cuda.synchronize()
        free, total = torch.cuda.mem_get_info()
        return total - free - torch.cuda.memory_reserved()

    base = outside()
    P = GpuProblem(x, R, (0, 0), (1, 1))
    P.integrate(1)
    P.assemble(om, wq, [1.0], [0.5], 0.0, dx, precision=mlpg.MLPG_MIXED)
    o = mlpg.mlpg_default_opts()
    o.precond = mlpg.MLPG_PRECOND_PATCH
    phi, pv, psi, info = P.step(torch.ones((P.n, 32), dtype=torch.float64, device="cuda"), opts=o)
    assert info["converged"] == 1
    grown = outside() - base
    ws = sum(P.workspace_bytes().values())
    print(f"workspaces {ws / 2**20:.1f} MiB; device memory outside torch grew by {grown / 2**20:.2f} MiB",
          flush=True)
    # allow the runtime's own bookkeeping (a few MiB), far below the workspaces
    assert grown <= max(8 << 20, ws // 20)
    P.close()
