"""Graph replay of the inner solves' restart cycles and the sweep's launch-shape autotuning.

* A solve whose restart cycles are captured once and replayed from HIP graphs
  gives the same fields bit for bit, and the same iteration counts, as one
  launched kernel by kernel -- FP64 and mixed, point and patch
  preconditioning, backward-Euler steps that replay cached graphs with
  eager work of the caller in between.
* The autotuner records the launch shape it picked for the problem's shape;
  every shape gives the same sums in the same order, so a solve with the
  tuned shape equals one with the built-in shape bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from tests._cases import lattice_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02205_amd import mlpg
    mlpg.lib()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _problem(n, M, precision, a0=100.0):
    """A lattice problem, integrated and assembled once."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    x, R, dx = lattice_case(n)
    P = GpuProblem(x, R, (0, 0), (1, 1))
    P.integrate(1)
    om, wq = mlpg.mlpg_angular_quadrature(2, M)
    P.assemble(om, wq, [1.0], [0.5], a0, dx, precision=precision)
    return x, om, P


def _run(P, x, om, precond, graphs, steps=2):
    """BE steps from the same initial state on an existing problem (one set of integrated
    blocks: the integration's atomics make separately built problems differ in the last bits)."""
    from paper_2008_02205_amd import mlpg
    P.set_state(_dev(W.mms_sin_psi(x, om, 0.0)))
    o = mlpg.mlpg_default_opts()
    o.graphs = 1 if graphs else 0
    o.precond = mlpg.MLPG_PRECOND_PATCH if precond == "patch" else mlpg.MLPG_PRECOND_JACOBI
    out = []
    for s in range(1, steps + 1):
        q = _dev(W.mms_sin_source(x, om, s * 0.01, 1.0, 0.5))
        phi, pv, psi, info = P.step(q, None, o)
        # eager work of the caller between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        out.append((phi.cpu().numpy(), psi.cpu().numpy(), info["inner_iters"], info["outer_iters"], float(junk)))
    return out


@pytest.mark.parametrize("precision,precond", [("fp64", "jacobi"), ("mixed", "jacobi"), ("fp64", "patch"),
                                               ("mixed", "patch")])
def test_graph_replay_equals_eager_launches(precision, precond):
    from paper_2008_02205_amd import mlpg
    print(f"[case] graphs precision={precision} precond={precond}", flush=True)
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    x, om, P = _problem(16, 64, prec)
    eager = _run(P, x, om, precond, graphs=False, steps=3)
    graph = _run(P, x, om, precond, graphs=True, steps=3)
    again = _run(P, x, om, precond, graphs=True, steps=3)   # replays of the cached graphs only
    P.close()
    for (pe, se, ie, oe, _), (pg, sg, ig, og, _), (pa, sa, ia, oa, _) in zip(eager, graph, again):
        assert np.array_equal(pe, pg) and np.array_equal(se, sg)
        assert np.array_equal(pe, pa) and np.array_equal(se, sa)
        assert ie == ig == ia and oe == og == oa


def test_autotuned_shape_is_recorded_and_exact():
    from paper_2008_02205_amd import mlpg
    print("[case] autotune", flush=True)
    mlpg.mlpg_set_autotune(2)     # empty table
    mlpg.mlpg_set_autotune(0)     # built-in shape
    x, om, P = _problem(14, 96, mlpg.MLPG_FP64)
    ref = _run(P, x, om, "jacobi", graphs=True, steps=1)
    assert mlpg.mlpg_get_tuning() == []
    mlpg.mlpg_set_autotune(1)
    got = _run(P, x, om, "jacobi", graphs=True, steps=1)
    P.close()
    table = mlpg.mlpg_get_tuning()
    print(table, flush=True)
    e = [t for t in table if t["n"] == 196 and t["n_ord"] == 96 and t["streams"] == 6 and t["value_bytes"] == 8]
    assert len(e) == 1
    e = e[0]
    assert e["waves_per_block"] in (2, 4, 8) and e["items_per_wave"] in (1, 2) and e["xcd_split"] in (1, 8)
    assert 0 < e["us_best"] <= e["us_default"]
    assert np.array_equal(ref[0][0], got[0][0]) and np.array_equal(ref[0][1], got[0][1])
    # a small ordinate count tunes the row-group kernel's block size
    x, om, P = _problem(10, 16, mlpg.MLPG_MIXED)
    _run(P, x, om, "jacobi", graphs=True, steps=1)
    P.close()
    small = [t for t in mlpg.mlpg_get_tuning() if t["n_ord"] == 16]
    assert small and all(t["threads"] in (128, 256, 512) for t in small)
