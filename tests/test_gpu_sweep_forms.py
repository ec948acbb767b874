"""The forms of the transport sweep give the same fields bit for bit.

Form 0 reads each row's stream values with scalar loads per wave; form 1
stages a round of rows' values and columns through LDS, two rounds deep, and
reads a round that does not fit its buffer from global memory instead.  Both
form every row's per-stream sums in the same order, so a solve is identical
whichever shape the launch-shape table holds.  Each shape is pinned with
mlpg_set_tuning (no autotuning): whole solves, FP64 and mixed precision (the
fused normalisation of the Arnoldi loop, the Jacobi-scaled first sweep, FP32
values), on a lattice whose rounds fit the LDS buffer (about 38 nonzeros per
row); and single applications of L on lattices whose rounds partly or wholly
overflow it (larger supports, about 60 and 77 per row).  Form 2 (more than 64
ordinates) takes 2 or 4 adjacent ordinates per lane, one vector gather per
nonzero, and is compared with form 0 the same way at 96, 128 and 256
ordinates, 6 streams (2D) and 10 (3D).  Form 0 is the form the parity tests
against the oracle cover with the built-in shape.
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
    yield
    mlpg.mlpg_set_autotune(2)
    mlpg.mlpg_set_autotune(1)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SHAPES = [
    {"form": 0, "waves_per_block": 4, "items_per_wave": 1, "xcd_split": 8},
    {"form": 0, "waves_per_block": 2, "items_per_wave": 2, "xcd_split": 1},
    {"form": 1, "waves_per_block": 4, "rounds": 1, "xcd_split": 8},
    {"form": 1, "waves_per_block": 4, "rounds": 4, "xcd_split": 8},
    {"form": 1, "waves_per_block": 8, "rounds": 2, "xcd_split": 8},
    {"form": 1, "waves_per_block": 8, "rounds": 3, "xcd_split": 1},
]


def _problem(side, rfac, M, prec):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    x, R, dx = lattice_case(side, rfac=rfac)
    P = GpuProblem(x, R, (0, 0), (1, 1))
    P.integrate(1)
    om, wq = mlpg.mlpg_angular_quadrature(2, M)
    P.assemble(om, wq, [1.0], [0.5], 100.0, dx, precision=prec)
    nnz = P.info["nnz"]
    print(f"[case] n={x.shape[0]} nnz={nnz} ({nnz / x.shape[0]:.1f} per row)", flush=True)
    return x, om, P


def _pin(sh, n, M, ns=6):
    from paper_2008_02205_amd import mlpg
    print(f"[case] shape {sh}", flush=True)
    for vb in (8, 4):
        mlpg.mlpg_set_tuning(dict(sh, n=n, n_ord=M, streams=ns, value_bytes=vb))
    table = [t for t in mlpg.mlpg_get_tuning() if t["n"] == n and t["n_ord"] == M]
    assert len(table) == 2 and all(t["form"] == sh["form"] for t in table)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep_forms_agree_bitwise_in_solves(precision):
    from paper_2008_02205_amd import mlpg
    print(f"[case] sweep forms in solves precision={precision}", flush=True)
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    M = 64
    x, om, P = _problem(15, 2.0, M, prec)
    n = x.shape[0]
    q = _dev(W.mms_sin_source(x, om, 0.01, 1.0, 0.5))
    psi0 = _dev(W.mms_sin_psi(x, om, 0.0))
    o = mlpg.mlpg_default_opts()
    mlpg.mlpg_set_autotune(2)
    mlpg.mlpg_set_autotune(0)
    ref = None
    for sh in SHAPES:
        _pin(sh, n, M)
        P.set_state(psi0)
        phi, pv, psi, info = P.step(q, None, o)
        got = (phi.cpu().numpy(), psi.cpu().numpy(), info["inner_iters"], info["outer_iters"])
        if ref is None:
            ref = got
            assert info["converged"]
            continue
        assert np.array_equal(ref[0], got[0]), sh
        assert np.array_equal(ref[1], got[1]), sh
        assert ref[2:] == got[2:], sh
    P.close()


@pytest.mark.parametrize("rfac", [2.5, 3.0])
def test_sweep_forms_agree_bitwise_when_rounds_overflow(rfac):
    from paper_2008_02205_amd import mlpg
    print(f"[case] sweep forms, single applications, rfac={rfac}", flush=True)
    M = 64
    x, om, P = _problem(15, rfac, M, mlpg.MLPG_FP64)
    n = x.shape[0]
    X = _dev(np.random.default_rng(5).standard_normal((n, M)))   # every column of L read
    mlpg.mlpg_set_autotune(2)
    mlpg.mlpg_set_autotune(0)
    ref = None
    for sh in SHAPES:
        _pin(sh, n, M)
        Y = mlpg.mlpg_apply(P.h, mlpg.MLPG_OP_L, X).cpu().numpy()
        if ref is None:
            ref = Y
            assert np.all(np.isfinite(Y)) and np.abs(Y).max() > 0
        else:
            assert np.array_equal(ref, Y), sh
    P.close()


def _wide_shapes(M):
    """Form 0 and the form-2 shapes that apply to M ordinates (2 per lane; 4 per lane at 256)."""
    shapes = [{"form": 0, "waves_per_block": 4, "items_per_wave": 1, "xcd_split": 8},
              {"form": 2, "ords_per_lane": 2, "waves_per_block": 4, "items_per_wave": 1, "xcd_split": 8},
              {"form": 2, "ords_per_lane": 2, "waves_per_block": 2, "items_per_wave": 2, "xcd_split": 1}]
    if M == 256:
        shapes.append({"form": 2, "ords_per_lane": 4, "waves_per_block": 4, "items_per_wave": 1, "xcd_split": 8})
    return shapes


def _wide_problem(dim, M, prec):
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    if dim == 2:
        x, R, dx = lattice_case(15, rfac=2.0)
        lo, hi = (0.0, 0.0), (1.0, 1.0)
    else:
        x, dx = W.jittered_lattice((5, 5, 5), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 0.2, 7)
        R = np.full(x.shape[0], 2.5 * dx)
        lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    P = GpuProblem(x, R, lo, hi)
    P.integrate(1)
    om, wq = mlpg.mlpg_angular_quadrature(dim, M)
    if dim == 2:
        P.assemble(om, wq, [1.0], [0.5], 100.0, dx, precision=prec)
    else:
        # steady, as the 3D parity tests (1/(c dt) = 100 with tau = h = 0.2 weights the streaming
        # term by 19 and the inner solves stagnate)
        P.assemble(om, wq, [1.0], [0.9], 0.0, dx, precision=prec)
    print(f"[case] dim={dim} n={x.shape[0]} M={M} nnz={P.info['nnz']}", flush=True)
    return x, om, P


@pytest.mark.parametrize("dim,M", [(2, 96), (2, 128), (2, 256), (3, 96)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_vector_form_agrees_bitwise_in_solves(dim, M, precision):
    """Form 2 (2 or 4 adjacent ordinates per lane, more than 64 ordinates) gives the solves of form 0 bit for
    bit: whole backward-Euler steps (the Jacobi-scaled first sweep, the fused normalisation, the refinement
    residual of the mixed path), 6 streams in 2D and 10 in 3D."""
    from paper_2008_02205_amd import mlpg
    print(f"[case] vector form in solves dim={dim} M={M} precision={precision}", flush=True)
    prec = mlpg.MLPG_FP64 if precision == "fp64" else mlpg.MLPG_MIXED
    x, om, P = _wide_problem(dim, M, prec)
    n = x.shape[0]
    rng = np.random.default_rng(11)
    o = mlpg.mlpg_default_opts()
    if dim == 2:
        q = _dev(rng.uniform(0.5, 1.5, (n, M)))
        psi0 = _dev(rng.uniform(0.0, 1.0, (n, M)))
    else:
        q = _dev(np.ones((n, M)))
        psi0 = _dev(np.zeros((n, M)))
    mlpg.mlpg_set_autotune(2)
    mlpg.mlpg_set_autotune(0)
    ref = None
    for sh in _wide_shapes(M):
        _pin(sh, n, M, ns=6 if dim == 2 else 10)
        P.set_state(psi0)
        phi, pv, psi, info = P.step(q, None, o)
        got = (phi.cpu().numpy(), psi.cpu().numpy(), info["inner_iters"], info["outer_iters"])
        if ref is None:
            ref = got
            assert info["converged"]
            continue
        assert np.array_equal(ref[0], got[0]), sh
        assert np.array_equal(ref[1], got[1]), sh
        assert ref[2:] == got[2:], sh
    P.close()


@pytest.mark.parametrize("dim,M", [(2, 128), (2, 256), (3, 96)])
def test_vector_form_agrees_bitwise_in_single_applications(dim, M):
    """Single applications of L to a random input: every form-2 shape equals form 0 bit for bit."""
    from paper_2008_02205_amd import mlpg
    print(f"[case] vector form, single applications, dim={dim} M={M}", flush=True)
    x, om, P = _wide_problem(dim, M, mlpg.MLPG_FP64)
    n = x.shape[0]
    X = _dev(np.random.default_rng(5).standard_normal((n, M)))
    mlpg.mlpg_set_autotune(2)
    mlpg.mlpg_set_autotune(0)
    ref = None
    for sh in _wide_shapes(M):
        _pin(sh, n, M, ns=6 if dim == 2 else 10)
        Y = mlpg.mlpg_apply(P.h, mlpg.MLPG_OP_L, X).cpu().numpy()
        if ref is None:
            ref = Y
            assert np.all(np.isfinite(Y)) and np.abs(Y).max() > 0
        else:
            assert np.array_equal(ref, Y), sh
    P.close()
