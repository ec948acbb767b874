// Stage workspaces: the device buffers of each stage carved, in a fixed
// order, out of one caller-owned allocation (Arena).  The *_workspace_bytes
// queries run the same layout functions in measuring mode, so a query and
// the stage that uses its workspace agree to the byte.
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace mlpg {

// Positions, radii and overlap lists (copies), the region boxes (up to 64),
// kernel counters, cells, the pattern, and the preconditioner patches (at
// most n patches of at most n points; the grid's cells for binning), with
// the stage's temporaries.
void layout_geometry(Problem &P, Arena &A, int64_t nnz_nb)
{
    const int64_t n = P.n;
    const int d = P.dim;
    A.take(P.reg_lo, 64 * d);
    A.take(P.reg_hi, 64 * d);
    A.take(P.reg_mat, 64);
    A.take(P.x, n * d);
    A.take(P.R, n);
    A.take(P.nb_off, n + 1);
    A.take(P.nb_idx, std::max<int64_t>(1, nnz_nb));
    A.take(P.counters, kNumCounters);
    A.take(P.V, n);
    A.take(P.rho, n);
    A.take(P.bq_off, n + 1);
    if (d == 2) {
        A.take(P.nv, n);
        A.take(P.tags, n * kCellCap2D);
        A.take(P.verts, n * kCellCap2D * 2);
    } else {
        A.take(P.nf, n);
        A.take(P.fnv, n * kFaceCap3);
        A.take(P.ftags, n * kFaceCap3);
        A.take(P.fverts, n * kFaceCap3 * kFaceVerts3 * 3);
    }
    A.take(P.row_off, n + 1);
    A.take(P.col, nnz_nb + n);
    A.take(P.diag_pos, n);
    A.take(P.poff, n + 1);
    A.take(P.boff, n + 1);
    A.take(P.pidx, n);
    // temporaries
    A.take(P.tmp_flags, n);
    A.take(P.tmp_bqc, n);
    A.take(P.tmp_key, n);
    A.take(P.tmp_s2, n);
    A.take(P.tmp_npc, P.ncell);
    A.take(P.tmp_off, P.ncell + 1);
    A.take(P.tmp_pbase, P.ncell + 1);
    A.take(P.tmp_cnt, P.ncell);
}

// Blocks, point-value matrix, boundary quadrature (sized by the cells), the
// surface-row offsets, the candidate and surface counts, and in 3D with one
// material and no fields the Gram panels of a batch of cells.
void layout_integrate(Problem &P, Arena &A)
{
    const int64_t n = P.n, nnz = P.nnz;
    const int64_t nbq = std::max<int64_t>(1, P.n_bq);
    const int nblk = P.n_mat * (1 + P.dim) + P.dim * P.dim + 2 * P.dim;
    A.take(P.blocks, (size_t)nblk * nnz);
    A.take(P.E, nnz);
    A.take(P.bq_y, nbq * P.dim);
    A.take(P.bq_w, nbq);
    A.take(P.bq_face, nbq);
    A.take(P.bq_nact, nbq);
    A.take(P.bq_act, nbq * P.bq_kmax);
    A.take(P.bq_N, nbq * P.bq_kmax);
    A.take(P.surf_off, n + 1);
    A.take(P.tmp_cand, n);
    A.take(P.tmp_scnt, n);
    const bool panels = P.dim == 3 && P.n_mat == 1 && P.n_fields == 0 && P.n_shells == 0;
    A.take(P.gram_ws, panels ? (size_t)std::min<int64_t>(n, kGramCells) * kGramPanelBytes : 0);
}

// The state (Psi, Phi: first, so that a workspace reused with the same
// ordinate count keeps it), value streams, per-ordinate coefficient tables,
// surface rows, Jacobi scaling, the diffusion-synthetic operators and the
// FP32 copies of the mixed path.
void layout_assemble(Problem &P, Arena &A, int n_ord, int precision)
{
    const int64_t n = P.n, nnz = P.nnz;
    const int d = P.dim;
    const int nsL = 1 + d + d * (d + 1) / 2, nsMD = 1 + d, nf = 2 * d;
    const int64_t nnz_s = std::max<int64_t>(1, P.nnz_s);
    const size_t nm = (size_t)n * n_ord;
    A.take(P.psi, nm);
    A.take(P.phi, n);
    A.take(P.sL, (size_t)nnz * nsL);
    A.take(P.sMD, (size_t)nnz * nsMD);
    A.take(P.sMS, (size_t)nnz * nsMD);
    A.take(P.coefL, (size_t)n_ord * nsL);
    A.take(P.coefMD, (size_t)n_ord * nsMD);
    A.take(P.coefF, (size_t)n_ord * nf);
    A.take(P.omega, (size_t)n_ord * d);
    A.take(P.wq, n_ord);
    A.take(P.surf_col, nnz_s);
    A.take(P.surf_val, nnz_s * nf);
    A.take(P.dinv, nm);
    A.take(P.dsaC, nnz);
    A.take(P.dsaMs, nnz);
    A.take(P.dsa_dinv, n);
    if (precision == MLPG_MIXED) {
        A.take(P.sL32, (size_t)nnz * nsL);
        A.take(P.coefL32, (size_t)n_ord * nsL);
        A.take(P.coefF32, (size_t)n_ord * nf);
        A.take(P.surf_val32, nnz_s * nf);
        A.take(P.dinv32, nm);
    }
}

// Scratch of one solve: right-hand sides and intermediate fields, the
// batched inner Krylov space (and its FP32 twin with the refinement vectors
// in the mixed path), the outer Krylov space, the diffusion solve's space
// (MLPG_ACCEL_DSA) and the patch inverses (MLPG_PRECOND_PATCH).
void layout_solve(Problem &P, Arena &A, const mlpg_solve_opts &o)
{
    const int64_t n = P.n;
    const int M = P.n_ord;
    const size_t nm = (size_t)n * M;
    A.take(P.F, nm);
    A.take(P.bpsi, nm);
    A.take(P.t1, nm);
    A.take(P.t2, nm);
    A.take(P.bphi, n);
    A.take(P.ovec, n);
    P.inner.carve(A, n, M, o.restart_inner);
    P.outer.carve(A, n, 1, o.restart_outer);
    if (P.precision == MLPG_MIXED) {
        P.inner32.carve(A, n, M, o.restart_inner);
        A.take(P.r32, nm);
        A.take(P.d32, nm);
        A.take(P.mr, nm);
        A.take(P.rn2, M);
        A.take(P.fn2, M);
        A.take(P.tolv, M);
    }
    if (o.accel == MLPG_ACCEL_DSA) {
        P.dsa.carve(A, n, 1, kDsaRestart);
        A.take(P.dsa_r, n);
        A.take(P.dsa_x, n);
        A.take(P.dsa_Z, (size_t)o.restart_outer * n);
    }
    if (o.precond == MLPG_PRECOND_PATCH) {
        const size_t cnt = (size_t)P.nbsq * M;
        A.take(P.binv, cnt);
        A.take(P.tmp_work, cnt);
        A.take(P.tmp_sing, 1);
        if (P.precision == MLPG_MIXED) A.take(P.binv32, cnt);
    }
}

}  // namespace mlpg
