// C ABI of libmlpg (declared in include/mlpg.h): argument validation, the
// problem handle, stage sequencing and the Krylov solve of one step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mlpg {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

void Problem::release()
{
    reg_lo.release(); reg_hi.release(); reg_mat.release(); x.release(); R.release(); nb_off.release();
    nb_idx.release(); nv.release(); tags.release(); verts.release(); V.release(); rho.release(); bq_off.release();
    nf.release(); fnv.release(); ftags.release(); fverts.release();
    bq_y.release(); bq_w.release(); bq_N.release(); bq_face.release(); bq_nact.release(); bq_act.release();
    row_off.release(); diag_pos.release(); col.release(); blocks.release(); E.release(); counters.release();
    wq.release(); omega.release(); sL.release(); sMD.release(); sMS.release(); coefL.release(); coefMD.release();
    coefF.release(); surf_off.release(); surf_col.release(); surf_val.release(); dinv.release(); psi.release();
    phi.release(); F.release(); bpsi.release(); t1.release(); t2.release(); bphi.release(); ovec.release();
    inner.release(); outer.release(); inner32.release();
    sL32.release(); coefL32.release(); coefF32.release(); surf_val32.release(); dinv32.release(); r32.release();
    d32.release(); mr.release(); rn2.release(); fn2.release(); tolv.release();
    dsaC.release(); dsaMs.release(); dsa_dinv.release(); dsa_r.release(); dsa_x.release(); dsa_Z.release();
    dsa.release();
    poff.release(); boff.release(); pidx.release(); binv.release(); binv32.release();
    patches_ok = binv_ok = false;
    tmp_flags.release(); tmp_cand.release(); gram_ws.release(); tmp_bqc.release(); tmp_key.release(); tmp_s2.release();
    tmp_npc.release(); tmp_off.release(); tmp_pbase.release(); tmp_scnt.release(); tmp_cnt.release();
    tmp_sing.release(); tmp_work.release();
    own_geo.release(); own_int.release(); own_asm.release(); own_slv.release();
}

namespace {

hipStream_t S(void *s) { return (hipStream_t)s; }

int op_L(Problem &P, const OpCall &c, hipStream_t s, void *)
{
    SpmvArgs a;
    a.vals = P.sL.p; a.ns = P.nsL; a.coef = P.coefL.p; a.x = c.in; a.dinv = c.dinv; a.surface = 1; a.y = c.out;
    a.sval = P.surf_val.p; a.coefF = P.coefF.p;
    a.colscale = c.colscale; a.vout = c.vout; a.vsrc = c.vsrc; a.gate = c.gate;
    int id = -1;
    if (prof_on()) {
        // the sweep's algorithmic bytes per unit (one row and ordinate): the
        // streams and column indices once per row, shared by the ordinates,
        // x read and y written once; summed over the rows and ordinates of
        // the launch, with the row offsets and the surface rows.  A fused
        // normalisation (the previous vector read, the basis vector written)
        // belongs to the Gram-Schmidt side of the step and is not counted.
        const double nm = 8.0 * (double)P.n * P.n_ord;
        double b = (double)P.nnz * (8.0 * P.nsL + 4.0) + 8.0 * (P.n + 1) + 2.0 * nm;
        b += (double)P.nnz_s * (8.0 * P.nfaces + 4.0) + 8.0 * (P.n + 1);
        id = prof_start(0, b, s);
    }
    MLPG_HIP(launch_spmv(P, a, s));
    prof_stop(id, s);
    return MLPG_OK;
}

// FP32 transport operator for the inner solves of the mixed path: FP32
// values, FP32 vectors, FP32 accumulation.
int op_L32(Problem &P, const OpCallT<float> &c, hipStream_t s, void *)
{
    SpmvArgsT<float> a;
    a.vals = P.sL32.p; a.ns = P.nsL; a.coef = P.coefL32.p; a.x = c.in; a.dinv = c.dinv; a.surface = 1;
    a.sval = P.surf_val32.p; a.coefF = P.coefF32.p; a.y = c.out;
    a.colscale = c.colscale; a.vout = c.vout; a.vsrc = c.vsrc; a.gate = c.gate;
    int id = -1;
    if (prof_on()) {
        // as for the FP64 sweep, with 4-byte values and vectors
        const double nm = 4.0 * (double)P.n * P.n_ord;
        double b = (double)P.nnz * (4.0 * P.nsL + 4.0) + 8.0 * (P.n + 1) + 2.0 * nm;
        b += (double)P.nnz_s * (4.0 * P.nfaces + 4.0) + 8.0 * (P.n + 1);
        id = prof_start(0, b, s);
    }
    MLPG_HIP(launch_spmv<float>(P, a, s));
    prof_stop(id, s);
    return MLPG_OK;
}

struct SolveCounters {
    const mlpg_solve_opts *o;
    int64_t its = 0, sweeps = 0, refinements = 0, fp64_completions = 0, accel_its = 0;
    double res_max = 0.0;
    bool conv = true;
    int solves = 0;
};

template <class T>
PatchPrecT<T> patch_prec(const Problem &P, const T *binv)
{
    PatchPrecT<T> pp;
    pp.npatch = P.npatch;
    pp.poff = P.poff.p;
    pp.pidx = P.pidx.p;
    pp.boff = P.boff.p;
    pp.binv = binv;
    return pp;
}

int inner_solve_fp64(Problem &P, SolveCounters &c, const double *f, double *x, hipStream_t s)
{
    const bool patch = c.o->precond == MLPG_PRECOND_PATCH;
    const PatchPrecT<double> pp = patch_prec<double>(P, P.binv.p);
    return gmres_batched<double>(P, P.inner, op_L, true, nullptr, patch ? nullptr : P.dinv.p, f, x, P.n, P.n_ord,
                                 c.o->tol_inner, c.o->restart_inner, c.o->max_inner, c.o->check_every, true, s,
                                 &c.its, &c.sweeps, &c.res_max, &c.conv, nullptr, false, patch ? &pp : nullptr,
                                 c.o->graphs != 0);
}

// Mixed precision: iterative refinement in FP64 around FP32 GMRES.
//   r = f - L x (FP64 values, FP64 accumulation); per ordinate, the
//   correction solves L d = r / ||r|| with FP32 GMRES to tol_inner_lo
//   (FP32 SpMV, FP32 basis, FP64 dot products and Hessenberg); x += ||r|| d.
// Stops when every ordinate has ||f - L x|| <= tol_inner ||f||.  Each
// correction gets at most ten restart cycles.  When a refinement fails to
// halve the residual of some unconverged ordinate (FP32 stagnating on an
// ill-conditioned operator) or the refinement budget is spent, the solve is
// finished by FP64 GMRES from the current iterate.
int inner_solve_mixed(Problem &P, SolveCounters &c, const double *f, double *x, hipStream_t s)
{
    const int64_t n = P.n;
    const int M = P.n_ord;
    const int64_t cnt = n * M;
    const mlpg_solve_opts &o = *c.o;
    MLPG_HIP(hipMemsetAsync(x, 0, sizeof(double) * cnt, s));
    MLPG_HIP(hipMemcpyAsync(P.mr.p, f, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
    MLPG_HIP(batched_norm2(P.inner, f, P.fn2.p, s));
    std::vector<double> fn2(M), rn2(M), tolm(M);
    MLPG_HIP(hipMemcpyAsync(fn2.data(), P.fn2.p, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    bool conv = false, stalled = false;
    double worst = 0.0;
    std::vector<double> prev(M, -1.0);
    for (int it = 0;; ++it) {
        MLPG_HIP(batched_norm2(P.inner, P.mr.p, P.rn2.p, s));
        MLPG_HIP(hipMemcpyAsync(rn2.data(), P.rn2.p, sizeof(double) * M, hipMemcpyDeviceToHost, s));
        MLPG_HIP(hipStreamSynchronize(s));
        worst = 0.0;
        conv = true;
        for (int m = 0; m < M; ++m) {
            double rel = fn2[m] > 0.0 ? std::sqrt(rn2[m] / fn2[m]) : 0.0;
            worst = std::max(worst, rel);
            if (fn2[m] > 0.0 && rel > o.tol_inner) {
                conv = false;
                if (prev[m] > 0.0 && rn2[m] > 0.25 * prev[m]) stalled = true;   // less than halved
            }
            prev[m] = rn2[m];
        }
        if (conv || stalled || it >= o.max_refine) break;
        // Per ordinate, the correction only has to close the remaining gap
        // (with a factor 2 to spare), never looser than 1/2 and never
        // tighter than tol_inner_lo.
        for (int m = 0; m < M; ++m) {
            const double need = rn2[m] > 0.0 ? 0.5 * o.tol_inner * std::sqrt(fn2[m] / rn2[m]) : 0.5;
            tolm[m] = std::min(0.5, std::max(o.tol_inner_lo, need));
        }
        MLPG_HIP(hipMemcpyAsync(P.tolv.p, tolm.data(), sizeof(double) * M, hipMemcpyHostToDevice, s));
        MLPG_HIP(launch_to_float_scaled(n, M, P.mr.p, P.rn2.p, P.fn2.p, o.tol_inner, P.r32.p, s));
        bool c32 = true;
        double rm32 = 0.0;
        const int cap = std::min(o.max_inner, 10 * o.restart_inner);
        const bool patch = o.precond == MLPG_PRECOND_PATCH;
        const PatchPrecT<float> pp32 = patch_prec<float>(P, P.binv32.p);
        int rc = gmres_batched<float>(P, P.inner32, op_L32, true, nullptr, patch ? nullptr : P.dinv32.p, P.r32.p,
                                      P.d32.p, n, M, o.tol_inner_lo, o.restart_inner, cap, o.check_every, true, s,
                                      &c.its, &c.sweeps, &rm32, &c32, P.tolv.p, false, patch ? &pp32 : nullptr,
                                      o.graphs != 0);
        MLPG_HIP(hipStreamSynchronize(s));   // tolm is read by the copy above
        if (rc) return rc;
        MLPG_HIP(launch_axpy_from_float(n, M, x, P.d32.p, P.rn2.p, s));
        SpmvArgs a;
        a.vals = P.sL.p; a.ns = P.nsL; a.coef = P.coefL.p; a.x = x; a.surface = 1; a.sval = P.surf_val.p;
        a.coefF = P.coefF.p; a.y = P.mr.p; a.yadd = f; a.ysign = -1;
        MLPG_HIP(launch_spmv<double>(P, a, s));
        c.refinements++;
    }
    if (!conv) {
        // FP64 completion from the current iterate
        bool c64 = true;
        double rm = 0.0;
        const bool patch = o.precond == MLPG_PRECOND_PATCH;
        const PatchPrecT<double> pp = patch_prec<double>(P, P.binv.p);
        int rc = gmres_batched<double>(P, P.inner, op_L, true, nullptr, patch ? nullptr : P.dinv.p, f, x, n, M,
                                       o.tol_inner, o.restart_inner, o.max_inner, o.check_every, false, s, &c.its,
                                       &c.sweeps, &rm, &c64, nullptr, false, patch ? &pp : nullptr, o.graphs != 0);
        if (rc) return rc;
        c.fp64_completions++;
        conv = c64;
        worst = rm;
    }
    c.res_max = std::max(c.res_max, worst);
    c.conv = c.conv && conv;
    return MLPG_OK;
}

// One batched L^-1 application.  An inner solve that misses its tolerance
// ends the whole step at once: the outer GMRES needs L^-1 as a fixed linear
// map, and iterating on an operator that is not one only burns sweeps.
int inner_solve(Problem &P, SolveCounters &c, const double *f, double *x, hipStream_t s)
{
    c.solves++;
    int rc = P.precision == MLPG_MIXED ? inner_solve_mixed(P, c, f, x, s) : inner_solve_fp64(P, c, f, x, s);
    if (rc) return rc;
    if (!c.conv) {
        set_error("mlpg_solve: an inner solve reached max_inner (" + std::to_string(c.o->max_inner) +
                  " Arnoldi steps) before its tolerance; largest relative residual " + std::to_string(c.res_max));
        return MLPG_ERR_NOT_CONVERGED;
    }
    return MLPG_OK;
}

// A phi = phi - D L^-1 MS phi  (Eq. krylov-operator)
int op_outer(Problem &P, const OpCall &oc, hipStream_t s, void *vctx)
{
    SolveCounters &c = *(SolveCounters *)vctx;
    SpmvArgs a;
    a.vals = P.sMS.p; a.ns = P.nsMD; a.coef = P.coefMD.p; a.x = oc.in; a.x_bcast = 1; a.y = P.t1.p;
    MLPG_HIP(launch_spmv(P, a, s));
    int rc = inner_solve(P, c, P.t1.p, P.t2.p, s);
    if (rc) return rc;
    MLPG_HIP(launch_ord_reduce(P, P.t2.p, oc.out, oc.in, -1.0, s));
    return MLPG_OK;
}

// The diffusion operator C of the synthetic acceleration, with point Jacobi
// from the right (gmres passes dinv).
int op_dsa(Problem &P, const OpCall &c, hipStream_t s, void *)
{
    MLPG_HIP(launch_csr_spmv(P, P.dsaC.p, c.in, c.dinv, c.out, c.gate, s));
    return MLPG_OK;
}

// out = M^-1 v = v + C^-1 (Ms v), C solved to a relative residual of
// kDsaTol (at most kDsaMaxIts steps).  The outer iteration is flexible GMRES
// (it keeps every M^-1 v_j and updates Phi with them), so the diffusion solve
// need not be exact nor the same linear map at every step: the outer
// residual is that of the unaccelerated system, and its converged Phi is the
// unaccelerated solution.
constexpr double kDsaTol = 1e-4;
constexpr int kDsaMaxIts = 2000;

int dsa_apply(Problem &P, SolveCounters &c, const double *v, double *out, hipStream_t s)
{
    MLPG_HIP(launch_csr_spmv(P, P.dsaMs.p, v, nullptr, P.dsa_r.p, nullptr, s));
    int64_t sweeps = 0;
    double rm = 0.0;
    bool conv = true;   // not required: an inexact diffusion solve only slows the outer iteration
    int rc = gmres_batched<double>(P, P.dsa, op_dsa, false, nullptr, P.dsa_dinv.p, P.dsa_r.p, P.dsa_x.p, P.n, 1,
                                   kDsaTol, kDsaRestart, kDsaMaxIts, 1, true, s, &c.accel_its, &sweeps, &rm, &conv,
                                   nullptr, true);
    if (rc) return rc;
    MLPG_HIP(launch_add(out, v, P.dsa_x.p, P.n, s));
    return MLPG_OK;
}

int dsa_flex_apply(Problem &P, const double *v, double *z, hipStream_t s, void *ctx)
{
    return dsa_apply(P, *(SolveCounters *)ctx, v, z, s);
}

bool P_ok_lo(const mlpg_solve_opts &o) { return o.tol_inner_lo > 0.0 && o.tol_inner_lo < 1.0; }

int check_stage(mlpg_handle h, int need, const char *who)
{
    if (!h) {
        set_error(std::string(who) + ": null handle");
        return MLPG_ERR_ARG;
    }
    Problem *P = (Problem *)h;
    if (P->stage < need) {
        set_error(std::string(who) + ": called before the preceding stage");
        return MLPG_ERR_STATE;
    }
    return MLPG_OK;
}

// Binds a stage's buffers: into the caller's workspace `ws` (at least the
// measured size, 256-byte aligned), or, when ws is null, into a library
// allocation `own` of the measured size (grown when needed).
template <class F>
static int bind_stage(Problem &P, DevBuf<char> &own, void *ws, size_t ws_bytes, const char *who, F layout)
{
    // measured on a copy, so that a workspace that is too small leaves the
    // handle's current buffers as they were
    Arena m;
    {
        Problem tmp = P;
        layout(tmp, m);
    }
    const size_t need = m.used;
    Arena A;
    if (ws) {
        if (((uintptr_t)ws & 255) != 0) {
            set_error(std::string(who) + ": the workspace must be 256-byte aligned");
            return MLPG_ERR_ARG;
        }
        if (ws_bytes < need) {
            set_error(std::string(who) + ": workspace of " + std::to_string(ws_bytes) + " bytes, the stage needs " +
                      std::to_string(need));
            return MLPG_ERR_WORKSPACE;
        }
        own.release();
        A.base = (char *)ws;
        A.cap = ws_bytes;
    } else {
        if (!own.p || !own.owned || own.count < need) MLPG_HIP(own.alloc(need));
        A.base = own.p;
        A.cap = own.count;
    }
    layout(P, A);
    if (A.over || A.used != need) {
        set_error(std::string(who) + ": workspace layout mismatch");
        return MLPG_ERR_WORKSPACE;
    }
    return MLPG_OK;
}

}  // namespace
}  // namespace mlpg

using namespace mlpg;

struct mlpg_problem : public Problem {};

extern "C" {

const char *mlpg_last_error(void) { return g_err.c_str(); }

int mlpg_cell_capacity(void) { return kCellCap2D; }

int mlpg_neighbors_count(int dim, int64_t n, const double *x, const double *R, int64_t *nbr_off, int64_t *total,
                         void *stream)
{
    MLPG_CHECK(dim == 2 || dim == 3, MLPG_ERR_ARG, "mlpg_neighbors_count: dim must be 2 or 3");
    MLPG_CHECK(n > 0 && n < (int64_t)1 << 31, MLPG_ERR_ARG, "mlpg_neighbors_count: n out of range");
    MLPG_CHECK(x && R && nbr_off && total, MLPG_ERR_ARG, "mlpg_neighbors_count: null pointer");
    hipStream_t s = S(stream);
    const int64_t mc = nb_max_cells(n);
    DevBuf<char> scratch;
    MLPG_HIP(scratch.alloc(nb_scratch_bytes(n, mc)));
    const NbScratch sc = nb_scratch_at(scratch.p, n, mc);
    // the counts go into nbr_off itself and are scanned in place
    MLPG_HIP(launch_neighbors_count(dim, n, x, R, nbr_off, sc, s));
    MLPG_HIP(launch_exclusive_scan(nbr_off, nbr_off, n, s));
    MLPG_HIP(hipMemcpyAsync(total, nbr_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipStreamSynchronize(s));
    scratch.release();
    return MLPG_OK;
}

int mlpg_neighbors_fill(int dim, int64_t n, const double *x, const double *R, const int64_t *nbr_off,
                        int32_t *nbr_idx, void *stream)
{
    MLPG_CHECK(dim == 2 || dim == 3, MLPG_ERR_ARG, "mlpg_neighbors_fill: dim must be 2 or 3");
    MLPG_CHECK(n > 0 && n < (int64_t)1 << 31 && x && R && nbr_off && nbr_idx, MLPG_ERR_ARG,
               "mlpg_neighbors_fill: bad argument");
    hipStream_t s = S(stream);
    const int64_t mc = nb_max_cells(n);
    DevBuf<char> scratch;
    MLPG_HIP(scratch.alloc(nb_scratch_bytes(n, mc)));
    const NbScratch sc = nb_scratch_at(scratch.p, n, mc);
    MLPG_HIP(launch_neighbors_fill(dim, n, x, R, nbr_off, nbr_idx, sc, s));
    MLPG_HIP(hipStreamSynchronize(s));   // the scratch is released below
    scratch.release();
    return MLPG_OK;
}

// Positions, radii and overlap lists of the points, then the cells (Sec. 3.1),
// the boundary quadrature sizing, the pattern and the preconditioner patches:
// the part of stage 1 that depends on where the points are.  Every buffer is
// carved from the geometry workspace; counters reset.
static int build_geometry(Problem &P, const double *x, const double *R, const int64_t *nbr_off,
                          const int32_t *nbr_idx, void *ws, size_t ws_bytes, const char *who, hipStream_t s)
{
    const int64_t n = P.n;
    const int dim = P.dim;
#define TRY(call)                                                                  \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));          \
            return MLPG_ERR_HIP;                                                   \
        }                                                                          \
    } while (0)
    P.failed = 0;
    P.oversize = 0;
    P.patches_ok = P.binv_ok = false;   // patches follow the positions, inverses the operators
    int64_t nnz_nb = 0;
    TRY(hipMemcpyAsync(&nnz_nb, nbr_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    if (nnz_nb < 0 || nnz_nb > ((int64_t)1 << 40)) {
        set_error(std::string(who) + ": neighbour list size out of range");
        return MLPG_ERR_ARG;
    }
    P.nnz_nb = nnz_nb;
    int64_t dims[3];
    P.ncell = patch_grid_cells(dim, n, P.dom_lo, P.dom_hi, nullptr, dims);
    int rc = bind_stage(P, P.own_geo, ws, ws_bytes, who,
                        [&](Problem &Q, Arena &A) { layout_geometry(Q, A, nnz_nb); });
    if (rc) return rc;
    P.ws_geo = ws;
    P.gen++;
    if (P.n_regions) {
        TRY(hipMemcpyAsync(P.reg_lo.p, P.reg_lo_h, sizeof(double) * P.n_regions * dim, hipMemcpyHostToDevice, s));
        TRY(hipMemcpyAsync(P.reg_hi.p, P.reg_hi_h, sizeof(double) * P.n_regions * dim, hipMemcpyHostToDevice, s));
        TRY(hipMemcpyAsync(P.reg_mat.p, P.reg_mat_h, sizeof(int32_t) * P.n_regions, hipMemcpyHostToDevice, s));
    }
    TRY(hipMemcpyAsync(P.x.p, x, sizeof(double) * n * dim, hipMemcpyDeviceToDevice, s));
    TRY(hipMemcpyAsync(P.R.p, R, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    TRY(hipMemcpyAsync(P.nb_off.p, nbr_off, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz_nb) TRY(hipMemcpyAsync(P.nb_idx.p, nbr_idx, sizeof(int32_t) * nnz_nb, hipMemcpyDeviceToDevice, s));
    // the lists steer every later kernel's reads: validate them before use
    TRY(hipMemsetAsync(P.counters.p, 0, sizeof(unsigned long long) * kNumCounters, s));
    TRY(launch_check_lists(n, nnz_nb, P.nb_off.p, P.nb_idx.p, P.counters.p + kBadLists, s));
    {
        unsigned long long bad = 0;
        TRY(hipMemcpyAsync(&bad, P.counters.p + kBadLists, sizeof(bad), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        if (bad) {
            set_error(std::string(who) + ": malformed overlap lists (" +
                      ((bad & 1) ? "offsets not non-decreasing from 0 within the list length" :
                                   "an index out of [0, n), equal to its row, or not strictly increasing") +
                      ")");
            return MLPG_ERR_ARG;
        }
    }
    if (dim == 2) {
        TRY(launch_clip2d(P, s, P.tmp_flags.p, P.tmp_bqc.p));
        P.bq_kmax = kBqAct;
    } else {
        TRY(launch_clip3d(P, s, P.tmp_flags.p, P.tmp_bqc.p));
        P.bq_kmax = kBqAct3;
    }
    TRY(launch_exclusive_scan(P.tmp_bqc.p, P.bq_off.p, n, s));
    std::vector<int32_t> hf(n);
    TRY(hipMemcpyAsync(hf.data(), P.tmp_flags.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    TRY(hipMemcpyAsync(&P.n_bq, P.bq_off.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
        if (hf[i] == 1) P.failed++;
        if (hf[i] == 2) P.oversize++;
    }
    if (P.failed) {
        set_error(std::string(who) + ": " + std::to_string(P.failed) +
                  " cells empty or over the face/vertex capacity");
        return MLPG_ERR_GEOMETRY;
    }
    P.nnz = nnz_nb + n;
    TRY(launch_pattern(P, s));
#undef TRY
    rc = build_patches(P, s);
    if (rc) return rc;
    P.patches_ok = true;
    return MLPG_OK;
}

int mlpg_geometry(mlpg_handle *out, int dim, int64_t n, const double *x, const double *R, const int64_t *nbr_off,
                  const int32_t *nbr_idx, const double *dom_lo, const double *dom_hi, int n_regions,
                  const double *region_lo, const double *region_hi, const int32_t *region_mat, void *workspace,
                  size_t ws_bytes, void *stream)
{
    MLPG_CHECK(out, MLPG_ERR_ARG, "mlpg_geometry: null output handle");
    *out = nullptr;
    MLPG_CHECK(dim == 2 || dim == 3, MLPG_ERR_ARG, "mlpg_geometry: dim must be 2 or 3");
    MLPG_CHECK(n > 0 && n < (int64_t)1 << 31, MLPG_ERR_ARG, "mlpg_geometry: n out of range");
    MLPG_CHECK(x && R && nbr_off && nbr_idx && dom_lo && dom_hi, MLPG_ERR_ARG, "mlpg_geometry: null pointer");
    for (int a = 0; a < dim; ++a)
        MLPG_CHECK(dom_hi[a] > dom_lo[a], MLPG_ERR_ARG, "mlpg_geometry: empty domain box");
    MLPG_CHECK(n_regions >= 0 && n_regions <= 64, MLPG_ERR_ARG, "mlpg_geometry: n_regions must be in [0, 64]");
    MLPG_CHECK(n_regions == 0 || (region_lo && region_hi && region_mat), MLPG_ERR_ARG,
               "mlpg_geometry: null region arrays");
    int n_mat = 1;
    for (int r = 0; r < n_regions; ++r) {
        MLPG_CHECK(region_mat[r] >= 0 && region_mat[r] < 8, MLPG_ERR_ARG, "mlpg_geometry: material id in [0, 8)");
        n_mat = std::max(n_mat, region_mat[r] + 1);
    }
    hipStream_t s = S(stream);
    mlpg_problem *P = new mlpg_problem();
    P->dim = dim;
    P->n = n;
    P->n_mat = n_mat;
    for (int a = 0; a < dim; ++a) { P->dom_lo[a] = dom_lo[a]; P->dom_hi[a] = dom_hi[a]; }
    P->n_regions = n_regions;
    for (int r = 0; r < n_regions; ++r) {
        for (int a = 0; a < dim; ++a) {
            P->reg_lo_h[r * dim + a] = region_lo[r * dim + a];
            P->reg_hi_h[r * dim + a] = region_hi[r * dim + a];
        }
        P->reg_mat_h[r] = region_mat[r];
    }
    int rc = build_geometry(*P, x, R, nbr_off, nbr_idx, workspace, ws_bytes, "mlpg_geometry", s);
    if (rc) {
        P->release();
        delete P;
        return rc;
    }
    P->stage = 1;
    *out = P;
    return MLPG_OK;
}

int mlpg_update_points(mlpg_handle h, const double *x, const double *R, const int64_t *nbr_off,
                       const int32_t *nbr_idx, void *workspace, size_t ws_bytes, void *stream)
{
    int rc = check_stage(h, 1, "mlpg_update_points");
    if (rc) return rc;
    MLPG_CHECK(x && R && nbr_off && nbr_idx, MLPG_ERR_ARG, "mlpg_update_points: null pointer");
    Problem *P = h;
    rc = build_geometry(*P, x, R, nbr_off, nbr_idx, workspace, ws_bytes, "mlpg_update_points", S(stream));
    // the integrated blocks and the assembled operators belong to the old
    // positions; the state (per-point coefficients) and the solver settings stay
    P->stage = 1;
    return rc;
}

size_t mlpg_geometry_workspace_bytes(int dim, int64_t n, int64_t nnz_nbr, const double *dom_lo, const double *dom_hi)
{
    if ((dim != 2 && dim != 3) || n <= 0 || nnz_nbr < 0 || !dom_lo || !dom_hi) return 0;
    for (int a = 0; a < dim; ++a)
        if (!(dom_hi[a] > dom_lo[a])) return 0;
    Problem P;
    P.dim = dim;
    P.n = n;
    for (int a = 0; a < dim; ++a) { P.dom_lo[a] = dom_lo[a]; P.dom_hi[a] = dom_hi[a]; }
    int64_t dims[3];
    P.ncell = patch_grid_cells(dim, n, P.dom_lo, P.dom_hi, nullptr, dims);
    Arena A;
    layout_geometry(P, A, nnz_nbr);
    return A.used;
}

int mlpg_get_info(mlpg_handle h, mlpg_info *info)
{
    int rc = check_stage(h, 1, "mlpg_get_info");
    if (rc) return rc;
    MLPG_CHECK(info, MLPG_ERR_ARG, "mlpg_get_info: null info");
    Problem *P = h;
    info->n = P->n;
    info->dim = P->dim;
    info->n_mat = P->n_mat;
    info->nnz = P->nnz;
    info->n_bq = P->n_bq;
    info->oversize_cells = P->oversize;
    info->failed_cells = P->failed;
    info->fallback_qps = P->fallbacks;
    info->missing_pairs = P->missing;
    info->n_ord = P->stage >= 3 ? P->n_ord : 0;
    info->n_blocks = P->n_mat * (1 + P->dim) + P->dim * P->dim + 2 * P->dim;
    return MLPG_OK;
}

int mlpg_get_volumes(mlpg_handle h, double *V, void *stream)
{
    int rc = check_stage(h, 1, "mlpg_get_volumes");
    if (rc) return rc;
    MLPG_CHECK(V, MLPG_ERR_ARG, "mlpg_get_volumes: null output");
    MLPG_HIP(hipMemcpyAsync(V, h->V.p, sizeof(double) * h->n, hipMemcpyDeviceToDevice, S(stream)));
    return MLPG_OK;
}

int mlpg_get_cells(mlpg_handle h, int32_t *nv, double *verts, int32_t *tags, void *stream)
{
    int rc = check_stage(h, 1, "mlpg_get_cells");
    if (rc) return rc;
    MLPG_CHECK(nv && verts && tags, MLPG_ERR_ARG, "mlpg_get_cells: null output");
    MLPG_CHECK(h->dim == 2, MLPG_ERR_ARG, "mlpg_get_cells: polygons of 2D problems only");
    hipStream_t s = S(stream);
    MLPG_HIP(hipMemcpyAsync(nv, h->nv.p, sizeof(int32_t) * h->n, hipMemcpyDeviceToDevice, s));
    MLPG_HIP(hipMemcpyAsync(verts, h->verts.p, sizeof(double) * h->n * kCellCap2D * 2, hipMemcpyDeviceToDevice, s));
    MLPG_HIP(hipMemcpyAsync(tags, h->tags.p, sizeof(int32_t) * h->n * kCellCap2D, hipMemcpyDeviceToDevice, s));
    return MLPG_OK;
}

int mlpg_boundary_points(mlpg_handle h, double *y, int32_t *face, void *stream)
{
    int rc = check_stage(h, 2, "mlpg_boundary_points");
    if (rc) return rc;
    MLPG_CHECK(y && face, MLPG_ERR_ARG, "mlpg_boundary_points: null output");
    if (h->n_bq == 0) return MLPG_OK;
    hipStream_t s = S(stream);
    MLPG_HIP(hipMemcpyAsync(y, h->bq_y.p, sizeof(double) * h->n_bq * h->dim, hipMemcpyDeviceToDevice, s));
    MLPG_HIP(hipMemcpyAsync(face, h->bq_face.p, sizeof(int32_t) * h->n_bq, hipMemcpyDeviceToDevice, s));
    return MLPG_OK;
}

int mlpg_material_fields(mlpg_handle h, int n_fields, const double *param, const int32_t *mat)
{
    int rc = check_stage(h, 1, "mlpg_material_fields");
    if (rc) return rc;
    MLPG_CHECK(n_fields >= 0 && n_fields <= kMaxFields, MLPG_ERR_ARG, "mlpg_material_fields: n_fields in [0, 8]");
    MLPG_CHECK(n_fields == 0 || (param && mat), MLPG_ERR_ARG, "mlpg_material_fields: NULL param or mat");
    for (int r = 0; r < n_fields; ++r)
        MLPG_CHECK(mat[r] >= 1 && mat[r] < kMaxMat, MLPG_ERR_ARG, "mlpg_material_fields: material in [1, 8)");
    Problem *P = h;
    P->n_fields = n_fields;
    for (int r = 0; r < kMaxFields; ++r) {
        for (int q = 0; q < 4; ++q) P->field_par[r][q] = r < n_fields ? param[4 * r + q] : 0.0;
        P->field_mat[r] = r < n_fields ? mat[r] : 0;
        if (r < n_fields) P->n_mat = std::max(P->n_mat, mat[r] + 1);
    }
    P->stage = 1;
    return MLPG_OK;
}

int mlpg_material_shells(mlpg_handle h, int n_shells, const double *center, const double *radii,
                         const int32_t *mat)
{
    int rc = check_stage(h, 1, "mlpg_material_shells");
    if (rc) return rc;
    MLPG_CHECK(n_shells >= 0 && n_shells <= kMaxFields, MLPG_ERR_ARG, "mlpg_material_shells: n_shells in [0, 8]");
    MLPG_CHECK(n_shells == 0 || (center && radii && mat), MLPG_ERR_ARG, "mlpg_material_shells: null array");
    for (int r = 0; r < n_shells; ++r) {
        MLPG_CHECK(mat[r] >= 0 && mat[r] < kMaxMat, MLPG_ERR_ARG, "mlpg_material_shells: material in [0, 8)");
        MLPG_CHECK(radii[2 * r] >= 0.0 && radii[2 * r + 1] >= radii[2 * r], MLPG_ERR_ARG,
                   "mlpg_material_shells: need 0 <= r_in <= r_out");
    }
    Problem *P = h;
    P->n_shells = n_shells;
    for (int r = 0; r < kMaxFields; ++r) {
        for (int q = 0; q < 5; ++q) P->shell_par[r][q] = 0.0;
        P->shell_mat[r] = 0;
        if (r >= n_shells) continue;
        for (int a = 0; a < P->dim; ++a) P->shell_par[r][a] = center[P->dim * r + a];
        P->shell_par[r][P->dim] = radii[2 * r];
        P->shell_par[r][P->dim + 1] = radii[2 * r + 1];
        P->shell_mat[r] = mat[r];
        P->n_mat = std::max(P->n_mat, mat[r] + 1);
    }
    P->stage = 1;
    return MLPG_OK;
}

int mlpg_integrate(mlpg_handle h, int rk_order, void *workspace, size_t ws_bytes, void *stream)
{
    int rc = check_stage(h, 1, "mlpg_integrate");
    if (rc) return rc;
    MLPG_CHECK(rk_order >= 0 && rk_order <= 2, MLPG_ERR_ARG, "mlpg_integrate: rk_order must be 0, 1 or 2");
    Problem *P = h;
    hipStream_t s = S(stream);
    P->stage = 1;   // the blocks are rebuilt; the operators must be assembled again
    P->rk_order = rk_order;
    P->n_blocks = P->n_mat * (1 + P->dim) + P->dim * P->dim + 2 * P->dim;
    rc = bind_stage(*P, P->own_int, workspace, ws_bytes, "mlpg_integrate",
                    [&](Problem &Q, Arena &A) { layout_integrate(Q, A); });
    if (rc) return rc;
    P->ws_int = workspace;
    P->gen++;
    MLPG_HIP(hipMemsetAsync(P->blocks.p, 0, sizeof(double) * P->n_blocks * P->nnz, s));
    MLPG_HIP(hipMemsetAsync(P->E.p, 0, sizeof(double) * P->nnz, s));
    MLPG_HIP(hipMemsetAsync(P->counters.p, 0, sizeof(unsigned long long) * kNumCounters, s));
    MLPG_HIP(hipMemsetAsync(P->bq_nact.p, 0, sizeof(int32_t) * std::max<int64_t>(1, P->n_bq), s));
    hipError_t e = P->dim == 2 ? launch_integrate2d(*P, s) : launch_integrate3d(*P, s);
    if (e == hipErrorInvalidValue) {
        set_error("mlpg_integrate: a cell has more candidate functions (" + std::to_string(P->cand_max) +
                  ") than the per-cell capacity");
        return MLPG_ERR_CAPACITY;
    }
    MLPG_HIP(e);
    // surface rows (direction independent): offsets here, entries at assembly
    MLPG_HIP(launch_surface_count(*P, P->tmp_scnt.p, s));
    MLPG_HIP(launch_exclusive_scan(P->tmp_scnt.p, P->surf_off.p, P->n, s));
    unsigned long long cnt[kNumCounters];
    MLPG_HIP(hipMemcpyAsync(cnt, P->counters.p, sizeof(cnt), hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipMemcpyAsync(&P->nnz_s, P->surf_off.p + P->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipStreamSynchronize(s));
    P->fallbacks = (int64_t)cnt[kFallbacks];
    P->missing = (int64_t)cnt[kMissing];
    MLPG_CHECK(cnt[kOverflow] == 0, MLPG_ERR_CAPACITY, "mlpg_integrate: per-cell or per-point capacity exceeded");
    // two functions active at one quadrature point overlap, so a pair absent
    // from the pattern means the caller's overlap lists were incomplete
    MLPG_CHECK(cnt[kMissing] == 0, MLPG_ERR_ARG,
               "mlpg_integrate: " + std::to_string(cnt[kMissing]) +
                   " co-active function pairs are missing from the overlap lists");
    P->stage = 2;
    return MLPG_OK;
}

size_t mlpg_integrate_workspace_bytes(mlpg_handle h, int rk_order)
{
    if (!h || h->stage < 1 || rk_order < 0 || rk_order > 2) return 0;
    Problem Q;   // sizes only
    Q.n = h->n; Q.nnz = h->nnz; Q.n_bq = h->n_bq; Q.bq_kmax = h->bq_kmax; Q.dim = h->dim; Q.n_mat = h->n_mat;
    Q.n_fields = h->n_fields; Q.n_shells = h->n_shells;
    Arena A;
    layout_integrate(Q, A);
    return A.used;
}

int mlpg_get_pattern(mlpg_handle h, int64_t *row_off, int32_t *col, void *stream)
{
    int rc = check_stage(h, 1, "mlpg_get_pattern");
    if (rc) return rc;
    MLPG_CHECK(row_off && col, MLPG_ERR_ARG, "mlpg_get_pattern: null output");
    hipStream_t s = S(stream);
    MLPG_HIP(hipMemcpyAsync(row_off, h->row_off.p, sizeof(int64_t) * (h->n + 1), hipMemcpyDeviceToDevice, s));
    MLPG_HIP(hipMemcpyAsync(col, h->col.p, sizeof(int32_t) * h->nnz, hipMemcpyDeviceToDevice, s));
    return MLPG_OK;
}

int mlpg_get_blocks(mlpg_handle h, double *blocks, double *E, void *stream)
{
    int rc = check_stage(h, 2, "mlpg_get_blocks");
    if (rc) return rc;
    hipStream_t s = S(stream);
    if (blocks)
        MLPG_HIP(hipMemcpyAsync(blocks, h->blocks.p, sizeof(double) * h->n_blocks * h->nnz, hipMemcpyDeviceToDevice,
                                s));
    if (E) MLPG_HIP(hipMemcpyAsync(E, h->E.p, sizeof(double) * h->nnz, hipMemcpyDeviceToDevice, s));
    return MLPG_OK;
}

int mlpg_assemble(mlpg_handle h, int n_ord, const double *omega, const double *w, int n_mat, const double *sigma_t,
                  const double *sigma_s, double inv_c_dt, const double *tau, int precision, void *workspace,
                  size_t ws_bytes, void *stream)
{
    int rc = check_stage(h, 2, "mlpg_assemble");
    if (rc) return rc;
    Problem *P = h;
    MLPG_CHECK(n_ord >= 1 && n_ord <= 256, MLPG_ERR_ARG, "mlpg_assemble: n_ord must be in [1, 256]");
    MLPG_CHECK(omega && w && sigma_t && sigma_s && tau, MLPG_ERR_ARG, "mlpg_assemble: null pointer");
    MLPG_CHECK(n_mat >= P->n_mat && n_mat <= 8, MLPG_ERR_ARG,
               "mlpg_assemble: n_mat must cover every material of the regions (and be <= 8)");
    MLPG_CHECK(inv_c_dt >= 0.0 && std::isfinite(inv_c_dt), MLPG_ERR_ARG, "mlpg_assemble: 1/(c dt) must be >= 0");
    MLPG_CHECK(precision == MLPG_FP64 || precision == MLPG_MIXED, MLPG_ERR_ARG,
               "mlpg_assemble: precision must be MLPG_FP64 or MLPG_MIXED");
    for (int g = 0; g < n_mat; ++g)
        MLPG_CHECK(sigma_t[g] >= 0.0 && sigma_s[g] >= 0.0 && sigma_s[g] <= sigma_t[g], MLPG_ERR_ARG,
                   "mlpg_assemble: need 0 <= sigma_s <= sigma_t");
    hipStream_t s = S(stream);
    const int d = P->dim;
    // The state Psi^{n-1}, Phi sits at the start of the assembly workspace.
    // It is kept when the ordinate count is unchanged: in place when the same
    // workspace comes back, copied from the previous one otherwise (which must
    // then stay valid until this call returns).
    const bool keep = P->psi.p && P->psi.count == (size_t)P->n * n_ord && P->phi.p;
    double *old_psi = P->psi.p, *old_phi = P->phi.p;
    DevBuf<char> prev_own;
    if (!workspace && P->own_asm.owned) {
        // a library-owned workspace is replaced only after the state is copied
        prev_own = P->own_asm;
        P->own_asm.p = nullptr;
        P->own_asm.count = 0;
        P->own_asm.owned = false;
    }
    rc = bind_stage(*P, P->own_asm, workspace, ws_bytes, "mlpg_assemble",
                    [&](Problem &Q, Arena &A) { layout_assemble(Q, A, n_ord, precision); });
    if (rc) {
        if (prev_own.p) {
            P->own_asm.release();
            P->own_asm = prev_own;
        }
        return rc;
    }
    P->stage = 2;         // until the new operators are complete
    P->binv_ok = false;   // the patch inverses belong to the previous operators
    P->ws_asm = workspace;
    P->gen++;
    const size_t nm = (size_t)P->n * n_ord;
    if (keep) {
        if (P->psi.p != old_psi)
            MLPG_HIP(hipMemcpyAsync(P->psi.p, old_psi, sizeof(double) * nm, hipMemcpyDeviceToDevice, s));
        if (P->phi.p != old_phi)
            MLPG_HIP(hipMemcpyAsync(P->phi.p, old_phi, sizeof(double) * P->n, hipMemcpyDeviceToDevice, s));
    } else {
        MLPG_HIP(hipMemsetAsync(P->psi.p, 0, sizeof(double) * nm, s));
        MLPG_HIP(hipMemsetAsync(P->phi.p, 0, sizeof(double) * P->n, s));
    }
    if (prev_own.p) {
        MLPG_HIP(hipStreamSynchronize(s));
        prev_own.release();
    }
    P->n_ord = n_ord;
    P->a0 = inv_c_dt;
    P->precision = precision;
    P->nsL = 1 + d + d * (d + 1) / 2;
    P->nsMD = 1 + d;
    P->nfaces = 2 * d;
    P->omega_h.assign(omega, omega + (size_t)n_ord * d);
    P->w_h.assign(w, w + n_ord);
    MLPG_HIP(launch_assemble(*P, sigma_t, sigma_s, tau, s));
    {
        // operators of the diffusion-synthetic acceleration (two values per pattern entry)
        std::vector<double> st(P->n_mat), sa(P->n_mat), ss(P->n_mat);
        for (int g = 0; g < P->n_mat; ++g) {
            st[g] = sigma_t[g] + inv_c_dt;
            sa[g] = sigma_t[g] - sigma_s[g] + inv_c_dt;
            ss[g] = sigma_s[g];
        }
        MLPG_HIP(launch_dsa_assemble(*P, st.data(), sa.data(), ss.data(), s));
    }
    // per-ordinate coefficient tables
    std::vector<double> cL((size_t)n_ord * P->nsL), cMD((size_t)n_ord * P->nsMD), cF((size_t)n_ord * P->nfaces);
    for (int m = 0; m < n_ord; ++m) {
        const double *W = omega + (size_t)m * d;
        double *l = &cL[(size_t)m * P->nsL];
        int k = 0;
        l[k++] = 1.0;
        for (int a = 0; a < d; ++a) l[k++] = W[a];
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b) l[k++] = W[a] * W[b];
        cMD[(size_t)m * P->nsMD] = 1.0;
        for (int a = 0; a < d; ++a) cMD[(size_t)m * P->nsMD + 1 + a] = W[a];
        for (int f = 0; f < P->nfaces; ++f) {
            double wn = ((f & 1) ? 1.0 : -1.0) * W[f >> 1];
            cF[(size_t)m * P->nfaces + f] = wn > 0.0 ? wn : 0.0;
        }
    }
    MLPG_HIP(hipMemcpyAsync(P->coefL.p, cL.data(), sizeof(double) * cL.size(), hipMemcpyHostToDevice, s));
    MLPG_HIP(hipMemcpyAsync(P->coefMD.p, cMD.data(), sizeof(double) * cMD.size(), hipMemcpyHostToDevice, s));
    MLPG_HIP(hipMemcpyAsync(P->coefF.p, cF.data(), sizeof(double) * cF.size(), hipMemcpyHostToDevice, s));
    MLPG_HIP(hipMemcpyAsync(P->omega.p, omega, sizeof(double) * n_ord * d, hipMemcpyHostToDevice, s));
    MLPG_HIP(hipMemcpyAsync(P->wq.p, w, sizeof(double) * n_ord, hipMemcpyHostToDevice, s));
    // surface rows (offsets from the integration)
    MLPG_HIP(launch_surface_fill(*P, nullptr, s));
    MLPG_HIP(launch_jacobi(*P, s));
    std::vector<float> cL32, cF32;
    if (precision == MLPG_MIXED) {
        // FP32 copies used by the inner FP32 solver (values rounded once)
        cL32.assign(cL.begin(), cL.end());
        cF32.assign(cF.begin(), cF.end());
        MLPG_HIP(launch_cast_f32(P->sL.p, P->sL32.p, (int64_t)P->nnz * P->nsL, s));
        if (P->nnz_s) MLPG_HIP(launch_cast_f32(P->surf_val.p, P->surf_val32.p, P->nnz_s * P->nfaces, s));
        MLPG_HIP(launch_cast_f32(P->dinv.p, P->dinv32.p, (int64_t)P->n * n_ord, s));
        MLPG_HIP(hipMemcpyAsync(P->coefL32.p, cL32.data(), sizeof(float) * cL32.size(), hipMemcpyHostToDevice, s));
        MLPG_HIP(hipMemcpyAsync(P->coefF32.p, cF32.data(), sizeof(float) * cF32.size(), hipMemcpyHostToDevice, s));
    }
    MLPG_HIP(hipStreamSynchronize(s));   // host staging vectors go out of scope
    MLPG_HIP(hipGetLastError());
    P->ws_slv_key = 0;   // the solve layout depends on the ordinates and the precision
    P->stage = 3;
    return MLPG_OK;
}

size_t mlpg_assemble_workspace_bytes(mlpg_handle h, int n_ord, int precision)
{
    if (!h || h->stage < 2 || n_ord < 1 || n_ord > 256 || (precision != MLPG_FP64 && precision != MLPG_MIXED))
        return 0;
    Problem Q;   // sizes only
    Q.n = h->n; Q.nnz = h->nnz; Q.dim = h->dim; Q.nnz_s = h->nnz_s;
    Arena A;
    layout_assemble(Q, A, n_ord, precision);
    return A.used;
}

int mlpg_apply(mlpg_handle h, int which, const double *X, double *Y, void *stream)
{
    int rc = check_stage(h, 3, "mlpg_apply");
    if (rc) return rc;
    MLPG_CHECK(X && Y, MLPG_ERR_ARG, "mlpg_apply: null pointer");
    Problem *P = h;
    SpmvArgs a;
    a.x = X;
    a.y = Y;
    switch (which) {
    case MLPG_OP_L:
        a.vals = P->sL.p; a.ns = P->nsL; a.coef = P->coefL.p; a.surface = 1; a.sval = P->surf_val.p;
        a.coefF = P->coefF.p;
        break;
    case MLPG_OP_T: a.vals = P->sMD.p; a.ns = P->nsMD; a.coef = P->coefMD.p; a.xs = P->a0; break;
    case MLPG_OP_MS: a.vals = P->sMS.p; a.ns = P->nsMD; a.coef = P->coefMD.p; break;
    case MLPG_OP_SRC: a.vals = P->sMD.p; a.ns = P->nsMD; a.coef = P->coefMD.p; break;
    default: set_error("mlpg_apply: unknown operator"); return MLPG_ERR_ARG;
    }
    MLPG_HIP(launch_spmv(*P, a, S(stream)));
    return MLPG_OK;
}

// Binds the solve workspace for the options; the patch inverses are built
// when they are not current (new operators, or a layout that moved them).
static int bind_solve(Problem &P, const mlpg_solve_opts &o, void *ws, size_t ws_bytes, const char *who, hipStream_t s)
{
    const double *old_binv = P.binv.p;
    int rc = bind_stage(P, P.own_slv, ws, ws_bytes, who, [&](Problem &Q, Arena &A) { layout_solve(Q, A, o); });
    if (rc) return rc;
    P.ws_slv = ws;
    if (o.precond == MLPG_PRECOND_PATCH) {
        if (P.binv.p != old_binv) P.binv_ok = false;
        if (!P.patches_ok) {
            rc = build_patches(P, s);
            if (rc) return rc;
            P.patches_ok = true;
        }
        if (!P.binv_ok) {
            rc = build_patch_inverses(P, s);
            if (rc) return rc;
            P.binv_ok = true;
        }
    } else {
        P.binv_ok = false;   // the layout has no inverses
    }
    return MLPG_OK;
}

static int check_opts(const mlpg_solve_opts &o, const char *who)
{
    const std::string w(who);
    MLPG_CHECK(o.tol_inner > 0 && o.tol_outer > 0, MLPG_ERR_ARG, w + ": tolerances must be positive");
    MLPG_CHECK(o.restart_inner >= 1 && o.restart_inner <= kMaxRestart && o.restart_outer >= 1 &&
                   o.restart_outer <= kMaxRestart,
               MLPG_ERR_ARG, w + ": restart lengths must be in [1, 60]");
    MLPG_CHECK(o.max_inner >= 1 && o.max_outer >= 0 && o.check_every >= 1 && o.max_refine >= 0, MLPG_ERR_ARG,
               w + ": iteration limits must be positive");
    MLPG_CHECK(P_ok_lo(o), MLPG_ERR_ARG, w + ": tol_inner_lo must be in (0, 1)");
    MLPG_CHECK(o.accel == MLPG_ACCEL_NONE || o.accel == MLPG_ACCEL_DSA, MLPG_ERR_ARG,
               w + ": accel must be MLPG_ACCEL_NONE or MLPG_ACCEL_DSA");
    MLPG_CHECK(o.precond == MLPG_PRECOND_JACOBI || o.precond == MLPG_PRECOND_PATCH, MLPG_ERR_ARG,
               w + ": precond must be MLPG_PRECOND_JACOBI or MLPG_PRECOND_PATCH");
    return MLPG_OK;
}

size_t mlpg_solve_workspace_bytes(mlpg_handle h, const mlpg_solve_opts *opts)
{
    if (!h || h->stage < 3) return 0;
    mlpg_solve_opts o;
    mlpg_default_opts(&o);
    if (opts) o = *opts;
    if (check_opts(o, "mlpg_solve_workspace_bytes")) return 0;
    Problem Q;   // sizes only
    Q.n = h->n; Q.n_ord = h->n_ord; Q.precision = h->precision; Q.nbsq = h->nbsq;
    Arena A;
    layout_solve(Q, A, o);
    return A.used;
}

int mlpg_apply_patch_precond(mlpg_handle h, const double *X, double *Y, int64_t *n_patches, void *workspace,
                             size_t ws_bytes, void *stream)
{
    int rc = check_stage(h, 3, "mlpg_apply_patch_precond");
    if (rc) return rc;
    MLPG_CHECK(X && Y && X != Y, MLPG_ERR_ARG, "mlpg_apply_patch_precond: need distinct X and Y");
    Problem *P = h;
    hipStream_t s = S(stream);
    mlpg_solve_opts o;
    mlpg_default_opts(&o);
    o.precond = MLPG_PRECOND_PATCH;
    rc = bind_solve(*P, o, workspace, ws_bytes, "mlpg_apply_patch_precond", s);
    if (rc) return rc;
    PatchPrecT<double> pp = patch_prec<double>(*P, P->binv.p);
    MLPG_HIP(launch_patch_apply<double>(pp, P->n_ord, X, Y, false, nullptr, s));
    if (n_patches) *n_patches = P->npatch;
    return MLPG_OK;
}

int mlpg_set_autotune(int mode)
{
    MLPG_CHECK(mode >= 0 && mode <= 2, MLPG_ERR_ARG, "mlpg_set_autotune: mode must be 0, 1 or 2");
    set_autotune(mode);
    return MLPG_OK;
}

int mlpg_get_tuning(int cap, mlpg_tune_entry *out)
{
    MLPG_CHECK(cap >= 0 && (cap == 0 || out), MLPG_ERR_ARG, "mlpg_get_tuning: need cap >= 0 and out");
    return get_tuning(cap, out);
}

int mlpg_set_tuning(const mlpg_tune_entry *entry)
{
    MLPG_CHECK(entry, MLPG_ERR_ARG, "mlpg_set_tuning: null entry");
    const std::string why = set_tuning(*entry);
    MLPG_CHECK(why.empty(), MLPG_ERR_ARG, "mlpg_set_tuning: " + why);
    return MLPG_OK;
}

void mlpg_default_opts(mlpg_solve_opts *o)
{
    if (!o) return;
    o->tol_inner = 1e-13;
    o->tol_outer = 1e-12;
    o->restart_inner = 30;
    o->restart_outer = 30;
    o->max_inner = 3000;
    o->max_outer = 500;
    o->check_every = 3;
    o->tol_inner_lo = 3e-5;
    o->max_refine = 12;
    o->accel = MLPG_ACCEL_NONE;
    o->precond = MLPG_PRECOND_JACOBI;
    o->graphs = 0;
}

int mlpg_set_state(mlpg_handle h, const double *psi, void *stream)
{
    int rc = check_stage(h, 3, "mlpg_set_state");
    if (rc) return rc;
    MLPG_CHECK(psi, MLPG_ERR_ARG, "mlpg_set_state: null psi");
    Problem *P = h;
    hipStream_t s = S(stream);
    MLPG_HIP(hipMemcpyAsync(P->psi.p, psi, sizeof(double) * P->n * P->n_ord, hipMemcpyDeviceToDevice, s));
    MLPG_HIP(launch_ord_reduce(*P, P->psi.p, P->phi.p, nullptr, 1.0, s));
    return MLPG_OK;
}

int mlpg_get_state(mlpg_handle h, double *psi, double *phi, void *stream)
{
    int rc = check_stage(h, 3, "mlpg_get_state");
    if (rc) return rc;
    Problem *P = h;
    hipStream_t s = S(stream);
    if (psi) MLPG_HIP(hipMemcpyAsync(psi, P->psi.p, sizeof(double) * P->n * P->n_ord, hipMemcpyDeviceToDevice, s));
    if (phi) MLPG_HIP(hipMemcpyAsync(phi, P->phi.p, sizeof(double) * P->n, hipMemcpyDeviceToDevice, s));
    return MLPG_OK;
}

int mlpg_point_values(mlpg_handle h, const double *coef, double *out, void *stream)
{
    int rc = check_stage(h, 2, "mlpg_point_values");
    if (rc) return rc;
    MLPG_CHECK(coef && out, MLPG_ERR_ARG, "mlpg_point_values: null pointer");
    MLPG_HIP(launch_point_values(*h, coef, out, S(stream)));
    return MLPG_OK;
}

int mlpg_solve(mlpg_handle h, const double *q, const double *psi_b, double *phi_coef, double *phi_point,
               double *psi_out, const mlpg_solve_opts *opts, mlpg_solve_info *info, void *workspace,
               size_t ws_bytes, void *stream)
{
    int rc = check_stage(h, 3, "mlpg_solve");
    if (rc) return rc;
    MLPG_CHECK(q && phi_coef, MLPG_ERR_ARG, "mlpg_solve: q and phi_coef are required");
    mlpg_solve_opts o;
    mlpg_default_opts(&o);
    if (opts) o = *opts;
    rc = check_opts(o, "mlpg_solve");
    if (rc) return rc;
    Problem *P = h;
    hipStream_t s = S(stream);
    rc = bind_solve(*P, o, workspace, ws_bytes, "mlpg_solve", s);
    if (rc) return rc;
    {
        // launch shapes of the inner sweeps, measured once per problem shape
        // (on scratch vectors of this solve, before any graph is captured)
        const size_t nm = (size_t)P->n * P->n_ord;
        MLPG_HIP(hipMemsetAsync(P->t1.p, 0, sizeof(double) * nm, s));
        SpmvArgs a;
        a.vals = P->sL.p; a.ns = P->nsL; a.coef = P->coefL.p; a.x = P->t1.p; a.surface = 1; a.y = P->t2.p;
        a.sval = P->surf_val.p; a.coefF = P->coefF.p; a.colscale = P->wq.p; a.vout = P->bpsi.p; a.vsrc = P->t1.p;
        MLPG_HIP(tune_spmv<double>(*P, a, P->inner.V.p, sizeof(double) * P->inner.V.count, s));
        if (P->precision == MLPG_MIXED) {
            MLPG_HIP(hipMemsetAsync(P->r32.p, 0, sizeof(float) * nm, s));
            SpmvArgsT<float> b;
            b.vals = P->sL32.p; b.ns = P->nsL; b.coef = P->coefL32.p; b.x = P->r32.p; b.surface = 1;
            b.y = P->d32.p; b.sval = P->surf_val32.p; b.coefF = P->coefF32.p; b.colscale = P->wq.p;
            b.vout = P->inner32.w.p; b.vsrc = P->r32.p;
            MLPG_HIP(tune_spmv<float>(*P, b, P->inner32.V.p, sizeof(float) * P->inner32.V.count, s));
        }
    }
    const int64_t n = P->n;
    const int M = P->n_ord;
    SolveCounters c;
    c.o = &o;
    int64_t oits = 0, osweeps = 0;
    double ores = 0.0;
    bool oconv = true;
    // every exit after this point reports what was done so far
    auto finish = [&](int code) {
        if (info) {
            info->outer_iters = (int)oits;
            info->inner_solves = c.solves;
            info->inner_iters = c.its;
            info->inner_sweeps = c.sweeps;
            info->outer_res = ores;
            info->inner_res_max = c.res_max;
            info->converged = (code == MLPG_OK && c.conv && oconv) ? 1 : 0;
            info->refinements = (int)c.refinements;
            info->fp64_completions = (int)c.fp64_completions;
            info->accel_iters = c.accel_its;
        }
        return code;
    };
#define STEP_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));                 \
            return finish(MLPG_ERR_HIP);                                                  \
        }                                                                                 \
    } while (0)
    // F = (Mass + tau W.D)(a0 Psi^{n-1} + q) + inflow term   (T Psi^{n-1} + r)
    {
        SpmvArgs a;
        a.vals = P->sMD.p; a.ns = P->nsMD; a.coef = P->coefMD.p; a.x = P->psi.p; a.xs = P->a0; a.x2 = q;
        a.y = P->F.p;
        STEP_HIP(launch_spmv(*P, a, s));
        if (psi_b) STEP_HIP(launch_boundary_rhs(*P, psi_b, P->F.p, s));
    }
    // b_psi = L^-1 F, b_phi = D b_psi
    rc = inner_solve(*P, c, P->F.p, P->bpsi.p, s);
    if (rc) return finish(rc);
    STEP_HIP(launch_ord_reduce(*P, P->bpsi.p, P->bphi.p, nullptr, 1.0, s));
    // outer GMRES on (I - D L^-1 MS) Phi = b_phi from the previous Phi.  With
    // FP32 inner corrections the outer operator is linear only to about the
    // inner tolerance times 1/(1 - c), so the mixed path stops the outer
    // iteration at 1e-10 at the tightest (far inside its 1e-8 bar on Phi).
    const double tol_outer = P->precision == MLPG_MIXED ? std::max(o.tol_outer, kMixedOuterFloor) : o.tol_outer;
    if (o.accel == MLPG_ACCEL_DSA) {
        // flexible GMRES on Phi itself, the synthetic acceleration as its variable right preconditioner
        // (from the previous Phi)
        FlexPrecT<double> fx;
        fx.apply = dsa_flex_apply;
        fx.ctx = &c;
        fx.Z = P->dsa_Z.p;
        fx.zs = n;
        rc = gmres_batched<double>(*P, P->outer, op_outer, false, &c, nullptr, P->bphi.p, P->phi.p, n, 1,
                                   tol_outer, o.restart_outer, std::max(1, o.max_outer), 1, false, s, &oits,
                                   &osweeps, &ores, &oconv, nullptr, false, nullptr, false, &fx);
        if (rc) return finish(rc);
    } else {
        rc = gmres_batched<double>(*P, P->outer, op_outer, false, &c, nullptr, P->bphi.p, P->phi.p, n, 1,
                                   tol_outer, o.restart_outer, std::max(1, o.max_outer), 1, false, s, &oits,
                                   &osweeps, &ores, &oconv);
        if (rc) return finish(rc);
    }
    // recovery Psi = L^-1 MS Phi + b_psi
    {
        SpmvArgs a;
        a.vals = P->sMS.p; a.ns = P->nsMD; a.coef = P->coefMD.p; a.x = P->phi.p; a.x_bcast = 1; a.y = P->t1.p;
        STEP_HIP(launch_spmv(*P, a, s));
    }
    rc = inner_solve(*P, c, P->t1.p, P->t2.p, s);
    if (rc) return finish(rc);
    STEP_HIP(launch_add(P->psi.p, P->t2.p, P->bpsi.p, n * M, s));
    STEP_HIP(hipMemcpyAsync(phi_coef, P->phi.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (phi_point) STEP_HIP(launch_point_values(*P, P->phi.p, phi_point, s));
    if (psi_out) STEP_HIP(hipMemcpyAsync(psi_out, P->psi.p, sizeof(double) * n * M, hipMemcpyDeviceToDevice, s));
#undef STEP_HIP
    if (!(c.conv && oconv)) {
        set_error("mlpg_solve: the outer Krylov iteration reached max_outer before its tolerance");
        return finish(MLPG_ERR_NOT_CONVERGED);
    }
    return finish(MLPG_OK);
}

void mlpg_destroy(mlpg_handle h)
{
    if (!h) return;
    h->release();
    delete h;
}

}  // extern "C"
