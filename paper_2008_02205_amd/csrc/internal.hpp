// Internal declarations of libmlpg: the problem handle, device buffers and
// the kernel launchers shared between translation units.  Nothing here is
// part of the C ABI (include/mlpg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mlpg.h"

namespace mlpg {

constexpr int kCellCap2D = 32;     // polygon vertex capacity of a 2D cell
constexpr int kSegRule = 5;        // Gauss-Legendre points on a boundary edge
constexpr int kTriN = 5;           // conical-product order on a triangle (25 points)
constexpr int kTriRule = kTriN * kTriN;
constexpr int kBqAct = 32;         // active functions stored per boundary point (2D)
constexpr int kCandMax2D = 64;     // functions possibly active on one 2D cell
constexpr int kFaceCap3 = 40;      // face capacity of a 3D cell
constexpr int kFaceVerts3 = 16;    // vertex capacity of one face of a 3D cell
constexpr int kTetN = 2;           // conical-product order on a tetrahedron (8 points)
constexpr int kTetRule = kTetN * kTetN * kTetN;
constexpr int kTri3N = 2;          // conical-product order on a boundary triangle in 3D (4 points)
constexpr int kTri3Rule = kTri3N * kTri3N;
constexpr int kBqAct3 = 128;       // active functions stored per boundary point (3D)
constexpr int kCandMax3D = 512;    // functions possibly active on one 3D cell
constexpr int kTileRows3 = 8;      // most Gram rows per 3D tile without fields (their values sit in registers)
// 3D, one material without fields: the cells' weighted function values are
// written to panels in the integration workspace, a batch of cells at a
// time, and their Gram products formed on the matrix cores.  The region holds
// up to kGramCells panels of the estimated size below (the batch shrinks
// when a problem's panels are larger).
constexpr int64_t kGramCells = 1024;
constexpr size_t kGramPanelBytes = size_t(2) << 20;
constexpr int kMaxRestart = 60;   // longest GMRES restart cycle
constexpr int kChunkRestart = 30; // basis vectors a streaming pass holds in registers; longer cycles run
                                  // their passes in two chunks
constexpr int kDsaRestart = 30;   // restart of the diffusion solves of the synthetic acceleration
constexpr int kMaxFields = 8;    // smooth material fields per problem
constexpr int kMaxMat = 8;       // materials per problem
constexpr double kMixedOuterFloor = 1e-10;   // tightest outer tolerance of the mixed path
constexpr int kTagBox = -100;      // edge of the kernel box not on the domain
constexpr int kPatchMax = 16;      // points per patch of the block-Jacobi preconditioner

// Thread-local error message for mlpg_last_error.
void set_error(const std::string &msg);

#define MLPG_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::mlpg::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
            return MLPG_ERR_HIP;                                                          \
        }                                                                                 \
    } while (0)

#define MLPG_CHECK(cond, code, msg)                                                       \
    do {                                                                                  \
        if (!(cond)) {                                                                    \
            ::mlpg::set_error(msg);                                                       \
            return code;                                                                  \
        }                                                                                 \
    } while (0)

// Device buffer: a view into a stage workspace (bound by an Arena), or an
// allocation of its own (alloc: only for the helper entry points outside the
// four stages and for workspaces the library allocates when the caller
// passes none).
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t count = 0;
    bool owned = false;
    hipError_t alloc(size_t n) {
        if (n <= count && p && owned) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, (n ? n : 1) * sizeof(T));
        if (e == hipSuccess) {
            count = n;
            owned = true;
        } else {
            p = nullptr;
        }
        return e;
    }
    void bind(T *q, size_t n) {
        release();
        p = q;
        count = n;
        owned = false;
    }
    void release() {
        if (p && owned) (void)hipFree(p);
        p = nullptr;
        count = 0;
        owned = false;
    }
};

// Carves the buffers of one stage out of a workspace, in a fixed order with
// 256-byte alignment.  In measuring mode (base == nullptr) it only adds up
// the bytes, so that a stage's size query and the stage itself run the same
// layout code and agree to the byte.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    bool over = false;
    static size_t align(size_t b) { return (b + 255) & ~(size_t)255; }
    template <class T>
    void take(DevBuf<T> &b, size_t n) {
        const size_t bytes = align((n ? n : 1) * sizeof(T));
        if (base && used + bytes <= cap) b.bind((T *)(base + used), n);
        else b.bind(nullptr, n);
        if (base && used + bytes > cap) over = true;
        used += bytes;
    }
};

// Host-side quadrature tables (computed once, uploaded as kernel arguments
// or constant memory).
struct Rules {
    double tri_pts[kTriRule][2];
    double tri_w[kTriRule];
    double seg_pts[kSegRule];
    double seg_w[kSegRule];
    double tet_pts[kTetRule][3];
    double tet_w[kTetRule];
    double tri3_pts[kTri3Rule][2];
    double tri3_w[kTri3Rule];
};
const Rules &rules();
hipError_t upload_rules(hipStream_t s);   // copies the tables to __constant__ memory

// Gauss-Legendre on [-1,1] and Gauss-Jacobi (weight (1-x)^alpha) on [-1,1].
void gauss_legendre(int n, double *x, double *w);
void gauss_jacobi(int n, double alpha, double *x, double *w);

// Counters written by kernels (device, zeroed at each stage that uses them).
enum Counter { kFallbacks = 0, kMissing = 1, kOverflow = 2, kBadLists = 3, kNumCounters = 4 };

// Launch arguments a captured restart cycle depends on (pointers, values and
// the problem's layout generation); a graph is replayed only for an equal key.
struct GraphKey {
    const void *ptr[11] = {};
    double tol = 0.0;
    int64_t val[6] = {};
    void set(uint64_t gen, const void *op, const void *ctx, const void *dinv, const void *f, const void *x,
             const void *tolv, const void *binv, const void *V, const void *part, const void *H, const void *nact,
             double tol_, int64_t n, int nb, int k, int max_its, int fused)
    {
        const void *p[11] = {op, ctx, dinv, f, x, tolv, binv, V, part, H, nact};
        for (int i = 0; i < 11; ++i) ptr[i] = p[i];
        tol = tol_;
        const int64_t v[6] = {(int64_t)gen, n, nb, k, max_its, fused};
        for (int i = 0; i < 6; ++i) val[i] = v[i];
    }
    bool operator==(const GraphKey &o) const
    {
        for (int i = 0; i < 11; ++i)
            if (ptr[i] != o.ptr[i]) return false;
        for (int i = 0; i < 6; ++i)
            if (val[i] != o.val[i]) return false;
        return tol == o.tol;
    }
};
constexpr size_t kGraphCache = 8;   // captured cycles kept per Krylov space

// Batched GMRES workspace for `nb` simultaneous systems of `n` unknowns
// (ordinates as the fastest index); T is the storage type of the basis and
// vectors (partial sums, Hessenberg and rotations are FP64 either way).
template <class T>
struct KrylovT {
    int64_t n = 0;
    int nb = 0;
    int k = 0;
    int64_t vs = 0;          // element stride between basis vectors (n*nb plus padding)
    DevBuf<T> V;             // [(k+1)][vs]
    DevBuf<T> w, w2;         // [n][nb] operator outputs (alternating)
    DevBuf<T> z;             // [n][nb] dinv .* w, the next operator input
    DevBuf<T> r;             // [n][nb]
    DevBuf<double> vscale;   // [nb] 1/h_{j+1,j} of the newest column (0 once a system stops)
    DevBuf<double> pu, pw;   // [n][nb] FP64 partial u and w between the chunks of pass B (k > 30 only)
    DevBuf<double> part;     // [nblk][2k+2][nb] block partial sums
    DevBuf<double> h1, h2;   // [2k+2][nb] reduced projections, pass-B coefficients
    DevBuf<double> H;        // [nb][k+1][k] rotated Hessenberg (upper triangular part used)
    DevBuf<double> Ht;       // [nb][k][k+1] unrotated Hessenberg, by columns
    DevBuf<double> cs, sn;   // [nb][k]
    DevBuf<double> g;        // [nb][k+1]
    DevBuf<double> y;        // [k][nb]
    DevBuf<double> fnorm;    // [nb]
    DevBuf<double> beta;     // [nb]
    DevBuf<double> resid;    // [nb] relative residual of the last cycle
    DevBuf<int> active;      // [nb] 1 while the system iterates in this cycle
    DevBuf<int> done;        // [nb] 1 once converged (or out of steps)
    DevBuf<int> its;         // [nb] Arnoldi steps so far in this solve
    DevBuf<int> jend;        // [nb] columns built in this cycle
    DevBuf<int> nactive;     // [3] rotating active counters (the gates of consecutive steps)
    int *nactive_host = nullptr;   // pinned, host-visible mirrors of nactive (one slot per sweep in flight)
    int *nactive_hdev = nullptr;   // device address of nactive_host
    hipEvent_t ev[8] = {};
    int part_blocks = 0;
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;   // captured restart cycles
    hipStream_t capture_stream = nullptr;                       // where they are captured (default priority)
    hipGraphExec_t find_graph(const GraphKey &key) const;
    void add_graph(const GraphKey &key, hipGraphExec_t ge);
    // device buffers for nb systems of n unknowns, restart length up to k_
    void carve(Arena &A, int64_t n_, int nb_, int k_);
    hipError_t host_init();   // pinned host mirrors of the active counts, events (once per handle)
    void release();
};
using Krylov = KrylovT<double>;

// Patch block-Jacobi right preconditioner of the inner solves (patches.hip):
// patch p holds the points pidx[poff[p] .. poff[p+1]) and the inverse of
// L_m restricted to them, binv[boff[p] M + (i s + j) M + m].
template <class T>
struct PatchPrecT {
    int64_t npatch = 0;
    const int64_t *poff = nullptr;
    const int32_t *pidx = nullptr;
    const int64_t *boff = nullptr;
    const T *binv = nullptr;
};

struct Problem {
    int dim = 0;
    int64_t n = 0;
    int n_mat = 1;
    double dom_lo[3] = {0, 0, 0}, dom_hi[3] = {0, 0, 0};
    int n_regions = 0;
    DevBuf<double> reg_lo, reg_hi;
    DevBuf<int32_t> reg_mat;
    int n_fields = 0;                          // smooth material fields (mlpg_material_fields)
    double field_par[kMaxFields][4] = {};      // a, b, k, phase
    int field_mat[kMaxFields] = {};
    int n_shells = 0;                          // shells (mlpg_material_shells)
    double shell_par[kMaxFields][5] = {};      // centre (dim), inner and outer radius
    int shell_mat[kMaxFields] = {};

    DevBuf<double> x, R;
    DevBuf<int64_t> nb_off;
    DevBuf<int32_t> nb_idx;
    int64_t nnz_nb = 0;

    // cells: 2D polygons (nv, tags, verts) or 3D polyhedra (nf, fnv, ftags,
    // fverts: [n][kFaceCap3][kFaceVerts3][3])
    DevBuf<int32_t> nv, tags;
    DevBuf<double> verts, V, rho;
    DevBuf<int32_t> nf, fnv, ftags;
    DevBuf<double> fverts;
    int64_t oversize = 0, failed = 0;

    // boundary quadrature
    int64_t n_bq = 0;
    int bq_kmax = kBqAct;     // active functions stored per boundary point
    DevBuf<int64_t> bq_off;   // [n+1] first boundary point of each cell
    DevBuf<double> bq_y, bq_w, bq_N;
    DevBuf<int32_t> bq_face, bq_nact, bq_act;

    // pattern and blocks
    int64_t nnz = 0;
    DevBuf<int64_t> row_off, diag_pos;
    DevBuf<int32_t> col;
    int n_blocks = 0;
    int rk_order = -1;
    DevBuf<double> blocks, E;
    DevBuf<unsigned long long> counters;
    int64_t fallbacks = 0, missing = 0;
    int cand_max = 0;

    // assembled operators
    int n_ord = 0;
    int precision = MLPG_FP64;
    double a0 = 0.0;
    std::vector<double> omega_h, w_h;
    DevBuf<double> wq;                    // [M]
    DevBuf<double> omega;                 // [M][dim]
    int nsL = 0, nsMD = 0, nfaces = 0;
    DevBuf<double> sL, sMD, sMS;          // [nnz][nsL], [nnz][1+d], [nnz][1+d]
    DevBuf<double> coefL, coefMD, coefF;  // [M][nsL], [M][1+d], [M][2d]
    DevBuf<int64_t> surf_off;             // [n+1]
    DevBuf<int32_t> surf_col;
    DevBuf<double> surf_val;              // [nnz_s][2d]
    int64_t nnz_s = 0;
    DevBuf<double> dinv;                  // [n][M]

    // state and solver scratch
    DevBuf<double> psi, phi;              // [n][M], [n]
    DevBuf<double> F, bpsi, t1, t2;       // [n][M]
    DevBuf<double> bphi, ovec;            // [n]
    Krylov inner, outer;
    KrylovT<float> inner32;
    // mixed precision: FP32 copies of the L streams, coefficients, surface
    // values and Jacobi scaling; refinement scratch
    DevBuf<float> sL32, coefL32, coefF32, surf_val32, dinv32, r32, d32;
    DevBuf<double> mr, rn2, fn2, tolv;
    // diffusion-synthetic acceleration of the outer iteration: C, Ms on the
    // pattern, 1/diag(C), and the diffusion solve's workspace
    DevBuf<double> dsaC, dsaMs, dsa_dinv, dsa_r, dsa_x;
    DevBuf<double> dsa_Z;   // [restart_outer][n] the outer iteration's preconditioned vectors
    Krylov dsa;
    // patch block-Jacobi preconditioner (mlpg_solve_opts.precond): patches of
    // the current positions, block inverses of the current operators
    int64_t npatch = 0, nbsq = 0, patch_singular = 0;
    DevBuf<int64_t> poff, boff;
    DevBuf<int32_t> pidx;
    DevBuf<double> binv;
    DevBuf<float> binv32;
    bool patches_ok = false, binv_ok = false;

    // stage workspaces: the caller's (views) or, when the caller passes none,
    // one allocation per stage made by the library; temporaries of a stage
    // live in its workspace too
    DevBuf<char> own_geo, own_int, own_asm, own_slv;
    void *ws_geo = nullptr, *ws_int = nullptr, *ws_asm = nullptr, *ws_slv = nullptr;
    size_t ws_slv_key = 0;                  // hash of the solve layout last carved
    double reg_lo_h[64 * 3] = {}, reg_hi_h[64 * 3] = {};
    int32_t reg_mat_h[64] = {};
    int64_t ncell = 0;                      // cells of the patch grid
    DevBuf<int32_t> tmp_flags, tmp_cand;
    DevBuf<char> gram_ws;                   // 3D panels of weighted values (integration workspace)
    DevBuf<int64_t> tmp_bqc, tmp_key, tmp_s2, tmp_npc, tmp_off, tmp_pbase, tmp_scnt;
    DevBuf<unsigned long long> tmp_cnt, tmp_sing;
    DevBuf<double> tmp_work;
    int stage = 0;                        // 1 geometry, 2 integrated, 3 assembled
    uint64_t gen = 0;                     // bumped whenever a stage lays its buffers out again

    void release();
};

// Stage layouts (workspace.cpp): carve every buffer of a stage, in order.
// The inputs are the sizes the stage depends on; the Problem's sizes from
// earlier stages are read.
void layout_geometry(Problem &P, Arena &A, int64_t nnz_nb);
void layout_integrate(Problem &P, Arena &A);
void layout_assemble(Problem &P, Arena &A, int n_ord, int precision);
void layout_solve(Problem &P, Arena &A, const mlpg_solve_opts &o);
// Cells of the patch grid over the domain box for n points (patches.hip).
int64_t patch_grid_cells(int dim, int64_t n, const double *lo, const double *hi, double *h, int64_t dims[3]);

// Patch block-Jacobi preconditioner (patches.hip): patches of the current
// points, then the block inverses of the assembled operators (FP32 copies in
// the mixed path); out = M^-1 in (add: out += M^-1 in).
int build_patches(Problem &P, hipStream_t s);
int build_patch_inverses(Problem &P, hipStream_t s);
template <class T>
hipError_t launch_patch_apply(const PatchPrecT<T> &pp, int M, const T *in, T *out, bool add, const int *gate,
                              hipStream_t s);

// Progress callback (mlpg_set_progress); no-op when unset.
void report_progress(int level, int64_t iters, double resid);

// Kernel-class timing (mlpg_profile_*): prof_start returns -1 when off.
bool prof_on();
int prof_start(int cls, double bytes, hipStream_t s);
void prof_stop(int id, hipStream_t s);

// ---- kernel launchers -----------------------------------------------------
// Cell-list neighbour search (neighbors.hip).  Scratch: bounding box (8
// doubles), each point's cell [n], cell counts [max_cells], cell starts
// [max_cells + 1], points in cell order [n].
struct NbScratch {
    double *bbox = nullptr;
    int32_t *cell = nullptr;
    uint32_t *cnt = nullptr;
    int64_t *coff = nullptr;
    int32_t *pts = nullptr;
    int64_t max_cells = 0;
};
int64_t nb_max_cells(int64_t n);
size_t nb_scratch_bytes(int64_t n, int64_t max_cells);
NbScratch nb_scratch_at(void *base, int64_t n, int64_t max_cells);
hipError_t launch_neighbors_count(int dim, int64_t n, const double *x, const double *R, int64_t *counts,
                                  const NbScratch &sc, hipStream_t s);
hipError_t launch_neighbors_fill(int dim, int64_t n, const double *x, const double *R, const int64_t *off,
                                 int32_t *idx, const NbScratch &sc, hipStream_t s);
hipError_t launch_exclusive_scan(const int64_t *counts, int64_t *off, int64_t n, hipStream_t s);
// validates caller-supplied overlap lists (sets bits of *bad, see geometry.hip)
hipError_t launch_check_lists(int64_t n, int64_t total, const int64_t *off, const int32_t *idx,
                              unsigned long long *bad, hipStream_t s);

hipError_t launch_clip2d(Problem &P, hipStream_t s, int32_t *flags, int64_t *bq_count);
hipError_t launch_clip3d(Problem &P, hipStream_t s, int32_t *flags, int64_t *bq_count);
hipError_t launch_pattern(Problem &P, hipStream_t s);
hipError_t launch_integrate2d(Problem &P, hipStream_t s);
hipError_t launch_integrate3d(Problem &P, hipStream_t s);

hipError_t launch_assemble(Problem &P, const double *sig_t, const double *sig_s, const double *tau,
                           hipStream_t s);
hipError_t launch_surface_count(Problem &P, int64_t *counts, hipStream_t s);
hipError_t launch_surface_fill(Problem &P, const double *omega_unused, hipStream_t s);
hipError_t launch_jacobi(Problem &P, hipStream_t s);
// C and Ms of the diffusion-synthetic preconditioner (mlpg_solve_opts.accel);
// sig_*: host [n_mat] effective cross sections (a0 included in sig_t, sig_a)
hipError_t launch_dsa_assemble(Problem &P, const double *sig_t_eff, const double *sig_a_eff, const double *sig_s,
                               hipStream_t s);
// y = A (dinv .* x) for one vector over the pattern (dinv may be NULL; gate as in the solvers)
hipError_t launch_csr_spmv(Problem &P, const double *vals, const double *x, const double *dinv, double *y,
                           const int *gate, hipStream_t s);

// y[i][m] = sum_p (sum_b coef[m][b] vals[p][b]) * xin[col[p]][m]  (+ surface part)
// with xin = xs*x + x2, optional right preconditioner dinv and per-ordinate
// scale colscale; T is the value/vector type (FP32 accumulates in FP32).
template <class T>
struct SpmvArgsT {
    const T *vals = nullptr;
    int ns = 0;
    const T *coef = nullptr;          // [M][ns]
    const T *x = nullptr;             // [n][M] or [n] when x_bcast
    int x_bcast = 0;
    const T *x2 = nullptr;            // optional second input added: x_eff = xs*x + x2
    T xs = 1;
    const T *dinv = nullptr;          // optional [n][M] right preconditioner
    const double *colscale = nullptr; // optional [M] per-ordinate scale of x
    int surface = 0;                  // add sum_f max(0, W.n_f) S_f
    const T *sval = nullptr;          // surface values [nnz_s][2d] (T copy)
    const T *coefF = nullptr;         // [M][2d]
    T *y = nullptr;
    const T *yadd = nullptr;          // optional: y = yadd + ysign * (A x)
    int ysign = 1;
    T *vout = nullptr;                // optional: vout[i][m] = colscale[m] vsrc[i][m] on each own row
    const T *vsrc = nullptr;          //   (vsrc defaults to x)
    const int *gate = nullptr;        // optional: the launch does nothing when *gate == 0
};
using SpmvArgs = SpmvArgsT<double>;
template <class T>
hipError_t launch_spmv(Problem &P, const SpmvArgsT<T> &a, hipStream_t s);
// measures the sweep's launch shapes for this problem's size once per process,
// reading the scratch region `evict` before each timed launch (ops.hip)
template <class T>
hipError_t tune_spmv(Problem &P, const SpmvArgsT<T> &a, const void *evict, size_t evict_bytes, hipStream_t s);
void set_autotune(int mode);   // 0 off, 1 on, 2 clear the table
int get_tuning(int cap, mlpg_tune_entry *out);
std::string set_tuning(const mlpg_tune_entry &t);   // "" or what is wrong with t
hipError_t launch_to_float_scaled(int64_t n, int M, const double *r, const double *rn2, const double *fn2, double tol,
                                  float *out, hipStream_t s);
hipError_t launch_axpy_from_float(int64_t n, int M, double *x, const float *d, const double *rn2, hipStream_t s);
hipError_t launch_cast_f32(const double *in, float *out, int64_t count, hipStream_t s);
hipError_t launch_point_values(Problem &P, const double *coef, double *out, hipStream_t s);
hipError_t launch_boundary_rhs(Problem &P, const double *psib, double *F, hipStream_t s);
hipError_t launch_ord_reduce(Problem &P, const double *X, double *out, const double *base, double sign,
                             hipStream_t s);
hipError_t launch_add(double *y, const double *a, const double *b, int64_t count, hipStream_t s);

// Batched GMRES driver.  The operator callback computes out = A(in) for all
// systems; `precond` (may be null) is the right point-Jacobi scaling.
// One operator application out = A(dinv .* (colscale .* in)).  When the
// operator supports it (`fused`), it also writes vout = colscale .* vsrc on
// its own rows, which normalises the next Krylov vector inside the SpMV.
template <class T>
struct OpCallT {
    const T *in = nullptr;
    const T *dinv = nullptr;
    const double *colscale = nullptr;
    T *vout = nullptr;
    const T *vsrc = nullptr;
    T *out = nullptr;
    const int *gate = nullptr;
};
using OpCall = OpCallT<double>;
template <class T>
using OpFnT = int (*)(Problem &P, const OpCallT<T> &c, hipStream_t s, void *ctx);
using OpFn = OpFnT<double>;
// A variable right preconditioner (flexible GMRES): z_j = M_j^-1 v_j is
// computed by `apply` before each operator application and kept in Z (slot j
// at Z + j * zs, k slots); the iterate is updated with Z y, so the residual
// stays that of the unpreconditioned system whatever M_j does.
template <class T>
struct FlexPrecT {
    int (*apply)(Problem &P, const T *v, T *z, hipStream_t s, void *ctx) = nullptr;
    void *ctx = nullptr;
    T *Z = nullptr;
    int64_t zs = 0;
};
template <class T>
int gmres_batched(Problem &P, KrylovT<T> &K, OpFnT<T> op, bool fused, void *ctx, const T *dinv, const T *f, T *x,
                  int64_t n, int nb, double tol, int restart, int max_its, int lag, bool x_zero, hipStream_t s,
                  int64_t *its_sum, int64_t *sweeps, double *res_max, bool *converged,
                  const double *tolv = nullptr, bool cheap_op = false,   // optional per-system relative tolerance (device [nb])
                  const PatchPrecT<T> *pp = nullptr,    // patch block-Jacobi instead of dinv (dinv must be null)
                  bool graphs = false,                  // replay restart cycles from captured HIP graphs
                  const FlexPrecT<T> *fx = nullptr);    // flexible right preconditioner (unfused operator only)
// out[m] = sum_i x[i][m]^2 for the nb systems of K's shape
hipError_t batched_norm2(KrylovT<double> &K, const double *x, double *out, hipStream_t s);

}  // namespace mlpg
