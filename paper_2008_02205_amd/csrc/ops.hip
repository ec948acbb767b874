// Assembly of the per-ordinate operators of Sec. 4.2 into
// direction-independent value streams, and the operator applications used
// by the solver: the ordinate-batched SpMV, the all-ordinate reduction D,
// the point values of Eq. flux-expansion and the inflow term of r.
//
// Streams are stored row-major interleaved ([nnz][ns]) so that one nonzero's
// values are read together; every lane of a row owns one ordinate and
// combines the streams with its own coefficients (products of Omega_m
// components) in registers, so L_m is never stored per ordinate.
#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace mlpg {

namespace {

__device__ __forceinline__ int64_t row_of(const int64_t *row_off, int64_t n, int64_t p)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (row_off[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct AsmArgs {
    int64_t n, nnz;
    int dim, G;
    const int64_t *row_off;
    const double *blocks;
    const double *tau;
    double a0;
    double sig_t[8], sig_s[8];
    double *sL, *sMD, *sMS;
    int nsL;
};

// One thread per nonzero: combine the material blocks with sigma_t, sigma_s,
// a0 = 1/(c dt) and tau_i (Eq. weak-transport, operator forms of Sec. 4.2).
__global__ void assemble_kernel(AsmArgs a)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.nnz) return;
    const int d = a.dim, G = a.G;
    const int64_t nnz = a.nnz;
    const int64_t i = row_of(a.row_off, a.n, p);
    const double tau = a.tau[i];
    double mass = 0.0, smass_t = 0.0, smass_s = 0.0;
    double D[3] = {0, 0, 0}, Dt[3] = {0, 0, 0}, Ds[3] = {0, 0, 0};
    for (int g = 0; g < G; ++g) {
        double mg = a.blocks[(int64_t)(g * (1 + d)) * nnz + p];
        mass += mg;
        smass_t += a.sig_t[g] * mg;
        smass_s += a.sig_s[g] * mg;
        for (int al = 0; al < d; ++al) {
            double dg = a.blocks[(int64_t)(g * (1 + d) + 1 + al) * nnz + p];
            D[al] += dg;
            Dt[al] += a.sig_t[g] * dg;
            Ds[al] += a.sig_s[g] * dg;
        }
    }
    const int kb = G * (1 + d);
    double *L = a.sL + p * a.nsL;
    L[0] = a.a0 * mass + smass_t;
    for (int al = 0; al < d; ++al) L[1 + al] = (a.a0 * tau - 1.0) * D[al] + tau * Dt[al];
    // SUPG second-order term: tau_i sum_ab W^a W^b K^ab, with the symmetric
    // pair K^ab + K^ba folded into one stream for a < b.
    int s = 1 + d;
    for (int al = 0; al < d; ++al)
        for (int be = al; be < d; ++be) {
            double k = a.blocks[(int64_t)(kb + al * d + be) * nnz + p];
            if (be != al) k += a.blocks[(int64_t)(kb + be * d + al) * nnz + p];
            L[s++] = tau * k;
        }
    double *MD = a.sMD + p * (1 + d);
    double *MS = a.sMS + p * (1 + d);
    const double f4pi = 1.0 / (4.0 * M_PI);
    MD[0] = mass;
    MS[0] = f4pi * smass_s;
    for (int al = 0; al < d; ++al) {
        MD[1 + al] = tau * D[al];
        MS[1 + al] = f4pi * tau * Ds[al];
    }
}

// Surface rows: count entries of row i with any nonzero face block.
__global__ void surface_count_kernel(int64_t n, int64_t nnz, int nf, int sb, const int64_t *row_off,
                                     const double *blocks, int64_t *counts)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t c = 0;
    for (int64_t p = row_off[i]; p < row_off[i + 1]; ++p) {
        bool nz = false;
        for (int f = 0; f < nf; ++f) nz |= blocks[(int64_t)(sb + f) * nnz + p] != 0.0;
        c += nz;
    }
    counts[i] = c;
}

__global__ void surface_fill_kernel(int64_t n, int64_t nnz, int nf, int sb, const int64_t *row_off,
                                    const int32_t *col, const double *blocks, const int64_t *soff, int32_t *scol,
                                    double *sval)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t o = soff[i];
    for (int64_t p = row_off[i]; p < row_off[i + 1]; ++p) {
        bool nz = false;
        for (int f = 0; f < nf; ++f) nz |= blocks[(int64_t)(sb + f) * nnz + p] != 0.0;
        if (!nz) continue;
        scol[o] = col[p];
        for (int f = 0; f < nf; ++f) sval[o * nf + f] = blocks[(int64_t)(sb + f) * nnz + p];
        o++;
    }
}

// dinv[i][m] = 1 / L_m[i,i]
__global__ void jacobi_kernel(int64_t n, int M, int nsL, int nf, const int64_t *diag_pos, const double *sL,
                              const double *coefL, const int64_t *soff, const int32_t *scol, const double *sval,
                              const double *coefF, double *dinv)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * M) return;
    int64_t i = t / M;
    int m = (int)(t - i * M);
    const double *v = sL + diag_pos[i] * nsL;
    double d = 0.0;
    for (int b = 0; b < nsL; ++b) d += coefL[m * nsL + b] * v[b];
    for (int64_t p = soff[i]; p < soff[i + 1]; ++p)
        if (scol[p] == i)
            for (int f = 0; f < nf; ++f) d += coefF[m * nf + f] * sval[p * nf + f];
    dinv[t] = d != 0.0 ? 1.0 / d : 1.0;
}

template <class T>
struct SpmvK {
    int64_t n;
    int M;
    const int64_t *row_off;
    const int32_t *col;
    const T *vals;
    const T *coef;
    const T *x;
    int x_bcast;
    const T *x2;
    T xs;
    const T *dinv;
    const double *colscale;
    const int64_t *soff;
    const int32_t *scol;
    const T *sval;
    const T *coefF;
    int nf;
    T *y;
    const T *yadd;
    int ysign;
    T *vout;
    const T *vsrc;
    const int *gate;
    int64_t items_per_block;   // wave kernel: contiguous items per workgroup
    int nxcd;                  // workgroups are dealt round-robin to this many dies
};

// Input modes of the SpMV (compile-time, so that the gathers of one row
// carry no branches and issue back to back):
enum { IN_PLAIN = 0, IN_DINV = 1, IN_BCAST = 2, IN_X2 = 3 };

// x value of column j for ordinate m: xs*x, times dinv (IN_DINV), the
// ordinate-independent x[j] (IN_BCAST), or plus a second input (IN_X2).
template <int MODE, class T>
__device__ __forceinline__ T xin(const SpmvK<T> &k, int64_t j, int m)
{
    const int64_t o = j * k.M + m;
    if (MODE == IN_BCAST) return k.xs * k.x[j];
    T xv = k.xs * k.x[o];
    if (MODE == IN_X2) xv += k.x2[o];
    if (MODE == IN_DINV) xv *= k.dinv[o];
    return xv;
}

template <class T>
__device__ __forceinline__ void spmv_finish(const SpmvK<T> &k, int64_t i, int m, T acc)
{
    const int64_t o = i * k.M + m;
    const T sc = k.colscale ? (T)k.colscale[m] : (T)1;
    if (k.vout) k.vout[o] = sc * (k.vsrc ? k.vsrc[o] : k.x[o]);
    acc *= sc;
    k.y[o] = k.yadd ? k.yadd[o] + (T)k.ysign * acc : acc;
}

// Surface rows (few): the outflow blocks weighted by max(0, W.n_f).
template <int MODE, class T>
__device__ __forceinline__ T spmv_surface(const SpmvK<T> &k, int64_t i, int m)
{
    T acc = 0;
    T cf[6] = {0, 0, 0, 0, 0, 0};
    for (int f = 0; f < k.nf; ++f) cf[f] = k.coefF[m * k.nf + f];
    for (int64_t p = k.soff[i]; p < k.soff[i + 1]; ++p) {
        T a = 0;
        for (int f = 0; f < k.nf; ++f) a += cf[f] * k.sval[p * k.nf + f];
        acc += a * xin<MODE>(k, k.scol[p], m);
    }
    return acc;
}

__device__ __forceinline__ double bcast(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float bcast(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Wave-per-row SpMV (used when the ordinates fill whole waves): each wave
// owns one (row, 64-ordinate chunk).  The row index is wave-uniform, so the
// row's column indices and stream values are read with scalar loads straight
// into SGPRs (read-only kernel arguments, no vector broadcast needed) and
// combined with the lane's own coefficients; the x gathers of eight nonzeros
// are issued back to back so that their latencies overlap.
template <int NS, class T, int MODE>
__global__ __launch_bounds__(512) void spmv_wave_kernel(SpmvK<T> k, const int64_t *__restrict__ row_off,
                                                        const int32_t *__restrict__ col,
                                                        const T *__restrict__ vals)
{
    if (k.gate && *k.gate == 0) return;
    // Workgroups are dealt round-robin to the dies (XCDs), each with its own
    // L2; renumber them so that every die walks one contiguous range of rows
    // and keeps that range's x neighbourhood in its own L2.
    const int G = gridDim.x, X = k.nxcd;
    const int bx = blockIdx.x;
    const int per = G / X;                    // the grid is a multiple of X
    const int lb = (bx % X) * per + bx / X;
    const int lane = threadIdx.x & 63;
    const int nchunk = (k.M + 63) >> 6;
    const int64_t nitems = k.n * nchunk;
    const int64_t i0 = (int64_t)lb * k.items_per_block;
    const int64_t i1 = i0 + k.items_per_block < nitems ? i0 + k.items_per_block : nitems;
    for (int64_t item = i0 + (threadIdx.x >> 6); item < i1; item += (blockDim.x >> 6)) {
        const int64_t iu = __builtin_amdgcn_readfirstlane((int)(item / nchunk));
        const int chunk = (int)(item - iu * nchunk);
        const int m = chunk * 64 + lane;
        const bool on = m < k.M;
        const int mm = on ? m : 0;
        T c[NS];
#pragma unroll
        for (int b = 0; b < NS; ++b) c[b] = k.coef[mm * NS + b];
        const int64_t p0 = row_off[iu], p1 = row_off[iu + 1];
        T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
        int64_t p = p0;
        for (; p + 7 < p1; p += 8) {
            int32_t jj[8];
            T xx[8], aa[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) jj[u] = col[p + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) xx[u] = xin<MODE>(k, jj[u], mm);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                T a = 0;
#pragma unroll
                for (int b = 0; b < NS; ++b) a += c[b] * vals[(p + u) * NS + b];
                aa[u] = a;
            }
            acc0 += aa[0] * xx[0] + aa[4] * xx[4];
            acc1 += aa[1] * xx[1] + aa[5] * xx[5];
            acc2 += aa[2] * xx[2] + aa[6] * xx[6];
            acc3 += aa[3] * xx[3] + aa[7] * xx[7];
        }
        for (; p + 3 < p1; p += 4) {
            const int32_t j0 = col[p], j1 = col[p + 1], j2 = col[p + 2], j3 = col[p + 3];
            const T x0 = xin<MODE>(k, j0, mm), x1 = xin<MODE>(k, j1, mm), x2 = xin<MODE>(k, j2, mm),
                    x3 = xin<MODE>(k, j3, mm);
            T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
            for (int b = 0; b < NS; ++b) {
                a0 += c[b] * vals[p * NS + b];
                a1 += c[b] * vals[(p + 1) * NS + b];
                a2 += c[b] * vals[(p + 2) * NS + b];
                a3 += c[b] * vals[(p + 3) * NS + b];
            }
            acc0 += a0 * x0;
            acc1 += a1 * x1;
            acc2 += a2 * x2;
            acc3 += a3 * x3;
        }
        for (; p < p1; ++p) {
            T a0 = 0;
#pragma unroll
            for (int b = 0; b < NS; ++b) a0 += c[b] * vals[p * NS + b];
            acc0 += a0 * xin<MODE>(k, col[p], mm);
        }
        T acc = (acc0 + acc1) + (acc2 + acc3);
        if (k.soff) acc += spmv_surface<MODE>(k, iu, mm);
        if (on) spmv_finish(k, iu, m, acc);
    }
}

// Row-group SpMV for small ordinate counts: thread (row group, m); lanes of
// one row share the row's stream values (broadcast loads).
template <int NS, class T, int MODE>
__global__ __launch_bounds__(512) void spmv_group_kernel(SpmvK<T> k)
{
    if (k.gate && *k.gate == 0) return;
    const int M = k.M;
    const int rpb = blockDim.x / M;
    const int rl = threadIdx.x / M;
    const int m = threadIdx.x - rl * M;
    if (rl >= rpb) return;
    T c[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) c[b] = k.coef[m * NS + b];
    for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < k.n; i += (int64_t)gridDim.x * rpb) {
        const int64_t p0 = k.row_off[i], p1 = k.row_off[i + 1];
        T acc0 = 0, acc1 = 0;
        int64_t p = p0;
        for (; p + 1 < p1; p += 2) {
            const int64_t j0 = k.col[p], j1 = k.col[p + 1];
            const T x0 = xin<MODE>(k, j0, m), x1 = xin<MODE>(k, j1, m);
            const T *v = k.vals + p * NS;
            T a0 = 0, a1 = 0;
#pragma unroll
            for (int b = 0; b < NS; ++b) {
                a0 += c[b] * v[b];
                a1 += c[b] * v[NS + b];
            }
            acc0 += a0 * x0;
            acc1 += a1 * x1;
        }
        for (; p < p1; ++p) {
            const T *v = k.vals + p * NS;
            T a = 0;
#pragma unroll
            for (int b = 0; b < NS; ++b) a += c[b] * v[b];
            acc0 += a * xin<MODE>(k, k.col[p], m);
        }
        T acc = acc0 + acc1;
        if (k.soff) acc += spmv_surface<MODE>(k, i, m);
        spmv_finish(k, i, m, acc);
    }
}

// Mixed-precision helpers for the refinement loop.
__global__ void to_float_scaled_kernel(int64_t n, int M, const double *r, const double *rn2, const double *fn2,
                                       double tol, float *out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * M) return;
    int m = (int)(t % M);
    double rn = sqrt(rn2[m]), fn = sqrt(fn2[m]);
    out[t] = (rn > tol * fn && rn > 0.0) ? (float)(r[t] / rn) : 0.0f;
}

__global__ void axpy_from_float_kernel(int64_t n, int M, double *x, const float *d, const double *rn2)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * M) return;
    int m = (int)(t % M);
    x[t] += sqrt(rn2[m]) * (double)d[t];
}

__global__ void cast_f32_kernel(const double *in, float *out, int64_t count)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = (float)in[t];
}

__global__ void point_values_kernel(int64_t n, const int64_t *row_off, const int32_t *col, const double *E,
                                    const double *coef, double *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t p = row_off[i]; p < row_off[i + 1]; ++p) s += E[p] * coef[col[p]];
    out[i] = s;
}

// Inflow term (N_i, |W.n| psi_b)_{W.n<0}: one thread per (boundary point, m).
__global__ void boundary_rhs_kernel(int64_t nbq, int M, int dim, int kmax, const int32_t *face, const double *bw,
                                    const int32_t *nact, const int32_t *act, const double *bN, const double *omega,
                                    const double *psib, double *F)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nbq * M) return;
    int64_t k = t / M;
    int m = (int)(t - k * M);
    int f = face[k];
    int ax = f >> 1;
    double sgn = (f & 1) ? 1.0 : -1.0;
    double wn = sgn * omega[m * dim + ax];
    if (wn >= 0.0) return;
    double val = psib[t];
    if (val == 0.0) return;
    double s = bw[k] * (-wn) * val;
    for (int a = 0; a < nact[k]; ++a) atomicAdd(&F[(int64_t)act[k * kmax + a] * M + m], s * bN[k * kmax + a]);
}

// out[i] = base[i] + sign * sum_m w_m X[i][m]; one wave per row.
__global__ __launch_bounds__(256) void ord_reduce_kernel(int64_t n, int M, const double *wq, const double *X,
                                                         const double *base, double sign, double *out)
{
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    if (i >= n) return;
    double s = 0.0;
    for (int m = lane; m < M; m += 64) s += wq[m] * X[i * M + m];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) out[i] = (base ? base[i] : 0.0) + sign * s;
}

__global__ void add_kernel(double *y, const double *a, const double *b, int64_t count)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) y[t] = a[t] + b[t];
}

inline int rows_per_block(int M) { return M >= 256 ? 1 : 256 / M; }

}  // namespace

hipError_t launch_assemble(Problem &P, const double *sig_t, const double *sig_s, const double *tau, hipStream_t s)
{
    AsmArgs a;
    a.n = P.n; a.nnz = P.nnz; a.dim = P.dim; a.G = P.n_mat; a.row_off = P.row_off.p; a.blocks = P.blocks.p;
    a.tau = tau; a.a0 = P.a0;
    for (int g = 0; g < 8; ++g) {
        a.sig_t[g] = g < P.n_mat ? sig_t[g] : 0.0;
        a.sig_s[g] = g < P.n_mat ? sig_s[g] : 0.0;
    }
    a.sL = P.sL.p; a.sMD = P.sMD.p; a.sMS = P.sMS.p; a.nsL = P.nsL;
    assemble_kernel<<<(unsigned)((P.nnz + 255) / 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_surface_count(Problem &P, int64_t *counts, hipStream_t s)
{
    int sb = P.n_mat * (1 + P.dim) + P.dim * P.dim;
    surface_count_kernel<<<(unsigned)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.nnz, 2 * P.dim, sb, P.row_off.p,
                                                                         P.blocks.p, counts);
    return hipGetLastError();
}

hipError_t launch_surface_fill(Problem &P, const double *, hipStream_t s)
{
    int sb = P.n_mat * (1 + P.dim) + P.dim * P.dim;
    surface_fill_kernel<<<(unsigned)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.nnz, 2 * P.dim, sb, P.row_off.p,
                                                                        P.col.p, P.blocks.p, P.surf_off.p,
                                                                        P.surf_col.p, P.surf_val.p);
    return hipGetLastError();
}

hipError_t launch_jacobi(Problem &P, hipStream_t s)
{
    int64_t tot = P.n * P.n_ord;
    jacobi_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(P.n, P.n_ord, P.nsL, P.nfaces, P.diag_pos.p, P.sL.p,
                                                                   P.coefL.p, P.surf_off.p, P.surf_col.p,
                                                                   P.surf_val.p, P.coefF.p, P.dinv.p);
    return hipGetLastError();
}

// ---- launch shapes of the sweep and their autotuning -------------------------
// Wave kernel (M >= 48): `wpb` waves per workgroup, each wave sweeping `ipw`
// (row, 64-ordinate chunk) items; with `xcd` = 8 workgroups are renumbered so
// that every die walks one contiguous range of rows.  Group kernel (M < 48):
// `threads` per workgroup (rows of M lanes).  The best shape per (rows,
// ordinates, streams, value size) is measured once per process on the
// problem's own operator and kept in a table (mlpg_get_tuning).
struct SpmvShape {
    int wpb = 4, ipw = 1, xcd = 8, threads = 256;
};

namespace {
struct TuneEntry {
    int64_t n;
    int M, ns, tbytes;
    SpmvShape shape;
    float us_best, us_default;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
bool g_autotune = true;

bool find_shape(int64_t n, int M, int ns, int tb, SpmvShape *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &e : g_tune)
        if (e.n == n && e.M == M && e.ns == ns && e.tbytes == tb) {
            *out = e.shape;
            return true;
        }
    return false;
}
}  // namespace

template <class T>
static hipError_t launch_spmv_shape(Problem &P, const SpmvArgsT<T> &a, const SpmvShape &sh, hipStream_t s)
{
    const int M = P.n_ord;
    SpmvK<T> k;
    k.items_per_block = 0;
    k.nxcd = sh.xcd;
    k.n = P.n; k.M = M; k.row_off = P.row_off.p; k.col = P.col.p; k.vals = a.vals; k.coef = a.coef; k.x = a.x;
    k.x_bcast = a.x_bcast; k.x2 = a.x2; k.xs = a.xs; k.dinv = a.dinv; k.colscale = a.colscale;
    k.soff = a.surface ? P.surf_off.p : nullptr; k.scol = P.surf_col.p; k.sval = a.sval; k.coefF = a.coefF;
    k.nf = P.nfaces; k.y = a.y; k.yadd = a.yadd; k.ysign = a.ysign; k.vout = a.vout; k.vsrc = a.vsrc;
    k.gate = a.gate;
    if (a.vout && !a.vsrc && (a.x_bcast || a.x2)) return hipErrorInvalidValue;
    if (a.surface && (!a.sval || !a.coefF)) return hipErrorInvalidValue;
    const bool wave = M >= 48;
    unsigned blocks;
    int threads;
    if (wave) {
        // sh.wpb waves per workgroup, sh.ipw items per wave, grid a multiple of the xcd count
        threads = 64 * sh.wpb;
        const int64_t items = P.n * ((M + 63) / 64);
        const int64_t per_block = (int64_t)sh.wpb * sh.ipw;
        int64_t b = (items + per_block - 1) / per_block;
        b = ((b + sh.xcd - 1) / sh.xcd) * sh.xcd;
        if (b < sh.xcd) b = sh.xcd;
        blocks = (unsigned)b;
        k.items_per_block = (items + b - 1) / b;
    } else {
        const int rpb = std::max(1, sh.threads / M);
        threads = rpb * M;
        int64_t b = (P.n + rpb - 1) / rpb;
        blocks = (unsigned)(b > 65536 ? 65536 : b);
    }
    int mode = IN_PLAIN;
    if (a.x_bcast) mode = IN_BCAST;
    if (a.x2) mode = IN_X2;
    if (a.dinv) mode = IN_DINV;
    if ((a.x_bcast != 0) + (a.x2 != nullptr) + (a.dinv != nullptr) > 1) return hipErrorInvalidValue;
#define MLPG_SPMV_M(NSV, MD)                                                      \
    if (wave) spmv_wave_kernel<NSV, T, MD><<<blocks, threads, 0, s>>>(k, k.row_off, k.col, k.vals); \
    else spmv_group_kernel<NSV, T, MD><<<blocks, threads, 0, s>>>(k)
#define MLPG_SPMV(NSV)                                                            \
    switch (mode) {                                                               \
    case IN_PLAIN: MLPG_SPMV_M(NSV, IN_PLAIN); break;                             \
    case IN_DINV: MLPG_SPMV_M(NSV, IN_DINV); break;                               \
    case IN_BCAST: MLPG_SPMV_M(NSV, IN_BCAST); break;                             \
    default: MLPG_SPMV_M(NSV, IN_X2); break;                                      \
    }
    switch (a.ns) {
    case 3: MLPG_SPMV(3); break;
    case 4: MLPG_SPMV(4); break;
    case 6: MLPG_SPMV(6); break;
    case 10: MLPG_SPMV(10); break;
    default: return hipErrorInvalidValue;
    }
#undef MLPG_SPMV
#undef MLPG_SPMV_M
    return hipGetLastError();
}

template <class T>
hipError_t launch_spmv(Problem &P, const SpmvArgsT<T> &a, hipStream_t s)
{
    SpmvShape sh;
    (void)find_shape(P.n, P.n_ord, a.ns, (int)sizeof(T), &sh);
    return launch_spmv_shape<T>(P, a, sh, s);
}

// Times every candidate shape of the transport sweep as the inner solver
// calls it (normalisation fused, per-ordinate column scale) on x -> y, both
// [n][M] scratch vectors of the caller, and records the fastest.  Runs once
// per (rows, ordinates, streams, value size) and process; never during a
// graph capture (the caller tunes before the first solve).
template <class T>
hipError_t tune_spmv(Problem &P, const SpmvArgsT<T> &a, hipStream_t s)
{
    SpmvShape cur;
    if (!g_autotune || find_shape(P.n, P.n_ord, a.ns, (int)sizeof(T), &cur)) return hipSuccess;
    std::vector<SpmvShape> cand;
    if (P.n_ord >= 48) {
        for (int wpb : {2, 4, 8})
            for (int ipw : {1, 2})
                for (int xcd : {8, 1}) {
                    SpmvShape c;
                    c.wpb = wpb; c.ipw = ipw; c.xcd = xcd;
                    cand.push_back(c);
                }
    } else {
        for (int th : {128, 256, 512}) {
            SpmvShape c;
            c.threads = th;
            cand.push_back(c);
        }
    }
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
    float best = 1e30f, dflt = 0.0f;
    SpmvShape pick;
    for (const SpmvShape &c : cand) {
        if ((e = launch_spmv_shape<T>(P, a, c, s)) != hipSuccess) break;   // warm-up
        float t = 1e30f;
        for (int r = 0; r < 2 && e == hipSuccess; ++r) {
            if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
            if ((e = launch_spmv_shape<T>(P, a, c, s)) != hipSuccess) break;
            if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            t = std::min(t, ms);
        }
        if (e != hipSuccess) break;
        const SpmvShape d;
        if (c.wpb == d.wpb && c.ipw == d.ipw && c.xcd == d.xcd && c.threads == d.threads) dflt = t;
        if (t < best) {
            best = t;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.push_back({P.n, P.n_ord, a.ns, (int)sizeof(T), pick, 1e3f * best, 1e3f * dflt});
    return hipSuccess;
}
template hipError_t tune_spmv<double>(Problem &, const SpmvArgsT<double> &, hipStream_t);
template hipError_t tune_spmv<float>(Problem &, const SpmvArgsT<float> &, hipStream_t);

void set_autotune(int mode)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (mode == 2) g_tune.clear();
    else g_autotune = mode != 0;
}

int get_tuning(int cap, mlpg_tune_entry *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int cnt = (int)g_tune.size();
    for (int i = 0; i < cnt && i < cap; ++i) {
        const TuneEntry &e = g_tune[i];
        out[i].n = e.n;
        out[i].n_ord = e.M;
        out[i].streams = e.ns;
        out[i].value_bytes = e.tbytes;
        out[i].waves_per_block = e.M >= 48 ? e.shape.wpb : 0;
        out[i].items_per_wave = e.M >= 48 ? e.shape.ipw : 0;
        out[i].xcd_split = e.M >= 48 ? e.shape.xcd : 0;
        out[i].threads = e.M >= 48 ? 64 * e.shape.wpb : e.shape.threads;
        out[i].us_best = e.us_best;
        out[i].us_default = e.us_default;
    }
    return cnt;
}

template hipError_t launch_spmv<double>(Problem &, const SpmvArgsT<double> &, hipStream_t);
template hipError_t launch_spmv<float>(Problem &, const SpmvArgsT<float> &, hipStream_t);

hipError_t launch_to_float_scaled(int64_t n, int M, const double *r, const double *rn2, const double *fn2, double tol,
                                  float *out, hipStream_t s)
{
    int64_t tot = n * M;
    to_float_scaled_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(n, M, r, rn2, fn2, tol, out);
    return hipGetLastError();
}

hipError_t launch_axpy_from_float(int64_t n, int M, double *x, const float *d, const double *rn2, hipStream_t s)
{
    int64_t tot = n * M;
    axpy_from_float_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(n, M, x, d, rn2);
    return hipGetLastError();
}

hipError_t launch_cast_f32(const double *in, float *out, int64_t count, hipStream_t s)
{
    cast_f32_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(in, out, count);
    return hipGetLastError();
}

hipError_t launch_point_values(Problem &P, const double *coef, double *out, hipStream_t s)
{
    point_values_kernel<<<(unsigned)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.row_off.p, P.col.p, P.E.p, coef, out);
    return hipGetLastError();
}

hipError_t launch_boundary_rhs(Problem &P, const double *psib, double *F, hipStream_t s)
{
    int64_t tot = P.n_bq * P.n_ord;
    if (tot == 0) return hipSuccess;
    boundary_rhs_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(P.n_bq, P.n_ord, P.dim, P.bq_kmax, P.bq_face.p,
                                                                        P.bq_w.p,
                                                                        P.bq_nact.p, P.bq_act.p, P.bq_N.p,
                                                                        P.omega.p, psib, F);
    return hipGetLastError();
}

hipError_t launch_ord_reduce(Problem &P, const double *X, double *out, const double *base, double sign, hipStream_t s)
{
    int64_t blocks = (P.n + 3) / 4;
    ord_reduce_kernel<<<(unsigned)blocks, 256, 0, s>>>(P.n, P.n_ord, P.wq.p, X, base, sign, out);
    return hipGetLastError();
}

hipError_t launch_add(double *y, const double *a, const double *b, int64_t count, hipStream_t s)
{
    add_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(y, a, b, count);
    return hipGetLastError();
}

}  // namespace mlpg
