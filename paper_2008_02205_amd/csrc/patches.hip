// Spatial patches of points and the patch block-Jacobi preconditioner of the
// inner transport solves (Sec. 4.2 preconditions every L_m; the paper factors
// each with ILUT, which is sequential; a block-diagonal inverse over small
// spatial patches is the data-parallel form used here).
//
// Patches: the domain box is cut into a uniform grid of cells of side
// 2 (|domain| / n)^(1/d) (twice the mean point spacing, so that a lattice
// patch holds 2^d points); the points of one cell, in increasing index,
// form one patch, split into consecutive chunks of at most kPatchMax.
// Patches are ordered by cell (row-major over the grid axes, the last axis
// fastest).
//
// Preconditioner: for every patch P and ordinate m the dense block
// B = L_m[P, P] (the same entries the operator applies, surface terms
// included) is inverted by Gauss-Jordan elimination with partial pivoting;
// z = M^-1 v applies these inverses patch by patch.  Stored as
// binv[boff[p] * M + (i s + j) M + m] for patch p of size s, so that the
// lanes of a wave (consecutive ordinates) read consecutive values.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace mlpg {

namespace {

struct Grid {
    double lo[3], inv_h;
    int64_t dims[3];
    int dim;
};

__device__ __forceinline__ int64_t cell_of(const Grid &g, const double *x)
{
    int64_t id = 0;
    for (int a = 0; a < g.dim; ++a) {
        const double t = (x[a] - g.lo[a]) * g.inv_h;
        int64_t b = 0;   // below the box or NaN
        if (t >= 0.0 && t < (double)g.dims[a]) b = (int64_t)t;
        else if (t >= (double)g.dims[a]) b = g.dims[a] - 1;
        id = id * g.dims[a] + b;
    }
    return id;
}

__global__ void bin_count_kernel(int64_t n, Grid g, const double *__restrict__ x, int64_t *__restrict__ key,
                                 unsigned long long *__restrict__ cnt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = cell_of(g, x + i * g.dim);
    key[i] = c;
    atomicAdd(&cnt[c], 1ull);
}

__global__ void bin_fill_kernel(int64_t n, const int64_t *__restrict__ key, const int64_t *__restrict__ off,
                                unsigned long long *__restrict__ cursor, int32_t *__restrict__ pts)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = key[i];
    const unsigned long long k = atomicAdd(&cursor[c], 1ull);
    pts[off[c] + (int64_t)k] = (int32_t)i;
}

// The fill above places a cell's points in arbitrary order: sort each cell
// (insertion sort; cells hold a handful of points).  Also the number of
// patches of the cell.
__global__ void bin_sort_kernel(int64_t ncell, const int64_t *__restrict__ off, int32_t *__restrict__ pts,
                                int64_t *__restrict__ npatch_of)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int64_t a = off[c], b = off[c + 1];
    for (int64_t p = a + 1; p < b; ++p) {
        const int32_t v = pts[p];
        int64_t q = p - 1;
        while (q >= a && pts[q] > v) {
            pts[q + 1] = pts[q];
            --q;
        }
        pts[q + 1] = v;
    }
    npatch_of[c] = (b - a + kPatchMax - 1) / kPatchMax;
}

// Patch starts (into the sorted point list) and the squared sizes.
__global__ void patch_fill_kernel(int64_t ncell, const int64_t *__restrict__ off, const int64_t *__restrict__ pbase,
                                  int64_t *__restrict__ poff, int64_t *__restrict__ s2, int64_t npatch, int64_t n)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0) poff[npatch] = n;
    if (c >= ncell) return;
    const int64_t a = off[c], b = off[c + 1];
    int64_t p = pbase[c];
    for (int64_t st = a; st < b; st += kPatchMax, ++p) {
        const int64_t s = (b - st) < kPatchMax ? (b - st) : kPatchMax;
        poff[p] = st;
        s2[p] = s * s;
    }
}

// Entry L_m[row, j] from the value streams and the surface rows; 0 when j is
// not in the row's pattern.
template <class T>
__device__ __forceinline__ double L_entry(const int64_t *row_off, const int32_t *col, const T *sL, int nsL,
                                          const T *cL, const int64_t *soff, const int32_t *scol, const T *sval,
                                          int nf, const T *cF, int64_t row, int32_t j)
{
    int64_t lo = row_off[row], hi = row_off[row + 1] - 1;
    double v = 0.0;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t cm = col[mid];
        if (cm == j) {
            for (int b = 0; b < nsL; ++b) v += (double)cL[b] * (double)sL[mid * nsL + b];
            break;
        }
        if (cm < j) lo = mid + 1;
        else hi = mid - 1;
    }
    for (int64_t q = soff[row]; q < soff[row + 1]; ++q)
        if (scol[q] == j)
            for (int f = 0; f < nf; ++f) v += (double)cF[f] * (double)sval[q * nf + f];
    return v;
}

// One thread per (patch, ordinate): B = L_m[P, P] into `work`, its inverse
// into `binv` by Gauss-Jordan elimination of [B | I] with partial pivoting.
// A block with a zero pivot falls back to the inverse of its diagonal
// (counted in *singular).
__global__ __launch_bounds__(256) void patch_build_kernel(int64_t npatch, int M, const int64_t *__restrict__ poff,
                                                          const int32_t *__restrict__ pidx,
                                                          const int64_t *__restrict__ boff,
                                                          const int64_t *__restrict__ row_off,
                                                          const int32_t *__restrict__ col, int nsL,
                                                          const double *__restrict__ sL,
                                                          const double *__restrict__ coefL,
                                                          const int64_t *__restrict__ soff,
                                                          const int32_t *__restrict__ scol,
                                                          const double *__restrict__ sval, int nf,
                                                          const double *__restrict__ coefF, double *__restrict__ work,
                                                          double *__restrict__ binv,
                                                          unsigned long long *__restrict__ singular)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npatch * M) return;
    const int64_t p = t / M;
    const int m = (int)(t - p * M);
    const int s = (int)(poff[p + 1] - poff[p]);
    const int32_t *pts = pidx + poff[p];
    double *A = work + boff[p] * M + m;
    double *X = binv + boff[p] * M + m;
#define AT(i, j) A[(int64_t)((i) * s + (j)) * M]
#define XT(i, j) X[(int64_t)((i) * s + (j)) * M]
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
            AT(i, j) = L_entry<double>(row_off, col, sL, nsL, coefL + (int64_t)m * nsL, soff, scol, sval, nf,
                                       coefF + (int64_t)m * nf, pts[i], pts[j]);
            XT(i, j) = i == j ? 1.0 : 0.0;
        }
    bool ok = true;
    for (int k = 0; k < s && ok; ++k) {
        int piv = k;
        double best = fabs(AT(k, k));
        for (int i = k + 1; i < s; ++i) {
            const double v = fabs(AT(i, k));
            if (v > best) {
                best = v;
                piv = i;
            }
        }
        if (!(best > 0.0) || !isfinite(best)) {
            ok = false;
            break;
        }
        if (piv != k)
            for (int j = 0; j < s; ++j) {
                double a = AT(k, j);
                AT(k, j) = AT(piv, j);
                AT(piv, j) = a;
                double x = XT(k, j);
                XT(k, j) = XT(piv, j);
                XT(piv, j) = x;
            }
        const double d = 1.0 / AT(k, k);
        for (int j = 0; j < s; ++j) {
            AT(k, j) *= d;
            XT(k, j) *= d;
        }
        for (int i = 0; i < s; ++i) {
            if (i == k) continue;
            const double f = AT(i, k);
            if (f == 0.0) continue;
            for (int j = 0; j < s; ++j) {
                AT(i, j) -= f * AT(k, j);
                XT(i, j) -= f * XT(k, j);
            }
        }
    }
    if (!ok) {
        atomicAdd(singular, 1ull);
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                double dg = i == j ? L_entry<double>(row_off, col, sL, nsL, coefL + (int64_t)m * nsL, soff, scol, sval,
                                                     nf, coefF + (int64_t)m * nf, pts[i], pts[i])
                                   : 0.0;
                XT(i, j) = i == j ? (dg != 0.0 ? 1.0 / dg : 1.0) : 0.0;
            }
    }
#undef AT
#undef XT
}

// out = M^-1 in (ADD: out += M^-1 in), one wave per (patch, 64-ordinate
// chunk), lane = ordinate.  The patch's inputs are loaded once into
// registers; every row of the block is then a dot product over them.
template <class T, bool ADD>
__global__ __launch_bounds__(256) void patch_apply_kernel(int64_t npatch, int M, const int64_t *__restrict__ poff,
                                                          const int32_t *__restrict__ pidx,
                                                          const int64_t *__restrict__ boff,
                                                          const T *__restrict__ binv, const T *__restrict__ in,
                                                          T *__restrict__ out, const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    const int nchunk = (M + 63) >> 6;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t p = wv / nchunk;
    if (p >= npatch) return;
    const int m = (int)(wv - p * nchunk) * 64 + lane;
    if (m >= M) return;
    const int64_t a = poff[p];
    const int s = (int)(poff[p + 1] - a);
    const T *B = binv + boff[p] * M + m;
    int32_t pt[kPatchMax];
    T v[kPatchMax];
#pragma unroll
    for (int j = 0; j < kPatchMax; ++j) {
        pt[j] = j < s ? pidx[a + j] : 0;
        v[j] = j < s ? in[(int64_t)pt[j] * M + m] : (T)0;
    }
#pragma unroll
    for (int i = 0; i < kPatchMax; ++i) {
        if (i < s) {
            T acc = 0;
#pragma unroll
            for (int j = 0; j < kPatchMax; ++j)
                if (j < s) acc += B[(int64_t)(i * s + j) * M] * v[j];
            const int64_t o = (int64_t)pt[i] * M + m;
            out[o] = ADD ? out[o] + acc : acc;
        }
    }
}

__global__ void cast_f32_patch_kernel(const double *in, float *out, int64_t count)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = (float)in[t];
}

inline unsigned blocks_of(int64_t count, int threads) { return (unsigned)((count + threads - 1) / threads); }

}  // namespace

int64_t patch_grid_cells(int dim, int64_t n, const double *lo, const double *hi, double *h_out, int64_t dims[3])
{
    double vol = 1.0;
    for (int a = 0; a < dim; ++a) vol *= hi[a] - lo[a];
    double h = 2.0 * std::pow(vol / (double)(n > 0 ? n : 1), 1.0 / dim);
    int64_t ncell = 1;
    for (;;) {
        ncell = 1;
        for (int a = 0; a < dim; ++a) {
            dims[a] = std::max<int64_t>(1, (int64_t)std::ceil((hi[a] - lo[a]) / h));
            ncell *= dims[a];
        }
        if (ncell <= ((int64_t)1 << 26)) break;
        h *= 2.0;
    }
    for (int a = dim; a < 3; ++a) dims[a] = 1;
    if (h_out) *h_out = h;
    return ncell;
}

// Patches of the current points into P.poff, P.pidx, P.boff (carved by the
// geometry layout with n-sized bounds; temporaries from the same workspace).
int build_patches(Problem &P, hipStream_t s)
{
    const int d = P.dim;
    const int64_t n = P.n;
    Grid g;
    g.dim = d;
    double h = 1.0;
    const int64_t ncell = patch_grid_cells(d, n, P.dom_lo, P.dom_hi, &h, g.dims);
    if (ncell != P.ncell) {
        set_error("patch grid does not match the geometry workspace");
        return MLPG_ERR_WORKSPACE;
    }
    for (int a = 0; a < 3; ++a) g.lo[a] = a < d ? P.dom_lo[a] : 0.0;
    g.inv_h = 1.0 / h;
    MLPG_HIP(hipMemsetAsync(P.tmp_cnt.p, 0, sizeof(unsigned long long) * ncell, s));
    bin_count_kernel<<<blocks_of(n, 256), 256, 0, s>>>(n, g, P.x.p, P.tmp_key.p, P.tmp_cnt.p);
    MLPG_HIP(launch_exclusive_scan((const int64_t *)P.tmp_cnt.p, P.tmp_off.p, ncell, s));
    MLPG_HIP(hipMemsetAsync(P.tmp_cnt.p, 0, sizeof(unsigned long long) * ncell, s));
    bin_fill_kernel<<<blocks_of(n, 256), 256, 0, s>>>(n, P.tmp_key.p, P.tmp_off.p, P.tmp_cnt.p, P.pidx.p);
    bin_sort_kernel<<<blocks_of(ncell, 256), 256, 0, s>>>(ncell, P.tmp_off.p, P.pidx.p, P.tmp_npc.p);
    MLPG_HIP(launch_exclusive_scan(P.tmp_npc.p, P.tmp_pbase.p, ncell, s));
    int64_t npatch = 0;
    MLPG_HIP(hipMemcpyAsync(&npatch, P.tmp_pbase.p + ncell, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipStreamSynchronize(s));
    if (npatch < 1 || npatch > n) {
        set_error("patch construction: patch count out of range");
        return MLPG_ERR_GEOMETRY;
    }
    patch_fill_kernel<<<blocks_of(ncell, 256), 256, 0, s>>>(ncell, P.tmp_off.p, P.tmp_pbase.p, P.poff.p, P.tmp_s2.p,
                                                              npatch, n);
    MLPG_HIP(launch_exclusive_scan(P.tmp_s2.p, P.boff.p, npatch, s));
    MLPG_HIP(hipMemcpyAsync(&P.nbsq, P.boff.p + npatch, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipStreamSynchronize(s));
    MLPG_HIP(hipGetLastError());
    P.npatch = npatch;
    return MLPG_OK;
}

// Block inverses of the assembled operators into P.binv (and P.binv32 in the
// mixed path), carved by the solve layout for the current patches.
int build_patch_inverses(Problem &P, hipStream_t s)
{
    const int M = P.n_ord;
    const int64_t cnt = P.nbsq * M;
    if (!P.binv.p || P.binv.count < (size_t)cnt || P.tmp_work.count < (size_t)cnt) {
        set_error("patch preconditioner: the solve workspace was laid out without it");
        return MLPG_ERR_WORKSPACE;
    }
    MLPG_HIP(hipMemsetAsync(P.tmp_sing.p, 0, sizeof(unsigned long long), s));
    patch_build_kernel<<<blocks_of(P.npatch * M, 256), 256, 0, s>>>(
        P.npatch, M, P.poff.p, P.pidx.p, P.boff.p, P.row_off.p, P.col.p, P.nsL, P.sL.p, P.coefL.p, P.surf_off.p,
        P.surf_col.p, P.surf_val.p, P.nfaces, P.coefF.p, P.tmp_work.p, P.binv.p, P.tmp_sing.p);
    MLPG_HIP(hipGetLastError());
    if (P.precision == MLPG_MIXED) {
        cast_f32_patch_kernel<<<blocks_of(cnt, 256), 256, 0, s>>>(P.binv.p, P.binv32.p, cnt);
        MLPG_HIP(hipGetLastError());
    }
    unsigned long long ns = 0;
    MLPG_HIP(hipMemcpyAsync(&ns, P.tmp_sing.p, sizeof(ns), hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipStreamSynchronize(s));
    P.patch_singular = (int64_t)ns;
    return MLPG_OK;
}

template <class T>
hipError_t launch_patch_apply(const PatchPrecT<T> &pp, int M, const T *in, T *out, bool add, const int *gate,
                              hipStream_t s)
{
    const int64_t waves = pp.npatch * ((M + 63) / 64);
    const unsigned blocks = blocks_of(waves * 64, 256);
    if (add)
        patch_apply_kernel<T, true><<<blocks, 256, 0, s>>>(pp.npatch, M, pp.poff, pp.pidx, pp.boff, pp.binv, in, out,
                                                           gate);
    else
        patch_apply_kernel<T, false><<<blocks, 256, 0, s>>>(pp.npatch, M, pp.poff, pp.pidx, pp.boff, pp.binv, in, out,
                                                            gate);
    return hipGetLastError();
}
template hipError_t launch_patch_apply<double>(const PatchPrecT<double> &, int, const double *, double *, bool,
                                               const int *, hipStream_t);
template hipError_t launch_patch_apply<float>(const PatchPrecT<float> &, int, const float *, float *, bool,
                                              const int *, hipStream_t);

}  // namespace mlpg
