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
#include <atomic>
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

// Surface rows: a row with any nonzero face block keeps the face values of
// every one of its nonzeros (zeros included), so that its surface entry
// s0 + (p - p0) belongs to nonzero p and the sweep can add the faces' sums
// in the row's main loop; other rows keep none.
__global__ void surface_count_kernel(int64_t n, int64_t nnz, int nf, int sb, const int64_t *row_off,
                                     const double *blocks, int64_t *counts)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool nz = false;
    for (int64_t p = row_off[i]; p < row_off[i + 1] && !nz; ++p)
        for (int f = 0; f < nf; ++f) nz |= blocks[(int64_t)(sb + f) * nnz + p] != 0.0;
    counts[i] = nz ? row_off[i + 1] - row_off[i] : 0;
}

__global__ void surface_fill_kernel(int64_t n, int64_t nnz, int nf, int sb, const int64_t *row_off,
                                    const int32_t *col, const double *blocks, const int64_t *soff, int32_t *scol,
                                    double *sval)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || soff[i + 1] == soff[i]) return;
    int64_t o = soff[i];
    for (int64_t p = row_off[i]; p < row_off[i + 1]; ++p, ++o) {
        scol[o] = col[p];
        for (int f = 0; f < nf; ++f) sval[o * nf + f] = blocks[(int64_t)(sb + f) * nnz + p];
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

// The same without the factor xs, where xs can be applied once to the row's
// sum instead (every mode but IN_X2); xs_out() is that factor.
template <int MODE, class T>
__device__ __forceinline__ T xraw(const SpmvK<T> &k, int64_t j, int m)
{
    if (MODE == IN_X2) return xin<MODE>(k, j, m);
    if (MODE == IN_BCAST) return k.x[j];
    const int64_t o = j * k.M + m;
    if (MODE == IN_DINV) return k.x[o] * k.dinv[o];
    return k.x[o];
}

template <int MODE, class T>
__device__ __forceinline__ T xs_out(const SpmvK<T> &k)
{
    return MODE == IN_X2 ? (T)1 : k.xs;
}

// Operands of one output entry o = (i, m) besides the row's nonzeros:
// the per-ordinate column scale, the input entry that becomes the scaled
// basis vector, the addend, and the row's range of surface entries.  Loaded
// before the row's nonzeros so that their latency hides under that loop.
template <class T>
struct RowEnds {
    T sc, vin, yad;
    int64_t s0, s1;
};

template <class T>
__device__ __forceinline__ RowEnds<T> row_ends(const SpmvK<T> &k, int64_t i, int m)
{
    const int64_t o = i * k.M + m;
    RowEnds<T> r;
    r.sc = k.colscale ? (T)k.colscale[m] : (T)1;
    r.vin = k.vout ? (k.vsrc ? k.vsrc[o] : k.x[o]) : (T)0;
    r.yad = k.yadd ? k.yadd[o] : (T)0;
    r.s0 = k.soff ? k.soff[i] : 0;
    r.s1 = k.soff ? k.soff[i + 1] : 0;
    return r;
}

template <class T>
__device__ __forceinline__ void spmv_finish(const SpmvK<T> &k, int64_t i, int m, T acc, const RowEnds<T> &r)
{
    const int64_t o = i * k.M + m;
    if (k.vout) k.vout[o] = r.sc * r.vin;
    acc *= r.sc;
    k.y[o] = k.yadd ? r.yad + (T)k.ysign * acc : acc;
}

// Surface entries [s0, s1) of a row (rows within a support radius of the
// boundary have some tens): the outflow blocks weighted by max(0, W.n_f), at
// most six faces.  Columns are read eight at a time and their x gathers
// issued together, as in the row's main loop; the sum runs over p in order.
template <int MODE, class T>
__device__ __forceinline__ T spmv_surface(const SpmvK<T> &k, int64_t s0, int64_t s1, int m)
{
    const int nf = k.nf;
    T cf[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) cf[f] = f < nf ? k.coefF[m * nf + f] : (T)0;
    T acc = 0;
    int64_t p = s0;
    for (; p + 7 < s1; p += 8) {
        int32_t jj[8];
        T xx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) jj[u] = k.scol[p + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) xx[u] = xin<MODE>(k, jj[u], m);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            T a = 0;
#pragma unroll
            for (int f = 0; f < 6; ++f)
                if (f < nf) a += cf[f] * k.sval[(p + u) * nf + f];
            acc += a * xx[u];
        }
    }
    for (; p < s1; ++p) {
        T a = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f)
            if (f < nf) a += cf[f] * k.sval[p * nf + f];
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

// One batch of B nonzeros at p (when the row has that many left), gathers
// issued together; the sums stay in nonzero order.  A row's last 0-7
// nonzeros go in batches of 4, 2 and 1 (at most three dependent round trips
// instead of seven; about 1 us of 49 at 128^2 x 64).
template <int NS, class T, int MODE, int B, class CI, class VI>
__device__ __forceinline__ void row_streams_batch(const SpmvK<T> &k, CI cl, VI vl, int64_t &p, int64_t p1, int mm,
                                                  T (&t)[NS])
{
    if (p + B - 1 >= p1) return;
    int32_t jj[B];
    T xx[B];
#pragma unroll
    for (int u = 0; u < B; ++u) jj[u] = cl[p + u];
#pragma unroll
    for (int u = 0; u < B; ++u) xx[u] = xraw<MODE>(k, jj[u], mm);
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
        for (int b = 0; b < NS; ++b) t[b] += vl[(p + u) * NS + b] * xx[u];
    p += B;
}

// The per-stream row sums t_b of one row from nonzeros [p, p1) whose column
// indices and stream values are read through `cl` and `vl` (global memory or
// the LDS stage): eight x gathers issued back to back, then the FMAs.  The
// next batch's column indices are loaded with this batch's stream values,
// while its gathers are in flight, so that a batch's gathers need not wait
// for their indices (about 1 us of 49 at 128^2 x 64).
template <int NS, class T, int MODE, class CI, class VI>
__device__ __forceinline__ void row_streams(const SpmvK<T> &k, CI cl, VI vl, int64_t p, int64_t p1, int mm, T (&t)[NS])
{
    int32_t jj[8];
    if (p + 7 < p1) {
#pragma unroll
        for (int u = 0; u < 8; ++u) jj[u] = cl[p + u];
    }
    for (; p + 7 < p1; p += 8) {
        T xx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xx[u] = xraw<MODE>(k, jj[u], mm);
        int32_t jn[8];
        const int64_t pn = p + 15 < p1 ? p + 8 : p;   // the last batch rereads its own indices
#pragma unroll
        for (int u = 0; u < 8; ++u) jn[u] = cl[pn + u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int b = 0; b < NS; ++b) t[b] += vl[(p + u) * NS + b] * xx[u];
#pragma unroll
        for (int u = 0; u < 8; ++u) jj[u] = jn[u];
    }
    row_streams_batch<NS, T, MODE, 4>(k, cl, vl, p, p1, mm, t);
    row_streams_batch<NS, T, MODE, 2>(k, cl, vl, p, p1, mm, t);
    row_streams_batch<NS, T, MODE, 1>(k, cl, vl, p, p1, mm, t);
}

// Face count of the transport operators' surface term: 4 in 2D (6 value
// streams), 6 in 3D (10 streams).
template <int NS>
struct FacesOf {
    static constexpr int value = NS == 10 ? 6 : 4;
};

// row_streams on a surface row, whose face values are stored aligned with
// its nonzeros (surface entry p + fofs belongs to nonzero p): the per-face
// sums u_f = sum_p s_f[p] x[col p] are accumulated from the same x gathers.
template <int NS, int NF, class T, int MODE, class CI, class VI>
__device__ __forceinline__ void row_streams_faces(const SpmvK<T> &k, CI cl, VI vl, const T *__restrict__ fv,
                                                  int64_t p, int64_t p1, int64_t fofs, int mm, T (&t)[NS],
                                                  T (&uf)[NF])
{
    for (; p + 7 < p1; p += 8) {
        int32_t jj[8];
        T xx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) jj[u] = cl[p + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) xx[u] = xraw<MODE>(k, jj[u], mm);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int b = 0; b < NS; ++b) t[b] += vl[(p + u) * NS + b] * xx[u];
#pragma unroll
            for (int f = 0; f < NF; ++f) uf[f] += fv[(p + u + fofs) * NF + f] * xx[u];
        }
    }
    for (; p < p1; ++p) {
        const T xv = xraw<MODE>(k, cl[p], mm);
#pragma unroll
        for (int b = 0; b < NS; ++b) t[b] += vl[p * NS + b] * xv;
#pragma unroll
        for (int f = 0; f < NF; ++f) uf[f] += fv[(p + fofs) * NF + f] * xv;
    }
}

// One row's sum over nonzeros [p0, p1) (indices into cl/vl; the row's
// surface entries start at re.s0) for the lane's ordinate, before the column
// scale: sum_b c_b t_b, plus sum_f max(0, W.n_f) u_f on a surface row, times
// xs.  The same operations in the same order for every launch form.  `fv`
// is the face values' array (k.sval), passed as a read-only kernel argument
// so that its wave-uniform reads become scalar loads.
template <int NS, class T, int MODE, class CI, class VI, class CO>
__device__ __forceinline__ T row_sum(const SpmvK<T> &k, CI cl, VI vl, const T *__restrict__ fv, int64_t p0, int64_t p1,
                                     const RowEnds<T> &re, CO coef, int mm)
{
    constexpr int NF = FacesOf<NS>::value;
    T t[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) t[b] = 0;
    const bool faces = re.s1 > re.s0 && re.s1 - re.s0 == p1 - p0 && k.nf == NF;   // uniform over the wave
    T acc = 0;
    if (faces) {
        T uf[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) uf[f] = 0;
        row_streams_faces<NS, NF, T, MODE>(k, cl, vl, fv, p0, p1, re.s0 - p0, mm, t, uf);
#pragma unroll
        for (int b = 0; b < NS; ++b) acc += coef(b) * t[b];
#pragma unroll
        for (int f = 0; f < NF; ++f) acc += k.coefF[mm * NF + f] * uf[f];
        acc *= xs_out<MODE>(k);
    } else {
        row_streams<NS, T, MODE>(k, cl, vl, p0, p1, mm, t);
#pragma unroll
        for (int b = 0; b < NS; ++b) acc += coef(b) * t[b];
        acc *= xs_out<MODE>(k);
        if (re.s1 > re.s0) acc += spmv_surface<MODE>(k, re.s0, re.s1, mm);
    }
    return acc;
}

// Wave-per-row SpMV (used when the ordinates fill whole waves): each wave
// owns one (row, 64-ordinate chunk).  The row index is wave-uniform, so the
// row's column indices and stream values are read with scalar loads straight
// into SGPRs (read-only kernel arguments, no vector broadcast needed).  The
// row is accumulated per stream, t_b = sum_p v_b[p] x[col p], and combined
// with the lane's coefficients once at the end: NS FMAs per nonzero and
// ordinate, with the x gathers of eight nonzeros issued back to back so that
// their latencies overlap.  A surface row accumulates its faces' sums in the
// same loop (row_sum).
template <int NS, class T, int MODE>
__global__ __launch_bounds__(512) void spmv_wave_kernel(SpmvK<T> k, const int64_t *__restrict__ row_off,
                                                        const int32_t *__restrict__ col,
                                                        const T *__restrict__ vals, const T *__restrict__ fv)
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
        const int64_t iu =
            __builtin_amdgcn_readfirstlane((int)(nchunk == 1 ? item : item / nchunk));
        const int chunk = (int)(item - iu * nchunk);
        const int m = chunk * 64 + lane;
        const bool on = m < k.M;
        const int mm = on ? m : 0;
        const RowEnds<T> re = row_ends(k, iu, mm);
        const int64_t p0 = row_off[iu], p1 = row_off[iu + 1];
        // the coefficients (a few KB, cache resident) are read after the sums,
        // so that they hold no registers during the row's loop
        const T acc = row_sum<NS, T, MODE>(k, col, vals, fv, p0, p1, re, [&](int b) { return k.coef[mm * NS + b]; }, mm);
        if (on) spmv_finish(k, iu, m, acc, re);
    }
}

// V adjacent ordinates of one lane, loaded as one aligned vector.
template <class T, int V>
struct alignas(sizeof(T) * V) Pack {
    T v[V];
};

// xraw for the V ordinates m0 .. m0 + V - 1 of column j (one vector load per
// input array; m0 and M multiples of V, the arrays aligned to V elements).
template <int MODE, class T, int V>
__device__ __forceinline__ void xraw_vec(const SpmvK<T> &k, int64_t j, int m0, T (&out)[V])
{
    if (MODE == IN_BCAST) {
        const T b = k.x[j];
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = b;
        return;
    }
    const int64_t o = j * k.M + m0;
    const Pack<T, V> a = *(const Pack<T, V> *)(k.x + o);
    if (MODE == IN_X2) {
        const Pack<T, V> b = *(const Pack<T, V> *)(k.x2 + o);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T xv = k.xs * a.v[v];
            xv += b.v[v];
            out[v] = xv;
        }
    } else if (MODE == IN_DINV) {
        const Pack<T, V> d = *(const Pack<T, V> *)(k.dinv + o);
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = a.v[v] * d.v[v];
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = a.v[v];
    }
}

// row_sum for V ordinates of one lane: the same per-stream (and per-face)
// sums over the row's nonzeros in the same order, combined with each
// ordinate's coefficients in the same order, so every ordinate's result is
// the one row_sum gives.  One x gather of V values per nonzero, and the
// row's stream values and columns read once for V ordinates.  The gathers
// of VB nonzeros are issued together (VecBatch: 4 where the accumulators of
// 10 FP64 streams for 2 ordinates would otherwise cost a wave per SIMD).
template <int NS, class T, int V>
struct VecBatch {
    static constexpr int value = (NS == 10 && V == 2 && sizeof(T) == 8) ? 4 : 8;
};

template <int NS, class T, int MODE, int V>
__device__ __forceinline__ void row_sum_vec(const SpmvK<T> &k, const int32_t *__restrict__ cl,
                                            const T *__restrict__ vl, const T *__restrict__ fv, int64_t p0,
                                            int64_t p1, int64_t s0, int64_t s1, int m0, T (&acc)[V])
{
    constexpr int NF = FacesOf<NS>::value;
    constexpr int VB = VecBatch<NS, T, V>::value;
    T t[V][NS];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int b = 0; b < NS; ++b) t[v][b] = 0;
    const bool faces = s1 > s0 && s1 - s0 == p1 - p0 && k.nf == NF;   // uniform over the wave
    if (faces) {
        T uf[V][NF];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int f = 0; f < NF; ++f) uf[v][f] = 0;
        const int64_t fofs = s0 - p0;
        int64_t p = p0;
        for (; p + VB - 1 < p1; p += VB) {
            int32_t jj[VB];
            T xx[VB][V];
#pragma unroll
            for (int u = 0; u < VB; ++u) jj[u] = cl[p + u];
#pragma unroll
            for (int u = 0; u < VB; ++u) xraw_vec<MODE, T, V>(k, jj[u], m0, xx[u]);
#pragma unroll
            for (int u = 0; u < VB; ++u) {
#pragma unroll
                for (int b = 0; b < NS; ++b)
#pragma unroll
                    for (int v = 0; v < V; ++v) t[v][b] += vl[(p + u) * NS + b] * xx[u][v];
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int v = 0; v < V; ++v) uf[v][f] += fv[(p + u + fofs) * NF + f] * xx[u][v];
            }
        }
        for (; p < p1; ++p) {
            T xv[V];
            xraw_vec<MODE, T, V>(k, cl[p], m0, xv);
#pragma unroll
            for (int b = 0; b < NS; ++b)
#pragma unroll
                for (int v = 0; v < V; ++v) t[v][b] += vl[p * NS + b] * xv[v];
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int v = 0; v < V; ++v) uf[v][f] += fv[(p + fofs) * NF + f] * xv[v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T a = 0;
#pragma unroll
            for (int b = 0; b < NS; ++b) a += k.coef[(m0 + v) * NS + b] * t[v][b];
#pragma unroll
            for (int f = 0; f < NF; ++f) a += k.coefF[(m0 + v) * NF + f] * uf[v][f];
            a *= xs_out<MODE>(k);
            acc[v] = a;
        }
    } else {
        int64_t p = p0;
        for (; p + VB - 1 < p1; p += VB) {
            int32_t jj[VB];
            T xx[VB][V];
#pragma unroll
            for (int u = 0; u < VB; ++u) jj[u] = cl[p + u];
#pragma unroll
            for (int u = 0; u < VB; ++u) xraw_vec<MODE, T, V>(k, jj[u], m0, xx[u]);
#pragma unroll
            for (int u = 0; u < VB; ++u)
#pragma unroll
                for (int b = 0; b < NS; ++b)
#pragma unroll
                    for (int v = 0; v < V; ++v) t[v][b] += vl[(p + u) * NS + b] * xx[u][v];
        }
        for (; p < p1; ++p) {
            T xv[V];
            xraw_vec<MODE, T, V>(k, cl[p], m0, xv);
#pragma unroll
            for (int b = 0; b < NS; ++b)
#pragma unroll
                for (int v = 0; v < V; ++v) t[v][b] += vl[p * NS + b] * xv[v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T a = 0;
#pragma unroll
            for (int b = 0; b < NS; ++b) a += k.coef[(m0 + v) * NS + b] * t[v][b];
            a *= xs_out<MODE>(k);
            if (s1 > s0) a += spmv_surface<MODE>(k, s0, s1, m0 + v);
            acc[v] = a;
        }
    }
}

// Wave-per-row SpMV with V adjacent ordinates per lane (form 2, more than 64
// ordinates): an item is a row and 64 V ordinates, so that a row of 96 or 128
// ordinates is one item (two of 64 in spmv_wave_kernel) and its stream values
// and columns are read once; each nonzero's x gather is one vector load per
// lane.  Same sums as spmv_wave_kernel, ordinate by ordinate.
template <int NS, class T, int MODE, int V>
__global__ __launch_bounds__(512) void spmv_vec_kernel(SpmvK<T> k, const int64_t *__restrict__ row_off,
                                                       const int32_t *__restrict__ col,
                                                       const T *__restrict__ vals, const T *__restrict__ fv)
{
    if (k.gate && *k.gate == 0) return;
    const int G = gridDim.x, X = k.nxcd;
    const int bx = blockIdx.x;
    const int per = G / X;
    const int lb = (bx % X) * per + bx / X;
    const int lane = threadIdx.x & 63;
    constexpr int CW = 64 * V;
    const int nchunk = (k.M + CW - 1) / CW;
    const int64_t nitems = k.n * nchunk;
    const int64_t i0 = (int64_t)lb * k.items_per_block;
    const int64_t i1 = i0 + k.items_per_block < nitems ? i0 + k.items_per_block : nitems;
    for (int64_t item = i0 + (threadIdx.x >> 6); item < i1; item += (blockDim.x >> 6)) {
        const int64_t iu =
            __builtin_amdgcn_readfirstlane((int)(nchunk == 1 ? item : item / nchunk));
        const int chunk = (int)(item - iu * nchunk);
        const int m0 = chunk * CW + V * lane;
        const bool on = m0 < k.M;   // M is a multiple of V: all V ordinates or none
        const int mm0 = on ? m0 : 0;
        RowEnds<T> re[V];
#pragma unroll
        for (int v = 0; v < V; ++v) re[v] = row_ends(k, iu, mm0 + v);
        const int64_t p0 = row_off[iu], p1 = row_off[iu + 1];
        T acc[V];
        row_sum_vec<NS, T, MODE, V>(k, col, vals, fv, p0, p1, re[0].s0, re[0].s1, mm0, acc);
        if (on) {
#pragma unroll
            for (int v = 0; v < V; ++v) spmv_finish(k, iu, m0 + v, acc[v], re[v]);
        }
    }
}

// LDS-staged sweep (at most 64 ordinates, so one item per row): a workgroup
// of W waves owns a contiguous range of rows and walks it in rounds of W rows,
// one row per wave.  The round's stream values and column indices (at most
// 64 W nonzeros) are brought in by coalesced vector loads of the whole
// workgroup and kept in LDS, two buffers deep: the loads of the next round
// are in flight while the waves compute the current one from LDS.  Many more
// bytes of the value streams are then in flight per CU than the scalar loads
// of the wave kernel allow, which is what the sweep waits on once the streams
// have left the caches.  A round with more nonzeros than the buffer reads
// them from global memory instead.  Sums are formed in the same order as in
// spmv_wave_kernel.
template <int NS, class T, int MODE, int W>
__global__ __launch_bounds__(64 * W) void spmv_lds_kernel(SpmvK<T> k, const int64_t *__restrict__ row_off,
                                                          const int32_t *__restrict__ col,
                                                          const T *__restrict__ vals, const T *__restrict__ fv)
{
    constexpr int CAP = 64 * W;   // nonzeros per staged round
    __shared__ T sv[2][CAP * NS];
    __shared__ int32_t sc[2][CAP];
    __shared__ T scoef[64 * NS];  // the lanes' coefficients, read once per row after its sums
    if (k.gate && *k.gate == 0) return;
    const int G = gridDim.x, X = k.nxcd;
    const int per = G / X;
    const int lb = (blockIdx.x % X) * per + blockIdx.x / X;
    const int64_t i0 = (int64_t)lb * k.items_per_block;
    const int64_t i1 = i0 + k.items_per_block < k.n ? i0 + k.items_per_block : k.n;
    if (i0 >= i1) return;   // uniform over the workgroup
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool on = lane < k.M;
    const int mm = on ? lane : 0;
    for (int e = tid; e < 64 * NS; e += 64 * W) scoef[e] = e < k.M * NS ? k.coef[e] : (T)0;
    // registers holding the next round on its way to LDS
    T rv[NS];
    int32_t rcol = 0;
    int64_t q0 = row_off[i0];
    int64_t r1 = i0 + W < i1 ? i0 + W : i1;
    int64_t cnt = row_off[r1] - q0;
    auto fetch = [&]() {
        if (cnt > CAP || cnt <= 0) return;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int64_t e = tid + s * 64 * W;
            rv[s] = vals[q0 * NS + (e < cnt * NS ? e : 0)];
        }
        rcol = col[q0 + (tid < cnt ? tid : 0)];
    };
    fetch();
    int buf = 0;
    for (int64_t r0 = i0; r0 < i1; r0 += W, buf ^= 1) {
        const bool staged = cnt <= CAP;
        if (staged) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int e = tid + s * 64 * W;
                if (e < cnt * NS) sv[buf][e] = rv[s];
            }
            if (tid < cnt) sc[buf][tid] = rcol;
        }
        const int64_t qc = q0, rend = r1;
        // buffer `buf` was last read two rounds ago, before the previous barrier
        __syncthreads();
        if (r0 + W < i1) {
            q0 = row_off[r0 + W];
            r1 = r0 + 2 * W < i1 ? r0 + 2 * W : i1;
            cnt = row_off[r1] - q0;
            fetch();
        }
        const int64_t iu = r0 + w;   // uniform over the wave
        if (iu < rend) {
            const RowEnds<T> re = row_ends(k, iu, mm);
            const int64_t p0 = row_off[iu], p1 = row_off[iu + 1];
            auto cf = [&](int b) { return scoef[mm * NS + b]; };
            const T acc = staged ? row_sum<NS, T, MODE>(k, &sc[buf][0], &sv[buf][0], fv, p0 - qc, p1 - qc, re, cf, mm)
                                 : row_sum<NS, T, MODE>(k, col, vals, fv, p0, p1, re, cf, mm);
            if (on) spmv_finish(k, iu, lane, acc, re);
        }
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
        const RowEnds<T> re = row_ends(k, i, m);
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
        if (re.s1 > re.s0) acc += spmv_surface<MODE>(k, re.s0, re.s1, m);
        spmv_finish(k, i, m, acc, re);
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
// Wave kernel (M >= 48), form 0: `wpb` waves per workgroup, each wave
// sweeping `ipw` (row, 64-ordinate chunk) items; with `xcd` = 8 workgroups
// are renumbered so that every die walks one contiguous range of rows.
// LDS-staged kernel, form 1 (48 <= M <= 64, 6 or 10 streams): `wpb` = 4 or 8
// waves, `rounds` rounds of one row per wave per workgroup.  Group kernel
// (M < 48): `threads` per workgroup (rows of M lanes).  The best shape per
// (rows, ordinates, streams, value size) is measured once per process on the
// problem's own operator and kept in a table (mlpg_get_tuning).
struct SpmvShape {
    int form = 0;
    int wpb = 4, ipw = 1, rounds = 1, xcd = 8, threads = 256, vec = 1;
};

// Form 2 (V ordinates per lane) applies to the transport operators when it
// makes fewer (row, ordinate) items than V/2 ordinates per lane would (form 0
// for V = 2): a multiple of V ordinates, more than 64 (96 and 128: V = 2;
// 256: V = 2 or 4).
static bool vec_form_fits(int M, int ns, int V)
{
    return (V == 2 || V == 4) && (ns == 6 || ns == 10) && M > 64 && M % V == 0 &&
           (M + 64 * V - 1) / (64 * V) < (M + 32 * V - 1) / (32 * V);
}

// Form 1 applies to one 64-ordinate chunk per row and the 2D/3D transport
// operators; its two LDS buffers (64 W nonzeros of values and columns each)
// stay within 64 KiB per workgroup.
static bool lds_form_fits(int M, int ns, int wpb, int tbytes)
{
    return M >= 48 && M <= 64 && (ns == 6 || ns == 10) && (wpb == 4 || wpb == 8) &&
           2 * 64 * wpb * (ns * tbytes + 4) <= 65536;
}

namespace {
struct TuneEntry {
    int64_t n;
    int M, ns, tbytes;
    SpmvShape shape;
    float us_best, us_default;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
std::atomic<bool> g_autotune{true};
// held while candidates are timed, so that threads serving several problems
// tune one key once and never time their candidates against each other
std::mutex g_tuning_mu;

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

// inserts or replaces the entry of e's key (caller holds g_tune_mu)
void put_entry(const TuneEntry &e)
{
    for (auto &o : g_tune)
        if (o.n == e.n && o.M == e.M && o.ns == e.ns && o.tbytes == e.tbytes) {
            o = e;
            return;
        }
    g_tune.push_back(e);
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
    const bool lds = sh.form == 1 && lds_form_fits(M, a.ns, sh.wpb, (int)sizeof(T));
    // form 2 loads V ordinates of an input row at once: the inputs must be
    // aligned to V elements (the solver's vectors are), and isotropic inputs
    // (one value per row) keep form 0
    const size_t va = sizeof(T) * (size_t)sh.vec;
    const bool vecf = sh.form == 2 && wave && vec_form_fits(M, a.ns, sh.vec) && !a.x_bcast &&
                      (uintptr_t)a.x % va == 0 && (uintptr_t)a.x2 % va == 0 && (uintptr_t)a.dinv % va == 0;
    unsigned blocks;
    int threads;
    if (wave) {
        // sh.wpb waves per workgroup, each taking sh.ipw items (forms 0 and 2)
        // or one row in each of sh.rounds rounds (form 1); grid a multiple of
        // the xcd count
        threads = 64 * sh.wpb;
        const int cw = vecf ? 64 * sh.vec : 64;
        const int64_t items = P.n * ((M + cw - 1) / cw);
        const int64_t per_block = (int64_t)sh.wpb * (lds ? std::max(sh.rounds, 1) : sh.ipw);
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
#define MLPG_SPMV_L(NSV, MD)                                                                       \
    if (sh.wpb == 4) spmv_lds_kernel<NSV, T, MD, 4><<<blocks, threads, 0, s>>>(k, k.row_off, k.col, k.vals, k.sval); \
    else spmv_lds_kernel<NSV, T, MD, 8><<<blocks, threads, 0, s>>>(k, k.row_off, k.col, k.vals, k.sval)
#define MLPG_SPMV_M(NSV, MD)                                                                       \
    if (wave) spmv_wave_kernel<NSV, T, MD><<<blocks, threads, 0, s>>>(k, k.row_off, k.col, k.vals, k.sval); \
    else spmv_group_kernel<NSV, T, MD><<<blocks, threads, 0, s>>>(k)
#define MLPG_SPMV_V(NSV, MD)                                                                       \
    if (sh.vec == 2) spmv_vec_kernel<NSV, T, MD, 2><<<blocks, threads, 0, s>>>(k, k.row_off, k.col, k.vals, k.sval); \
    else spmv_vec_kernel<NSV, T, MD, 4><<<blocks, threads, 0, s>>>(k, k.row_off, k.col, k.vals, k.sval)
#define MLPG_SPMV(NSV, KER)                                                       \
    switch (mode) {                                                               \
    case IN_PLAIN: KER(NSV, IN_PLAIN); break;                                     \
    case IN_DINV: KER(NSV, IN_DINV); break;                                       \
    case IN_BCAST: KER(NSV, IN_BCAST); break;                                     \
    default: KER(NSV, IN_X2); break;                                              \
    }
    if (lds) {
        if (a.ns == 6) { MLPG_SPMV(6, MLPG_SPMV_L); }
        else { MLPG_SPMV(10, MLPG_SPMV_L); }
    } else if (vecf) {
#define MLPG_SPMV_VM(NSV)                                                          \
        switch (mode) {                                                            \
        case IN_PLAIN: MLPG_SPMV_V(NSV, IN_PLAIN); break;                          \
        case IN_DINV: MLPG_SPMV_V(NSV, IN_DINV); break;                            \
        default: MLPG_SPMV_V(NSV, IN_X2); break;                                   \
        }
        if (a.ns == 6) { MLPG_SPMV_VM(6); }
        else { MLPG_SPMV_VM(10); }
#undef MLPG_SPMV_VM
    } else {
        switch (a.ns) {
        case 3: MLPG_SPMV(3, MLPG_SPMV_M); break;
        case 4: MLPG_SPMV(4, MLPG_SPMV_M); break;
        case 6: MLPG_SPMV(6, MLPG_SPMV_M); break;
        case 10: MLPG_SPMV(10, MLPG_SPMV_M); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef MLPG_SPMV
#undef MLPG_SPMV_V
#undef MLPG_SPMV_M
#undef MLPG_SPMV_L
    return hipGetLastError();
}

template <class T>
hipError_t launch_spmv(Problem &P, const SpmvArgsT<T> &a, hipStream_t s)
{
    SpmvShape sh;
    (void)find_shape(P.n, P.n_ord, a.ns, (int)sizeof(T), &sh);
    return launch_spmv_shape<T>(P, a, sh, s);
}

// Reads n4 x 32 bytes (a pass that evicts the caches before a timed launch);
// the guarded store never happens for finite data and keeps the reads alive.
__global__ void evict_kernel(const double4 *__restrict__ a, int64_t n4, double *sink)
{
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n4; t += (int64_t)gridDim.x * blockDim.x) {
        const double4 v = a[t];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc == 1.0e308) sink[0] = acc;
}

// Times every candidate shape of the transport sweep as the inner solver
// calls it (normalisation fused, per-ordinate column scale) on x -> y, both
// [n][M] scratch vectors of the caller, and records the fastest.  Runs once
// per (rows, ordinates, streams, value size) and process; never during a
// graph capture (the caller tunes before the first solve).  Before each
// timed launch the caller's scratch region `evict` (the Krylov basis) is read
// once, as the Gram-Schmidt passes read it between two sweeps of the Arnoldi
// loop, so that the candidates are compared with the stream values as far
// out of the caches as the solver finds them.
template <class T>
hipError_t tune_spmv(Problem &P, const SpmvArgsT<T> &a, const void *evict, size_t evict_bytes, hipStream_t s)
{
    SpmvShape cur;
    if (!g_autotune.load() || find_shape(P.n, P.n_ord, a.ns, (int)sizeof(T), &cur)) return hipSuccess;
    std::lock_guard<std::mutex> tuning(g_tuning_mu);
    if (find_shape(P.n, P.n_ord, a.ns, (int)sizeof(T), &cur)) return hipSuccess;   // tuned meanwhile
    std::vector<SpmvShape> cand;
    if (P.n_ord >= 48) {
        for (int wpb : {2, 4, 8})
            for (int ipw : {1, 2})
                for (int xcd : {8, 1}) {
                    SpmvShape c;
                    c.wpb = wpb; c.ipw = ipw; c.xcd = xcd;
                    cand.push_back(c);
                }
        for (int wpb : {4, 8})
            for (int rounds : {2, 4})
                if (lds_form_fits(P.n_ord, a.ns, wpb, (int)sizeof(T))) {
                    SpmvShape c;
                    c.form = 1; c.wpb = wpb; c.rounds = rounds; c.xcd = 8;
                    cand.push_back(c);
                }
        for (int V : {2, 4})
            if (vec_form_fits(P.n_ord, a.ns, V))
                for (int wpb : {2, 4, 8})
                    for (int xcd : {8, 1}) {
                        SpmvShape c;
                        c.form = 2; c.vec = V; c.wpb = wpb; c.xcd = xcd;
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
            if (evict && evict_bytes >= 32) {
                evict_kernel<<<2048, 256, 0, s>>>((const double4 *)evict, (int64_t)(evict_bytes / 32),
                                                  (double *)(void *)a.y);
                if ((e = hipGetLastError()) != hipSuccess) break;
            }
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
        if (c.form == d.form && c.wpb == d.wpb && c.ipw == d.ipw && c.xcd == d.xcd && c.threads == d.threads) dflt = t;
        if (t < best) {
            best = t;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    put_entry({P.n, P.n_ord, a.ns, (int)sizeof(T), pick, 1e3f * best, 1e3f * dflt});
    return hipSuccess;
}
template hipError_t tune_spmv<double>(Problem &, const SpmvArgsT<double> &, const void *, size_t, hipStream_t);
template hipError_t tune_spmv<float>(Problem &, const SpmvArgsT<float> &, const void *, size_t, hipStream_t);

void set_autotune(int mode)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (mode == 2) g_tune.clear();
    else g_autotune.store(mode != 0);
}

int get_tuning(int cap, mlpg_tune_entry *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int cnt = (int)g_tune.size();
    for (int i = 0; i < cnt && i < cap; ++i) {
        const TuneEntry &e = g_tune[i];
        const bool wave = e.M >= 48;
        out[i].n = e.n;
        out[i].n_ord = e.M;
        out[i].streams = e.ns;
        out[i].value_bytes = e.tbytes;
        out[i].form = wave ? e.shape.form : 0;
        out[i].waves_per_block = wave ? e.shape.wpb : 0;
        out[i].items_per_wave = wave && e.shape.form != 1 ? e.shape.ipw : (wave ? 1 : 0);
        out[i].rounds = wave && e.shape.form == 1 ? e.shape.rounds : (wave ? 1 : 0);
        out[i].xcd_split = wave ? e.shape.xcd : 0;
        out[i].threads = wave ? 64 * e.shape.wpb : e.shape.threads;
        out[i].ords_per_lane = wave && e.shape.form == 2 ? e.shape.vec : 1;
        out[i].us_best = e.us_best;
        out[i].us_default = e.us_default;
    }
    return cnt;
}

std::string set_tuning(const mlpg_tune_entry &t)
{
    if (t.n < 1 || t.n_ord < 1 || (t.value_bytes != 4 && t.value_bytes != 8)) return "bad n, n_ord or value_bytes";
    if (t.streams != 3 && t.streams != 4 && t.streams != 6 && t.streams != 10) return "streams must be 3, 4, 6 or 10";
    SpmvShape sh;
    if (t.n_ord >= 48) {
        if (t.xcd_split != 1 && t.xcd_split != 8) return "xcd_split must be 1 or 8";
        sh.xcd = t.xcd_split;
        sh.form = t.form;
        if (t.form == 0) {
            if (t.waves_per_block < 1 || t.waves_per_block > 8 || t.items_per_wave < 1 || t.items_per_wave > 64)
                return "form 0 needs 1..8 waves per block and 1..64 items per wave";
            sh.wpb = t.waves_per_block;
            sh.ipw = t.items_per_wave;
        } else if (t.form == 1) {
            if (!lds_form_fits(t.n_ord, t.streams, t.waves_per_block, t.value_bytes) || t.rounds < 1 ||
                t.rounds > 64)
                return "form 1 needs 48..64 ordinates, 6 or 10 streams, 4 or 8 waves (4 for 10 FP64 streams) "
                       "and 1..64 rounds";
            sh.wpb = t.waves_per_block;
            sh.rounds = t.rounds;
        } else if (t.form == 2) {
            if (!vec_form_fits(t.n_ord, t.streams, t.ords_per_lane) || t.waves_per_block < 1 ||
                t.waves_per_block > 8 || t.items_per_wave < 1 || t.items_per_wave > 64)
                return "form 2 needs 6 or 10 streams, 2 or 4 ordinates per lane dividing n_ord > 64 into fewer "
                       "items than form 0, 1..8 waves per block and 1..64 items per wave";
            sh.wpb = t.waves_per_block;
            sh.ipw = t.items_per_wave;
            sh.vec = t.ords_per_lane;
        } else {
            return "form must be 0, 1 or 2";
        }
    } else {
        if (t.threads < t.n_ord || t.threads > 512) return "threads must be in [n_ord, 512]";
        sh.threads = t.threads;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    put_entry({t.n, t.n_ord, t.streams, t.value_bytes, sh, t.us_best, t.us_default});
    return "";
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
