// Batched restarted GMRES on gfx950 (the Krylov solves of Sec. 4.2).
//
// `nb` independent systems of `n` unknowns advance together, vectors stored
// [n][nb] with the system index fastest (for the inner solves, nb = the
// ordinates; the outer scattering iteration uses nb = 1).  Each Arnoldi step
// is one operator application over all systems, then classical Gram-Schmidt
// with one reorthogonalisation in three streaming passes over the basis
//   pass 1: h1 = V^T w
//   pass 2: w -= V h1 and h2 = V^T w       (fused: the basis is read once)
//   pass 3: w -= V h2 and ||w||^2          (fused)
// with block partial sums reduced in a fixed order (deterministic), and a
// one-thread-per-system kernel for the Hessenberg column, Givens rotations,
// residual estimate and convergence flag.  The normalisation of the new
// basis vector is folded into the next operator application when the
// operator supports it.  Systems that converge stop updating; kernels of a
// sweep in which no system is active return at once, and the host reads the
// active count a few sweeps late (through host-visible memory and events) so
// that the queue never drains while it waits.
#include "internal.hpp"

namespace mlpg {

namespace {

constexpr int kThreads = 256;       // small kernels
constexpr int kMaxThreads = 512;    // streaming Gram-Schmidt passes (2 waves per SIMD: ~190 VGPRs fit)
constexpr int kPartBlocks = 256;    // workgroups (and partial sums) of a streaming pass
constexpr int kRowsPerThread = 4;
constexpr int KP = kMaxRestart + 1;   // basis vectors held in registers
constexpr int QC = 8;                 // partial sums reduced per LDS round
constexpr int kSlots = 8;

inline int rpb_of(int nb)
{
    int r = 1;
    while (r * 2 * nb <= kThreads) r *= 2;
    return r;
}

inline int pow2_floor(int v)
{
    int r = 1;
    while (r * 2 <= v) r *= 2;
    return r;
}

// Reduce acc[q] (q < NQ) over the rpb row groups of the block into
// part[blockIdx][q][m], QC values at a time through a fixed-shape LDS tree.
template <int NQ>
__device__ __forceinline__ void block_reduce_store(const double (&acc)[NQ], int rpb, int rl, int m, int nb,
                                                   double *red, double *part)
{
#pragma unroll
    for (int q0 = 0; q0 < NQ; q0 += QC) {
#pragma unroll
        for (int qq = 0; qq < QC; ++qq)
            if (q0 + qq < NQ) red[(rl * QC + qq) * nb + m] = acc[q0 + qq < NQ ? q0 + qq : 0];
        __syncthreads();
        for (int s = rpb >> 1; s > 0; s >>= 1) {
            if (rl < s) {
#pragma unroll
                for (int qq = 0; qq < QC; ++qq)
                    if (q0 + qq < NQ) red[(rl * QC + qq) * nb + m] += red[((rl + s) * QC + qq) * nb + m];
            }
            __syncthreads();
        }
        if (rl == 0) {
#pragma unroll
            for (int qq = 0; qq < QC; ++qq)
                if (q0 + qq < NQ) part[((int64_t)blockIdx.x * (KP + 1) + q0 + qq) * nb + m] = red[qq * nb + m];
        }
        __syncthreads();
    }
}

// part[b][q][m] = sum over the block's rows of V_q[i][m] * w[i][m], q < NQ,
// and part[b][NQ][m] = the block's share of ||w_m||^2 (products and sums in
// FP64 whatever the storage type T).  NQ is a
// template argument so that all NQ loads of a row issue back to back.
template <class T, int NQ>
__global__ __launch_bounds__(kMaxThreads) void dots_kernel(int64_t n, int nb, const T *__restrict__ V,
                                                           int64_t vstride, const T *__restrict__ w,
                                                           double *__restrict__ part, const int *__restrict__ gate)
{
    extern __shared__ double red[];
    if (gate && *gate == 0) return;
    const int rpb = blockDim.x / nb;
    const int rl = threadIdx.x / nb, m = threadIdx.x - rl * nb;
    double acc[NQ + 1];   // V_q^T w for q < NQ, then ||w||^2
#pragma unroll
    for (int q = 0; q <= NQ; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < n; i += (int64_t)gridDim.x * rpb) {
        const int64_t o = i * nb + m;
        T v[NQ];
        const double wv = (double)w[o];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = V[q * vstride + o];
        // keep every load of the row in flight before the first use (left
        // alone, the scheduler trades them for registers and serialises them)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += (double)v[q] * wv;
        acc[NQ] += wv * wv;
    }
    block_reduce_store<NQ + 1>(acc, rpb, rl, m, nb, red, part);
}

// Selective reorthogonalisation: a system needs the second Gram-Schmidt
// pass when the first one cancelled most of w, ||w'|| < 0.7 ||w|| (the
// "twice is enough" test of Kahan and Parlett).
__device__ __forceinline__ bool needs_reorth(double s1, double s2) { return s2 < 0.49 * s1; }

// MODE 0: w -= sum_q h1[q][m] V_q, then part = [V^T w, ||w||^2] and
//         z = dinv .* w (the next operator input when no second pass runs).
// MODE 1: the second pass, only for the systems that need it (s1, s2 are
//         ||w||^2 before and after the first pass): w -= sum_q h2[q][m] V_q,
//         part[0] = ||w||^2, z rewritten.  The whole launch returns at once
//         when no system needs it.
template <class T, int MODE, int NQ>
__global__ __launch_bounds__(kMaxThreads) void gs_update_kernel(int64_t n, int nb, const T *__restrict__ V,
                                                                int64_t vstride, T *__restrict__ w,
                                                                const double *__restrict__ h,
                                                                double *__restrict__ part,
                                                                const T *__restrict__ dinv,
                                                                T *__restrict__ z, const double *__restrict__ s1,
                                                                const double *__restrict__ s2,
                                                                const int *__restrict__ gate)
{
    extern __shared__ double red[];
    if (gate && *gate == 0) return;
    const int rpb = blockDim.x / nb;
    const int rl = threadIdx.x / nb, m = threadIdx.x - rl * nb;
    bool mine = true;
    if (MODE == 1) {
        mine = needs_reorth(s1[m], s2[m]);
        if (!__syncthreads_or(mine)) return;
    }
    constexpr int NA = MODE == 0 ? NQ + 1 : 1;
    double hq[NQ], acc[NA];
#pragma unroll
    for (int q = 0; q < NQ; ++q) hq[q] = mine ? h[q * nb + m] : 0.0;
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < n; i += (int64_t)gridDim.x * rpb) {
        const int64_t o = i * nb + m;
        T v[NQ];
        double wv = (double)w[o];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = V[q * vstride + o];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) wv -= hq[q] * (double)v[q];
        const T wt = (T)wv;
        if (MODE == 0 || mine) {
            w[o] = wt;
            if (z) z[o] = dinv ? dinv[o] * wt : wt;
        }
        wv = (double)wt;
        if (MODE == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += (double)v[q] * wv;
            acc[NQ] += wv * wv;
        } else {
            acc[0] += wv * wv;
        }
    }
    block_reduce_store<NA>(acc, rpb, rl, m, nb, red, part);
}

// out[q][m] = sum_b part[b][q][m]: one workgroup per q; threads split the
// block partials into interleaved strands (four independent accumulators each
// so that loads overlap), then a fixed-shape tree in LDS (deterministic).
__global__ __launch_bounds__(kThreads) void reduce_part_kernel(int nblk, int nq, int nb,
                                                               const double *__restrict__ part,
                                                               double *__restrict__ out, const int *__restrict__ gate,
                                                               const double *__restrict__ s1 = nullptr,
                                                               const double *__restrict__ s2 = nullptr)
{
    __shared__ double red[kThreads];
    if (gate && *gate == 0) return;
    const int q = blockIdx.x;
    const int ns = blockDim.x / nb;          // strands per system (power of two)
    const int st = threadIdx.x / nb, m = threadIdx.x - st * nb;
    if (s1 && !__syncthreads_or(needs_reorth(s1[m], s2[m]))) return;
    if (st >= ns) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = st;
    for (; b + 3 * ns < nblk; b += 4 * ns) {
        a0 += part[((int64_t)b * (KP + 1) + q) * nb + m];
        a1 += part[((int64_t)(b + ns) * (KP + 1) + q) * nb + m];
        a2 += part[((int64_t)(b + 2 * ns) * (KP + 1) + q) * nb + m];
        a3 += part[((int64_t)(b + 3 * ns) * (KP + 1) + q) * nb + m];
    }
    for (; b < nblk; b += ns) a0 += part[((int64_t)b * (KP + 1) + q) * nb + m];
    red[threadIdx.x] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int s = ns >> 1; s > 0; s >>= 1) {
        if (st < s) red[threadIdx.x] += red[threadIdx.x + s * nb];
        __syncthreads();
    }
    if (st == 0) out[q * nb + m] = red[m];
}

__global__ void sqrt_kernel(int nb, const double *in, double *out)
{
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < nb) out[m] = sqrt(fmax(in[m], 0.0));
}

// Number of threads of the (single) block with v != 0, written to count[0]
// and, when given, to a host-visible slot.
__device__ __forceinline__ void block_count(int v, int *count, int *host_slot)
{
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    if (v) atomicAdd(&s_cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        count[0] = s_cnt;
        if (host_slot) host_slot[0] = s_cnt;
    }
}

// Start of a restart cycle: beta = ||r||; decide which systems iterate.
__global__ __launch_bounds__(kThreads) void cycle_init_kernel(int nb, int k, const double *__restrict__ beta2, const double *__restrict__ fnorm,
                                  double tol, int max_its, const int *__restrict__ its, int *__restrict__ active,
                                  int *__restrict__ done, double *__restrict__ g, double *__restrict__ beta,
                                  double *__restrict__ resid, int *__restrict__ jend, int *__restrict__ nactive,
                                  int *__restrict__ host_slot)
{
    int m = threadIdx.x;
    int act = 0;
    if (m < nb) {
        double b = sqrt(fmax(beta2[m], 0.0));
        double fn = fnorm[m];
        beta[m] = b;
        resid[m] = fn > 0.0 ? b / fn : 0.0;
        bool ok = (fn == 0.0) || (b <= tol * fn);
        bool out = its[m] >= max_its;
        done[m] = ok ? 1 : (out ? 2 : 0);
        act = (!ok && !out) ? 1 : 0;
        active[m] = act;
        jend[m] = 0;
        for (int q = 0; q <= k; ++q) g[m * (k + 1) + q] = 0.0;
        g[m * (k + 1)] = b;
    }
    block_count(act, nactive, host_slot);
}

// Hessenberg column j, Givens rotations and convergence test per system;
// the column lives in registers while the earlier rotations are applied.
__global__ __launch_bounds__(kThreads) void arnoldi_kernel(int nb, int k, int j, const double *__restrict__ h1, const double *__restrict__ h2,
                               const double *__restrict__ hn2_second, double *__restrict__ H, double *__restrict__ cs,
                               double *__restrict__ sn, double *__restrict__ g, const double *__restrict__ fnorm,
                               double tol, int max_its, int *__restrict__ active, int *__restrict__ its,
                               int *__restrict__ jend, double *__restrict__ vscale, double *__restrict__ resid,
                               int *__restrict__ nactive, int *__restrict__ host_slot, const int *__restrict__ gate)
{
    if (gate && *gate == 0) {
        if (threadIdx.x == 0 && host_slot) host_slot[0] = 0;
        return;
    }
    int m = threadIdx.x;
    int still = 0;
    if (m < nb && active[m]) {
        double *Hm = H + (int64_t)m * (k + 1) * k;
        double *c = cs + m * k, *s = sn + m * k, *gm = g + m * (k + 1);
        // h1[j+1] = ||w||^2 before, h2[j+1] = after the first pass; the
        // second pass ran for this system only when it was needed
        const bool re = needs_reorth(h1[(j + 1) * nb + m], h2[(j + 1) * nb + m]);
        double hn = sqrt(fmax(re ? hn2_second[m] : h2[(j + 1) * nb + m], 0.0));
        double col[KP + 1];
        double cq[KP], sq[KP];
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            col[q] = (q <= j) ? h1[q * nb + m] + (re ? h2[q * nb + m] : 0.0) : 0.0;
            cq[q] = (q < j) ? c[q] : 1.0;
            sq[q] = (q < j) ? s[q] : 0.0;
        }
        col[KP] = 0.0;
#pragma unroll
        for (int q = 0; q < KP - 1; ++q) {
            if (q < j) {
                double a = col[q], b = col[q + 1];
                col[q] = cq[q] * a + sq[q] * b;
                col[q + 1] = -sq[q] * a + cq[q] * b;
            }
        }
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < KP; ++q)
            if (q == j) a = col[q];
        double den = sqrt(a * a + hn * hn);
        double cj = den == 0.0 ? 1.0 : a / den;
        double sj = den == 0.0 ? 0.0 : hn / den;
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            if (q < j) Hm[q * k + j] = col[q];
            if (q == j) Hm[q * k + j] = den;
        }
        c[j] = cj;
        s[j] = sj;
        double gj = gm[j];
        gm[j + 1] = -sj * gj;
        gm[j] = cj * gj;
        its[m] += 1;
        jend[m] = j + 1;
        double r = fabs(sj * gj);
        resid[m] = r / fnorm[m];
        if (r <= tol * fnorm[m] || hn == 0.0 || its[m] >= max_its) {
            active[m] = 0;
            vscale[m] = 0.0;
        } else {
            still = 1;
            vscale[m] = 1.0 / hn;
        }
    } else if (m < nb) {
        vscale[m] = 0.0;
    }
    block_count(still, nactive, host_slot);
}

// V_{j+1} = w * vscale (0 for systems that stopped).
template <class T>
__global__ void normalize_kernel(int64_t n, int nb, const T *__restrict__ w, const double *__restrict__ vscale,
                                 T *__restrict__ vout, const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    int m = (int)(t % nb);
    vout[t] = (T)((double)w[t] * vscale[m]);
}

template <class T>
__global__ void init_v0_kernel(int64_t n, int nb, const T *__restrict__ r, const double *__restrict__ beta,
                               const int *__restrict__ active, T *__restrict__ v0)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    int m = (int)(t % nb);
    v0[t] = active[m] ? (T)((double)r[t] / beta[m]) : (T)0;
}

// Least squares: back substitution H y = g over the jend columns.
__global__ void lsq_kernel(int nb, int k, const double *__restrict__ H, const double *__restrict__ g,
                           const int *__restrict__ jend, double *__restrict__ y)
{
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nb) return;
    const double *Hm = H + (int64_t)m * (k + 1) * k;
    const double *gm = g + m * (k + 1);
    int je = jend[m];
    for (int q = k - 1; q >= 0; --q) {
        if (q >= je) { y[q * nb + m] = 0.0; continue; }
        double s = gm[q];
        for (int p = q + 1; p < je; ++p) s -= Hm[q * k + p] * y[p * nb + m];
        y[q * nb + m] = s / Hm[q * k + q];
    }
}

// x += dinv .* (V y)
template <class T>
__global__ __launch_bounds__(kThreads) void x_update_kernel(int64_t n, int nb, int nq, const T *__restrict__ V,
                                                            int64_t vstride, const double *__restrict__ y,
                                                            const T *__restrict__ dinv, T *__restrict__ x)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    int m = (int)(t % nb);
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += y[q * nb + m] * (double)V[q * vstride + t];
    x[t] = (T)((double)x[t] + (dinv ? (double)dinv[t] * s : s));
}

// r = f - r
template <class T>
__global__ void residual_kernel(int64_t count, const T *__restrict__ f, T *__restrict__ r)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) r[t] = f[t] - r[t];
}

inline unsigned grid_of(int64_t count) { return (unsigned)((count + kThreads - 1) / kThreads); }

struct Launch {
    int rpb, threads;
    unsigned blocks;
    size_t shmem;
};

// Streaming passes: up to kPartBlocks workgroups of up to kMaxThreads
// threads, each thread covering at least kRowsPerThread rows, at least one
// full wave per workgroup.
Launch vec_launch(int64_t n, int nb)
{
    Launch L;
    const int rmax = pow2_floor(kMaxThreads / nb > 0 ? kMaxThreads / nb : 1);
    const int rmin = nb >= 64 ? 1 : 64 / pow2_floor(nb);
    int rpb = rmax;
    while (rpb > rmin && (n + (int64_t)rpb * kRowsPerThread - 1) / ((int64_t)rpb * kRowsPerThread) < kPartBlocks)
        rpb /= 2;
    L.rpb = rpb;
    L.threads = rpb * nb;
    int64_t b = (n + (int64_t)kRowsPerThread * rpb - 1) / ((int64_t)kRowsPerThread * rpb);
    if (b < 1) b = 1;
    L.blocks = (unsigned)(b < kPartBlocks ? b : kPartBlocks);
    L.shmem = sizeof(double) * QC * L.threads;
    return L;
}

// Algorithmic bytes of one streaming pass: nv vectors of n*nb elements plus
// the block partial sums it writes.
template <class T>
double pass_bytes(const KrylovT<T> &K, double nvec, int nq, unsigned blocks)
{
    return sizeof(T) * nvec * (double)K.n * K.nb + 8.0 * (double)blocks * nq * K.nb;
}

#define MLPG_NQ_CASES(X)                                                                                   \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
    X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31)

template <class T>
hipError_t dots(KrylovT<T> &K, const T *V, int nq, const T *w, double *out, const int *gate, hipStream_t s,
                bool timed = false, int64_t vstride = 0, bool norm_row = false)
{
    if (vstride == 0) vstride = K.vs;
    if (nq < 1 || nq > KP) return hipErrorInvalidValue;
    Launch L = vec_launch(K.n, K.nb);
    int id = timed ? prof_start(1, pass_bytes(K, nq + 1, nq, L.blocks), s) : -1;
    switch (nq) {
#define MLPG_DOTS_CASE(Q)                                                                                      \
    case Q:                                                                                                     \
        dots_kernel<T, Q><<<L.blocks, L.threads, L.shmem, s>>>(K.n, K.nb, V, vstride, w, K.part.p, gate);      \
        break;
        MLPG_NQ_CASES(MLPG_DOTS_CASE)
#undef MLPG_DOTS_CASE
    }
    prof_stop(id, s);
    // nq inner products, then ||w||^2 in row nq when norm_row is set
    const int nr = nq + (norm_row ? 1 : 0);
    reduce_part_kernel<<<nr, rpb_of(K.nb) * K.nb, 0, s>>>((int)L.blocks, nr, K.nb, K.part.p, out, gate);
    return hipGetLastError();
}

template <class T, int MODE>
hipError_t gs_update(KrylovT<T> &K, int nq, T *w, const double *h, double *out, const T *dinv, T *z,
                     const double *s1, const double *s2, const int *gate, hipStream_t s)
{
    if (nq < 1 || nq > KP) return hipErrorInvalidValue;
    Launch L = vec_launch(K.n, K.nb);
    // V_0..V_{nq-1} read, w read and written, dinv read and z written
    double nvec = nq + 2 + (z ? (dinv ? 2 : 1) : 0);
    int id = prof_start(MODE == 0 ? 2 : 3, pass_bytes(K, nvec, MODE == 0 ? nq + 1 : 1, L.blocks), s);
    switch (nq) {
#define MLPG_GS_CASE(Q)                                                                                        \
    case Q:                                                                                                     \
        gs_update_kernel<T, MODE, Q><<<L.blocks, L.threads, L.shmem, s>>>(K.n, K.nb, K.V.p, K.vs, w, h,         \
                                                                          K.part.p, dinv, z, s1, s2, gate);    \
        break;
        MLPG_NQ_CASES(MLPG_GS_CASE)
#undef MLPG_GS_CASE
    }
    prof_stop(id, s);
    const int nr = MODE == 0 ? nq + 1 : 1;
    reduce_part_kernel<<<nr, rpb_of(K.nb) * K.nb, 0, s>>>((int)L.blocks, nr, K.nb, K.part.p, out, gate,
                                                          MODE == 1 ? s1 : nullptr, MODE == 1 ? s2 : nullptr);
    return hipGetLastError();
}

}  // namespace

template <class T>
hipError_t KrylovT<T>::ensure(int64_t n_, int nb_, int k_)
{
    if (n == n_ && nb == nb_ && k == k_ && V.p) return hipSuccess;
    n = n_; nb = nb_; k = k_;
    hipError_t e;
    // Basis vectors are spaced by n*nb plus an odd number of 128-byte lines so
    // that the same row of different vectors does not fall into the same
    // cache set and memory channel (n*nb is often a large power of two).
    vs = n * nb + (int64_t)(21 * 128 / sizeof(T));
    if ((e = V.alloc((size_t)(k + 1) * vs)) != hipSuccess) return e;
    if ((e = w.alloc((size_t)n * nb)) != hipSuccess) return e;
    if ((e = w2.alloc((size_t)n * nb)) != hipSuccess) return e;
    if ((e = z.alloc((size_t)n * nb)) != hipSuccess) return e;
    if ((e = r.alloc((size_t)n * nb)) != hipSuccess) return e;
    part_blocks = kPartBlocks;   // partial-sum rows; vec_launch never exceeds it
    if ((e = part.alloc((size_t)part_blocks * (KP + 1) * nb)) != hipSuccess) return e;
    if ((e = h1.alloc((size_t)(KP + 1) * nb)) != hipSuccess) return e;
    if ((e = h2.alloc((size_t)(KP + 1) * nb)) != hipSuccess) return e;
    if ((e = H.alloc((size_t)nb * (k + 1) * k)) != hipSuccess) return e;
    if ((e = cs.alloc((size_t)nb * k)) != hipSuccess) return e;
    if ((e = sn.alloc((size_t)nb * k)) != hipSuccess) return e;
    if ((e = g.alloc((size_t)nb * (k + 1))) != hipSuccess) return e;
    if ((e = y.alloc((size_t)k * nb)) != hipSuccess) return e;
    if ((e = vscale.alloc(nb)) != hipSuccess) return e;
    if ((e = fnorm.alloc(nb)) != hipSuccess) return e;
    if ((e = beta.alloc(nb)) != hipSuccess) return e;
    if ((e = resid.alloc(nb)) != hipSuccess) return e;
    if ((e = active.alloc(nb)) != hipSuccess) return e;
    if ((e = done.alloc(nb)) != hipSuccess) return e;
    if ((e = its.alloc(nb)) != hipSuccess) return e;
    if ((e = jend.alloc(nb)) != hipSuccess) return e;
    if ((e = nactive.alloc(1)) != hipSuccess) return e;
    if (!nactive_host) {
        if ((e = hipHostMalloc((void **)&nactive_host, sizeof(int) * kSlots, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
            return e;
        if ((e = hipHostGetDevicePointer((void **)&nactive_hdev, nactive_host, 0)) != hipSuccess) return e;
        for (int i = 0; i < kSlots; ++i)
            if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class T>
void KrylovT<T>::release()
{
    V.release(); w.release(); w2.release(); z.release(); r.release(); part.release(); h1.release(); h2.release(); H.release();
    cs.release(); sn.release(); g.release(); y.release(); vscale.release(); fnorm.release(); beta.release();
    resid.release(); active.release(); done.release(); its.release(); jend.release(); nactive.release();
    if (nactive_host) {
        (void)hipHostFree(nactive_host);
        for (int i = 0; i < kSlots; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
    nactive_host = nullptr;
    nactive_hdev = nullptr;
    for (int i = 0; i < kSlots; ++i) ev[i] = nullptr;
    n = 0; nb = 0; k = 0;
}

template <class T>
int gmres_batched(Problem &P, KrylovT<T> &K, OpFnT<T> op, bool fused, void *ctx, const T *dinv, const T *f, T *x,
                  int64_t n, int nb, double tol, int restart, int max_its, int lag, bool x_zero, hipStream_t s,
                  int64_t *its_sum, int64_t *sweeps, double *res_max, bool *converged)
{
    MLPG_CHECK(nb >= 1 && nb <= kThreads, MLPG_ERR_ARG, "batched GMRES: system count must be in [1, 256]");
    MLPG_CHECK(restart >= 1 && restart <= kMaxRestart, MLPG_ERR_ARG, "GMRES restart must be in [1, 30]");
    MLPG_HIP(K.ensure(n, nb, restart));
    if (lag < 1) lag = 1;
    if (lag > kSlots - 1) lag = kSlots - 1;
    const int k = restart;
    const int64_t cnt = n * nb;
    const int nbt = ((nb + 63) / 64) * 64;
    const int *gate = K.nactive.p;
    // ||f||
    MLPG_HIP(dots<T>(K, f, 1, f, K.beta.p, nullptr, s, false, cnt));
    sqrt_kernel<<<(nb + 255) / 256, 256, 0, s>>>(nb, K.beta.p, K.fnorm.p);
    MLPG_HIP(hipMemsetAsync(K.its.p, 0, sizeof(int) * nb, s));
    if (x_zero) {
        MLPG_HIP(hipMemsetAsync(x, 0, sizeof(T) * cnt, s));
        MLPG_HIP(hipMemcpyAsync(K.r.p, f, sizeof(T) * cnt, hipMemcpyDeviceToDevice, s));
    } else {
        OpCallT<T> c;
        c.in = x;
        c.out = K.r.p;
        int rc = op(P, c, s, ctx);
        if (rc) return rc;
        residual_kernel<T><<<grid_of(cnt), kThreads, 0, s>>>(cnt, f, K.r.p);
    }
    int64_t sw = 0;
    for (;;) {
        MLPG_HIP(dots<T>(K, K.r.p, 1, K.r.p, K.h1.p, nullptr, s, false, cnt));
        cycle_init_kernel<<<1, nbt, 0, s>>>(nb, k, K.h1.p, K.fnorm.p, tol, max_its, K.its.p, K.active.p, K.done.p,
                                            K.g.p, K.beta.p, K.resid.p, K.jend.p, K.nactive.p, K.nactive_hdev);
        MLPG_HIP(hipStreamSynchronize(s));
        if (K.nactive_host[0] == 0) break;
        init_v0_kernel<T><<<grid_of(cnt), kThreads, 0, s>>>(n, nb, K.r.p, K.beta.p, K.active.p, K.V.p);
        int jc = 0;
        T *wcur = K.w.p, *wprev = K.w2.p;
        const int64_t base = sw;   // sweeps before this cycle
        for (int j = 0; j < k; ++j) {
            OpCallT<T> c;
            c.dinv = dinv;
            c.gate = gate;
            if (j == 0 || !fused) {
                c.in = K.V.p + (int64_t)j * K.vs;
            } else {
                // z = dinv .* w of the previous step, scaled by 1/h_{j,j-1};
                // the SpMV also stores the normalised basis vector V_j
                c.in = K.z.p;
                c.dinv = nullptr;
                c.colscale = K.vscale.p;
                c.vout = K.V.p + (int64_t)j * K.vs;
                c.vsrc = wprev;
            }
            c.out = wcur;
            int rc = op(P, c, s, ctx);
            if (rc) return rc;
            MLPG_HIP(dots<T>(K, K.V.p, j + 1, wcur, K.h1.p, gate, s, true, 0, true));
            // first pass (z written for every system), then the second pass for
            // the systems whose first pass cancelled most of w
            T *zz = fused ? K.z.p : nullptr;
            const double *s1 = K.h1.p + (int64_t)(j + 1) * nb, *s2 = K.h2.p + (int64_t)(j + 1) * nb;
            MLPG_HIP((gs_update<T, 0>(K, j + 1, wcur, K.h1.p, K.h2.p, dinv, zz, nullptr, nullptr, gate, s)));
            MLPG_HIP((gs_update<T, 1>(K, j + 1, wcur, K.h2.p, K.beta.p, dinv, zz, s1, s2, gate, s)));
            // K.beta holds ||w||^2 during the cycle; cycle_init rewrites it.
            const int slot = (int)(sw % kSlots);
            arnoldi_kernel<<<1, nbt, 0, s>>>(nb, k, j, K.h1.p, K.h2.p, K.beta.p, K.H.p, K.cs.p, K.sn.p, K.g.p,
                                             K.fnorm.p, tol, max_its, K.active.p, K.its.p, K.jend.p, K.vscale.p,
                                             K.resid.p, K.nactive.p, K.nactive_hdev + slot, gate);
            MLPG_HIP(hipEventRecord(K.ev[slot], s));
            sw++;
            jc = j + 1;
            if (j == k - 1) break;
            if (!fused)
                normalize_kernel<T><<<grid_of(cnt), kThreads, 0, s>>>(n, nb, wcur, K.vscale.p,
                                                                      K.V.p + (int64_t)(j + 1) * K.vs, gate);
            std::swap(wcur, wprev);
            // read the active count of the sweep `lag` steps back (same cycle)
            const int64_t chk = sw - lag;
            if (chk >= base) {
                const int cs = (int)(chk % kSlots);
                MLPG_HIP(hipEventSynchronize(K.ev[cs]));
                if (K.nactive_host[cs] == 0) break;
            }
        }
        lsq_kernel<<<(nb + 255) / 256, 256, 0, s>>>(nb, k, K.H.p, K.g.p, K.jend.p, K.y.p);
        x_update_kernel<T><<<grid_of(cnt), kThreads, 0, s>>>(n, nb, jc, K.V.p, K.vs, K.y.p, dinv, x);
        OpCallT<T> c;
        c.in = x;
        c.out = K.r.p;
        int rc = op(P, c, s, ctx);
        if (rc) return rc;
        residual_kernel<T><<<grid_of(cnt), kThreads, 0, s>>>(cnt, f, K.r.p);
        MLPG_HIP(hipGetLastError());
    }
    std::vector<int> its(nb), done(nb);
    std::vector<double> res(nb);
    MLPG_HIP(hipMemcpyAsync(its.data(), K.its.p, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipMemcpyAsync(done.data(), K.done.p, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipMemcpyAsync(res.data(), K.resid.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    MLPG_HIP(hipStreamSynchronize(s));
    int64_t tot = 0;
    double rm = 0.0;
    bool ok = true;
    for (int m = 0; m < nb; ++m) {
        tot += its[m];
        rm = res[m] > rm ? res[m] : rm;
        ok = ok && done[m] == 1;
    }
    *its_sum += tot;
    *sweeps += sw;
    if (rm > *res_max) *res_max = rm;
    *converged = *converged && ok;
    return MLPG_OK;
}

hipError_t batched_norm2(KrylovT<double> &K, const double *x, double *out, hipStream_t s)
{
    return dots<double>(K, x, 1, x, out, nullptr, s, false, K.n * K.nb);
}

template struct KrylovT<double>;
template struct KrylovT<float>;
template int gmres_batched<double>(Problem &, KrylovT<double> &, OpFnT<double>, bool, void *, const double *,
                                   const double *, double *, int64_t, int, double, int, int, int, bool, hipStream_t,
                                   int64_t *, int64_t *, double *, bool *);
template int gmres_batched<float>(Problem &, KrylovT<float> &, OpFnT<float>, bool, void *, const float *,
                                  const float *, float *, int64_t, int, double, int, int, int, bool, hipStream_t,
                                  int64_t *, int64_t *, double *, bool *);

}  // namespace mlpg
