// Batched restarted GMRES on gfx950 (the Krylov solves of Sec. 4.2).
//
// `nb` independent systems of `n` unknowns advance together, vectors stored
// [n][nb] with the system index fastest (for the inner solves, nb = the
// ordinates; the outer scattering iteration uses nb = 1).  Each Arnoldi step
// is one operator application over all systems, classical Gram-Schmidt with
// one reorthogonalisation in three streaming passes over the basis
//   pass 1: h1 = V^T w
//   pass 2: w -= V h1 and h2 = V^T w       (fused: the basis is read once)
//   pass 3: w -= V h2 and ||w||^2          (fused)
// with block partial sums reduced in a fixed order (deterministic), and a
// one-thread-per-system kernel for the Hessenberg column, Givens rotations,
// residual estimate and convergence flag.  Converged systems stop updating;
// the host looks at the count of active systems every few steps.
#include "internal.hpp"

namespace mlpg {

namespace {

constexpr int kThreads = 256;
constexpr int kPartBlocks = 512;
constexpr int KP = kMaxRestart + 1;   // basis vectors held in registers

inline int rpb_of(int nb)
{
    int r = 1;
    while (r * 2 * nb <= kThreads) r *= 2;
    return r;
}

// Reduce acc[q] over the row groups of the block into part[blockIdx][q][m].
template <int NQMAX>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NQMAX], int nq, int rpb, int rl, int m, int nb,
                                                   double *red, double *part)
{
    for (int q = 0; q < NQMAX; ++q) {
        if (q >= nq) break;
        red[rl * nb + m] = acc[q];
        __syncthreads();
        for (int s = rpb >> 1; s > 0; s >>= 1) {
            if (rl < s) red[rl * nb + m] += red[(rl + s) * nb + m];
            __syncthreads();
        }
        if (rl == 0) part[((int64_t)blockIdx.x * (KP + 1) + q) * nb + m] = red[m];
        __syncthreads();
    }
}

// part[b][q][m] = sum over the block's rows of V_q[i][m] * w[i][m], q < nq.
__global__ __launch_bounds__(kThreads) void dots_kernel(int64_t n, int nb, int nq, const double *__restrict__ V,
                                                        int64_t vstride, const double *__restrict__ w,
                                                        double *__restrict__ part)
{
    __shared__ double red[kThreads];
    const int rpb = blockDim.x / nb;
    const int rl = threadIdx.x / nb, m = threadIdx.x - rl * nb;
    double acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < n; i += (int64_t)gridDim.x * rpb) {
        const int64_t o = i * nb + m;
        const double wv = w[o];
#pragma unroll
        for (int q = 0; q < KP; ++q)
            if (q < nq) acc[q] += V[q * vstride + o] * wv;
    }
    block_reduce_store<KP>(acc, nq, rpb, rl, m, nb, red, part);
}

// w -= sum_q h[q][m] V_q ; then part = V^T w (MODE 0) or part[0] = ||w||^2 (MODE 1).
template <int MODE>
__global__ __launch_bounds__(kThreads) void gs_update_kernel(int64_t n, int nb, int nq, const double *__restrict__ V,
                                                             int64_t vstride, double *__restrict__ w,
                                                             const double *__restrict__ h,
                                                             double *__restrict__ part)
{
    __shared__ double red[kThreads];
    const int rpb = blockDim.x / nb;
    const int rl = threadIdx.x / nb, m = threadIdx.x - rl * nb;
    double hq[KP], acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        hq[q] = (q < nq) ? h[q * nb + m] : 0.0;
        acc[q] = 0.0;
    }
    for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < n; i += (int64_t)gridDim.x * rpb) {
        const int64_t o = i * nb + m;
        double vq[KP];
        double wv = w[o];
#pragma unroll
        for (int q = 0; q < KP; ++q)
            if (q < nq) {
                vq[q] = V[q * vstride + o];
                wv -= hq[q] * vq[q];
            }
        w[o] = wv;
        if (MODE == 0) {
#pragma unroll
            for (int q = 0; q < KP; ++q)
                if (q < nq) acc[q] += vq[q] * wv;
        } else {
            acc[0] += wv * wv;
        }
    }
    block_reduce_store<KP>(acc, MODE == 0 ? nq : 1, rpb, rl, m, nb, red, part);
}

// out[q][m] = sum_b part[b][q][m]  (fixed order)
__global__ void reduce_part_kernel(int nblk, int nq, int nb, const double *__restrict__ part, double *__restrict__ out)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * nb) return;
    int q = t / nb, m = t - q * nb;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[((int64_t)b * (KP + 1) + q) * nb + m];
    out[t] = s;
}

__global__ void sqrt_kernel(int nb, const double *in, double *out)
{
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < nb) out[m] = sqrt(fmax(in[m], 0.0));
}

// Count of 1s in flag[0..nb) from a single block, written to *count.
__device__ __forceinline__ void block_count(int v, int *count)
{
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    if (v) atomicAdd(&s_cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) *count = s_cnt;
}

// Start of a restart cycle: beta = ||r||; decide which systems iterate.
__global__ void cycle_init_kernel(int nb, int k, const double *__restrict__ beta2, const double *__restrict__ fnorm,
                                  double tol, int max_its, const int *__restrict__ its, int *__restrict__ active,
                                  int *__restrict__ done, double *__restrict__ g, double *__restrict__ beta,
                                  double *__restrict__ resid, int *__restrict__ jend, int *__restrict__ nactive)
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
    block_count(act, nactive);
}

// Hessenberg column j, Givens rotations and convergence test per system.
__global__ void arnoldi_kernel(int nb, int k, int j, const double *__restrict__ h1, const double *__restrict__ h2,
                               const double *__restrict__ hn2, double *__restrict__ H, double *__restrict__ cs,
                               double *__restrict__ sn, double *__restrict__ g, const double *__restrict__ fnorm,
                               double tol, int max_its, int *__restrict__ active, int *__restrict__ its,
                               int *__restrict__ jend, double *__restrict__ hnv, double *__restrict__ resid,
                               int *__restrict__ nactive)
{
    int m = threadIdx.x;
    int still = 0;
    if (m < nb && active[m]) {
        double *Hm = H + (int64_t)m * (k + 1) * k;
        double *c = cs + m * k, *s = sn + m * k, *gm = g + m * (k + 1);
        double hn = sqrt(fmax(hn2[m], 0.0));
        hnv[m] = hn;
        for (int q = 0; q <= j; ++q) Hm[q * k + j] = h1[q * nb + m] + h2[q * nb + m];
        Hm[(j + 1) * k + j] = hn;
        for (int q = 0; q < j; ++q) {
            double a = Hm[q * k + j], b = Hm[(q + 1) * k + j];
            Hm[q * k + j] = c[q] * a + s[q] * b;
            Hm[(q + 1) * k + j] = -s[q] * a + c[q] * b;
        }
        double a = Hm[j * k + j], b = Hm[(j + 1) * k + j];
        double den = sqrt(a * a + b * b);
        c[j] = den == 0.0 ? 1.0 : a / den;
        s[j] = den == 0.0 ? 0.0 : b / den;
        Hm[j * k + j] = den;
        Hm[(j + 1) * k + j] = 0.0;
        gm[j + 1] = -s[j] * gm[j];
        gm[j] = c[j] * gm[j];
        its[m] += 1;
        jend[m] = j + 1;
        double r = fabs(gm[j + 1]);
        resid[m] = r / fnorm[m];
        if (r <= tol * fnorm[m] || hn == 0.0 || its[m] >= max_its) active[m] = 0;
        else still = 1;
    }
    block_count(still, nactive);
}

// V_{j+1} = w / h_{j+1,j} for systems still iterating, else 0.
__global__ void normalize_kernel(int64_t n, int nb, const double *__restrict__ w, const double *__restrict__ hnv,
                                 const int *__restrict__ active, double *__restrict__ vout)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    int m = (int)(t % nb);
    vout[t] = active[m] ? w[t] / hnv[m] : 0.0;
}

__global__ void init_v0_kernel(int64_t n, int nb, const double *__restrict__ r, const double *__restrict__ beta,
                               const int *__restrict__ active, double *__restrict__ v0)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    int m = (int)(t % nb);
    v0[t] = active[m] ? r[t] / beta[m] : 0.0;
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
__global__ __launch_bounds__(kThreads) void x_update_kernel(int64_t n, int nb, int nq, const double *__restrict__ V,
                                                            int64_t vstride, const double *__restrict__ y,
                                                            const double *__restrict__ dinv, double *__restrict__ x)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    int m = (int)(t % nb);
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += y[q * nb + m] * V[q * vstride + t];
    x[t] += dinv ? dinv[t] * s : s;
}

// r = f - r
__global__ void residual_kernel(int64_t count, const double *__restrict__ f, double *__restrict__ r)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) r[t] = f[t] - r[t];
}

inline unsigned grid_of(int64_t count) { return (unsigned)((count + kThreads - 1) / kThreads); }

}  // namespace

hipError_t Krylov::ensure(int64_t n_, int nb_, int k_)
{
    if (n == n_ && nb == nb_ && k == k_ && V.p) return hipSuccess;
    n = n_; nb = nb_; k = k_;
    hipError_t e;
    if ((e = V.alloc((size_t)(k + 1) * n * nb)) != hipSuccess) return e;
    if ((e = w.alloc((size_t)n * nb)) != hipSuccess) return e;
    if ((e = r.alloc((size_t)n * nb)) != hipSuccess) return e;
    part_blocks = kPartBlocks;
    if ((e = part.alloc((size_t)part_blocks * (KP + 1) * nb)) != hipSuccess) return e;
    if ((e = h1.alloc((size_t)(KP + 1) * nb)) != hipSuccess) return e;
    if ((e = h2.alloc((size_t)(KP + 1) * nb)) != hipSuccess) return e;
    if ((e = H.alloc((size_t)nb * (k + 1) * k)) != hipSuccess) return e;
    if ((e = cs.alloc((size_t)nb * k)) != hipSuccess) return e;
    if ((e = sn.alloc((size_t)nb * k)) != hipSuccess) return e;
    if ((e = g.alloc((size_t)nb * (k + 1))) != hipSuccess) return e;
    if ((e = y.alloc((size_t)k * nb)) != hipSuccess) return e;
    if ((e = fnorm.alloc(nb)) != hipSuccess) return e;
    if ((e = beta.alloc(nb)) != hipSuccess) return e;
    if ((e = resid.alloc(nb)) != hipSuccess) return e;
    if ((e = active.alloc(nb)) != hipSuccess) return e;
    if ((e = done.alloc(nb)) != hipSuccess) return e;
    if ((e = its.alloc(nb)) != hipSuccess) return e;
    if ((e = jend.alloc(nb)) != hipSuccess) return e;
    if ((e = nactive.alloc(1)) != hipSuccess) return e;
    if (!nactive_host) {
        if ((e = hipHostMalloc((void **)&nactive_host, sizeof(int), hipHostMallocDefault)) != hipSuccess) return e;
    }
    return hipSuccess;
}

void Krylov::release()
{
    V.release(); w.release(); r.release(); part.release(); h1.release(); h2.release(); H.release();
    cs.release(); sn.release(); g.release(); y.release(); fnorm.release(); beta.release(); resid.release();
    active.release(); done.release(); its.release(); jend.release(); nactive.release();
    if (nactive_host) (void)hipHostFree(nactive_host);
    nactive_host = nullptr;
    n = 0; nb = 0; k = 0;
}

namespace {

struct Launch {
    int rpb, threads;
    unsigned blocks;
};

Launch vec_launch(int64_t n, int nb, int part_blocks)
{
    Launch L;
    L.rpb = rpb_of(nb);
    L.threads = L.rpb * nb;
    int64_t b = (n + L.rpb - 1) / L.rpb;
    L.blocks = (unsigned)(b < part_blocks ? b : part_blocks);
    return L;
}

hipError_t dots(Krylov &K, const double *V, int nq, const double *w, double *out, hipStream_t s)
{
    Launch L = vec_launch(K.n, K.nb, K.part_blocks);
    dots_kernel<<<L.blocks, L.threads, 0, s>>>(K.n, K.nb, nq, V, K.n * K.nb, w, K.part.p);
    reduce_part_kernel<<<grid_of((int64_t)nq * K.nb), kThreads, 0, s>>>((int)L.blocks, nq, K.nb, K.part.p, out);
    return hipGetLastError();
}

template <int MODE>
hipError_t gs_update(Krylov &K, int nq, const double *h, double *out, hipStream_t s)
{
    Launch L = vec_launch(K.n, K.nb, K.part_blocks);
    gs_update_kernel<MODE><<<L.blocks, L.threads, 0, s>>>(K.n, K.nb, nq, K.V.p, K.n * K.nb, K.w.p, h, K.part.p);
    reduce_part_kernel<<<grid_of((int64_t)(MODE == 0 ? nq : 1) * K.nb), kThreads, 0, s>>>(
        (int)L.blocks, MODE == 0 ? nq : 1, K.nb, K.part.p, out);
    return hipGetLastError();
}

}  // namespace

int gmres_batched(Problem &P, Krylov &K, OpFn op, void *ctx, const double *dinv, const double *f, double *x,
                  int64_t n, int nb, double tol, int restart, int max_its, int check_every, bool x_zero,
                  hipStream_t s, int64_t *its_sum, int64_t *sweeps, double *res_max, bool *converged)
{
    MLPG_CHECK(nb >= 1 && nb <= 1024, MLPG_ERR_ARG, "batched GMRES: system count must be in [1, 1024]");
    MLPG_CHECK(restart >= 1 && restart <= kMaxRestart, MLPG_ERR_ARG, "GMRES restart must be in [1, 30]");
    MLPG_HIP(K.ensure(n, nb, restart));
    const int k = restart;
    const int64_t cnt = n * nb;
    const int nbt = ((nb + 63) / 64) * 64;
    // ||f||
    MLPG_HIP(dots(K, f, 1, f, K.beta.p, s));
    sqrt_kernel<<<(nb + 255) / 256, 256, 0, s>>>(nb, K.beta.p, K.fnorm.p);
    MLPG_HIP(hipMemsetAsync(K.its.p, 0, sizeof(int) * nb, s));
    if (x_zero) {
        MLPG_HIP(hipMemsetAsync(x, 0, sizeof(double) * cnt, s));
        MLPG_HIP(hipMemcpyAsync(K.r.p, f, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
    } else {
        int rc = op(P, x, nullptr, K.r.p, s, ctx);
        if (rc) return rc;
        residual_kernel<<<grid_of(cnt), kThreads, 0, s>>>(cnt, f, K.r.p);
    }
    int64_t sw = 0;
    for (;;) {
        MLPG_HIP(dots(K, K.r.p, 1, K.r.p, K.h1.p, s));
        cycle_init_kernel<<<1, nbt, 0, s>>>(nb, k, K.h1.p, K.fnorm.p, tol, max_its, K.its.p, K.active.p, K.done.p,
                                            K.g.p, K.beta.p, K.resid.p, K.jend.p, K.nactive.p);
        MLPG_HIP(hipMemcpyAsync(K.nactive_host, K.nactive.p, sizeof(int), hipMemcpyDeviceToHost, s));
        MLPG_HIP(hipStreamSynchronize(s));
        if (*K.nactive_host == 0) break;
        init_v0_kernel<<<grid_of(cnt), kThreads, 0, s>>>(n, nb, K.r.p, K.beta.p, K.active.p, K.V.p);
        int jc = 0;
        for (int j = 0; j < k; ++j) {
            const double *vj = K.V.p + (int64_t)j * cnt;
            int rc = op(P, vj, dinv, K.w.p, s, ctx);
            if (rc) return rc;
            MLPG_HIP(dots(K, K.V.p, j + 1, K.w.p, K.h1.p, s));
            MLPG_HIP(gs_update<0>(K, j + 1, K.h1.p, K.h2.p, s));
            MLPG_HIP(gs_update<1>(K, j + 1, K.h2.p, K.beta.p + 0, s));
            // K.beta is reused as ||w||^2 scratch here; cycle_init rewrites it.
            arnoldi_kernel<<<1, nbt, 0, s>>>(nb, k, j, K.h1.p, K.h2.p, K.beta.p, K.H.p, K.cs.p, K.sn.p, K.g.p,
                                             K.fnorm.p, tol, max_its, K.active.p, K.its.p, K.jend.p, K.y.p,
                                             K.resid.p, K.nactive.p);
            sw++;
            jc = j + 1;
            if (j == k - 1) break;
            if ((j + 1) % check_every == 0) {
                MLPG_HIP(hipMemcpyAsync(K.nactive_host, K.nactive.p, sizeof(int), hipMemcpyDeviceToHost, s));
                MLPG_HIP(hipStreamSynchronize(s));
                if (*K.nactive_host == 0) break;
            }
            // the ||w|| of each system sits in K.y (first nb entries) until lsq
            normalize_kernel<<<grid_of(cnt), kThreads, 0, s>>>(n, nb, K.w.p, K.y.p, K.active.p,
                                                               K.V.p + (int64_t)(j + 1) * cnt);
        }
        lsq_kernel<<<(nb + 255) / 256, 256, 0, s>>>(nb, k, K.H.p, K.g.p, K.jend.p, K.y.p);
        x_update_kernel<<<grid_of(cnt), kThreads, 0, s>>>(n, nb, jc, K.V.p, cnt, K.y.p, dinv, x);
        int rc = op(P, x, nullptr, K.r.p, s, ctx);
        if (rc) return rc;
        residual_kernel<<<grid_of(cnt), kThreads, 0, s>>>(cnt, f, K.r.p);
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

}  // namespace mlpg
