// Meshless integration on gfx950 (Sec. 2.2, Sec. 3.2, Alg. 1, App. A), in
// 2D (fan triangles) and 3D (fan tetrahedra).
//
// One workgroup per cell.  The functions that can be nonzero on the cell
// (the cell's generator and the overlap neighbours whose support reaches the
// cell) are staged in LDS.  Each thread takes quadrature points of the fan
// triangles, evaluates the moment matrix M = sum_j V_j P P^T W_j and its
// gradient, factors M by Cholesky in FP64 (dropping one order while a pivot
// is below 1e-6 of the largest diagonal entry), forms C = M^-1 e0 and
// dC = -M^-1 dM C, and adds w N_a N_b, w dN_a N_b and w dN_a dN_b for every
// pair of functions active at the point into an LDS Gram tile with LDS FP64
// atomics.  The tile is then scattered into the global CSR blocks with one
// FP64 atomic per pair and block.  When the Gram tile of a cell would not
// fit in LDS, the pair rows are split into tiles and the points revisited.
#include "internal.hpp"

namespace mlpg {

__constant__ double c_tri_pts[kTriRule][2];
__constant__ double c_tri_w[kTriRule];
__constant__ double c_seg_pts[kSegRule];
__constant__ double c_seg_w[kSegRule];

namespace {
hipError_t upload_rules3(hipStream_t s);
}

hipError_t upload_rules(hipStream_t s)
{
    const Rules &r = rules();
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tri_pts), r.tri_pts, sizeof(r.tri_pts), 0,
                                          hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tri_w), r.tri_w, sizeof(r.tri_w), 0, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_seg_pts), r.seg_pts, sizeof(r.seg_pts), 0, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_seg_w), r.seg_w, sizeof(r.seg_w), 0, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = upload_rules3(s);
    return e;
}

namespace {

constexpr int kThreads = 256;
constexpr int kThreads3 = 256;   // 3D: one quadrature point per thread, its RK correction kept in registers

template <int ORD>
struct Basis2 {
    static constexpr int B = ORD == 0 ? 1 : (ORD == 1 ? 3 : 6);
};

__host__ __device__ constexpr int bsize2(int o) { return o == 0 ? 1 : (o == 1 ? 3 : 6); }

// Cubic B-spline in q = |r| / h, h = R/2: returns W and the factor W'(q)/q
// so that grad W = (W'(q)/q) r / h^2.  Support q < 2.
__device__ __forceinline__ double spline(double r2, double h, double *dfac)
{
    double q = sqrt(r2) / h;
    if (q < 1.0) {
        *dfac = (-3.0 + 2.25 * q) / (h * h);
        return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    }
    if (q < 2.0) {
        double t = 2.0 - q;
        *dfac = (-0.75 * t * t / q) / (h * h);
        return 0.25 * t * t * t;
    }
    *dfac = 0.0;
    return 0.0;
}

// Monomials of degree <= ORD in z (2D): [1, z0, z1, z0^2, z0 z1, z1^2] and
// their z-derivatives.
template <int ORD>
__device__ __forceinline__ void basis2(double z0, double z1, double *P, double *D0, double *D1)
{
    P[0] = 1.0; D0[0] = 0.0; D1[0] = 0.0;
    if (ORD >= 1) {
        P[1] = z0; D0[1] = 1.0; D1[1] = 0.0;
        P[2] = z1; D0[2] = 0.0; D1[2] = 1.0;
    }
    if (ORD >= 2) {
        P[3] = z0 * z0; D0[3] = 2.0 * z0; D1[3] = 0.0;
        P[4] = z0 * z1; D0[4] = z1;       D1[4] = z0;
        P[5] = z1 * z1; D0[5] = 0.0;      D1[5] = 2.0 * z1;
    }
}

// Cholesky of the leading b x b block of M (B x B storage) with the pivot
// test; solves for C = M^-1 e0 and dC_g = -M^-1 dM_g C.  Returns false when a
// pivot fails.
template <int B>
__device__ __forceinline__ bool chol_solve(int b, const double (&M)[B][B], const double (&dM0)[B][B],
                                           const double (&dM1)[B][B], double (&C)[B], double (&dC0)[B],
                                           double (&dC1)[B])
{
    double L[B][B];
    double dmax = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k)
        if (k < b) dmax = fmax(dmax, M[k][k]);
    if (!(dmax > 0.0)) return false;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        if (k >= b) break;
        double s = M[k][k];
#pragma unroll
        for (int p = 0; p < B; ++p)
            if (p < k) s -= L[k][p] * L[k][p];
        if (!(s > 1e-6 * dmax)) return false;
        L[k][k] = sqrt(s);
        double inv = 1.0 / L[k][k];
#pragma unroll
        for (int r = 0; r < B; ++r) {
            if (r <= k || r >= b) continue;
            double t = M[r][k];
#pragma unroll
            for (int p = 0; p < B; ++p)
                if (p < k) t -= L[r][p] * L[k][p];
            L[r][k] = t * inv;
        }
    }
    auto solve = [&](const double (&rhs)[B], double (&out)[B]) {
        double t[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (k >= b) { t[k] = 0.0; continue; }
            double s = rhs[k];
#pragma unroll
            for (int p = 0; p < B; ++p)
                if (p < k) s -= L[k][p] * t[p];
            t[k] = s / L[k][k];
        }
#pragma unroll
        for (int k = B - 1; k >= 0; --k) {
            if (k >= b) { out[k] = 0.0; continue; }
            double s = t[k];
#pragma unroll
            for (int p = 0; p < B; ++p)
                if (p > k && p < b) s -= L[p][k] * out[p];
            out[k] = s / L[k][k];
        }
    };
    double e0[B];
#pragma unroll
    for (int k = 0; k < B; ++k) e0[k] = (k == 0) ? 1.0 : 0.0;
    solve(e0, C);
    double r0[B], r1[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < B; ++q)
            if (r < b && q < b) {
                s0 += dM0[r][q] * C[q];
                s1 += dM1[r][q] * C[q];
            }
        r0[r] = -s0;
        r1[r] = -s1;
    }
    solve(r0, dC0);
    solve(r1, dC1);
    return true;
}

// RK correction at point y from the staged candidates.  Returns the order
// used (-1: no function covers y) and the bitmask of active candidates.
template <int ORD>
__device__ int rk_prepare(double y0, double y1, int A, const double *sx, const double *sR, const double *sV, double hs,
                          double (&C)[Basis2<ORD>::B], double (&dC0)[Basis2<ORD>::B],
                          double (&dC1)[Basis2<ORD>::B], uint64_t *mask)
{
    constexpr int B = Basis2<ORD>::B;
    double M[B][B], dM0[B][B], dM1[B][B];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int s = 0; s < B; ++s) { M[r][s] = 0.0; dM0[r][s] = 0.0; dM1[r][s] = 0.0; }
    uint64_t act = 0;
    const double ihs = 1.0 / hs;
    for (int a = 0; a < A; ++a) {
        double r0 = y0 - sx[2 * a], r1 = y1 - sx[2 * a + 1];
        double h = 0.5 * sR[a];
        double r2 = r0 * r0 + r1 * r1;
        if (!(r2 < 4.0 * h * h)) continue;
        double dfac;
        double W = spline(r2, h, &dfac);
        if (W == 0.0) continue;
        act |= (1ull << a);
        double dW0 = dfac * r0, dW1 = dfac * r1;
        double P[B], D0[B], D1[B];
        basis2<ORD>(r0 * ihs, r1 * ihs, P, D0, D1);
        double v = sV[a];
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int s = 0; s < B; ++s) {
                if (s < r) continue;
                double pp = P[r] * P[s];
                M[r][s] += v * pp * W;
                dM0[r][s] += v * ((D0[r] * P[s] + P[r] * D0[s]) * ihs * W + pp * dW0);
                dM1[r][s] += v * ((D1[r] * P[s] + P[r] * D1[s]) * ihs * W + pp * dW1);
            }
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int s = 0; s < B; ++s)
            if (s < r) { M[r][s] = M[s][r]; dM0[r][s] = dM0[s][r]; dM1[r][s] = dM1[s][r]; }
    *mask = act;
    if (act == 0) return -1;
#pragma unroll
    for (int o = ORD; o >= 0; --o) {
        if (chol_solve<B>(bsize2(o), M, dM0, dM1, C, dC0, dC1)) return o;
    }
    return -1;
}

template <int ORD>
__device__ __forceinline__ void rk_value(double y0, double y1, int a, const double *sx, const double *sR,
                                         const double *sV, double hs, const double (&C)[Basis2<ORD>::B],
                                         const double (&dC0)[Basis2<ORD>::B], const double (&dC1)[Basis2<ORD>::B],
                                         double *N, double *dN0, double *dN1)
{
    constexpr int B = Basis2<ORD>::B;
    double r0 = y0 - sx[2 * a], r1 = y1 - sx[2 * a + 1];
    double h = 0.5 * sR[a];
    double dfac;
    double W = spline(r0 * r0 + r1 * r1, h, &dfac);
    double dW0 = dfac * r0, dW1 = dfac * r1;
    const double ihs = 1.0 / hs;
    double P[B], D0[B], D1[B];
    basis2<ORD>(r0 * ihs, r1 * ihs, P, D0, D1);
    double pc = 0.0, t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int r = 0; r < B; ++r) {
        pc += P[r] * C[r];
        t0 += D0[r] * ihs * C[r] + P[r] * dC0[r];
        t1 += D1[r] * ihs * C[r] + P[r] * dC1[r];
    }
    double v = sV[a];
    *N = v * pc * W;
    *dN0 = v * (t0 * W + pc * dW0);
    *dN1 = v * (t1 * W + pc * dW1);
}

// Smooth material fields: each moves a + b prod_a cos(k y_a + phase) of a
// quadrature point's weight from material 0 to its material (the spatially
// varying opacities of the manufactured problems, Sec. 5.1).
struct FieldSet {
    int n;
    double par[kMaxFields][4];   // a, b, k, phase
    int mat[kMaxFields];
    int nshell;                  // shells (annuli in 2D): centre, inner and outer radius
    double shell[kMaxFields][5];
    int shell_mat[kMaxFields];
};

// w times the fraction of every material at y: the box indicator (material
// `mat`), overridden by the shells containing y (last match wins), then the
// fields in order.  Unrolled over kMaxMat so that the fractions stay in
// registers.
template <int D>
__device__ __forceinline__ void material_weights(const double *y, int mat, double w, const FieldSet &F,
                                                 double (&wf)[kMaxMat])
{
    for (int r = 0; r < F.nshell; ++r) {
        double d2 = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) d2 += (y[a] - F.shell[r][a]) * (y[a] - F.shell[r][a]);
        const double d = sqrt(d2);
        if (d >= F.shell[r][D] && d <= F.shell[r][D + 1]) mat = F.shell_mat[r];
    }
    double f[kMaxMat];
#pragma unroll
    for (int m = 0; m < kMaxMat; ++m) f[m] = m == mat ? 1.0 : 0.0;
    for (int r = 0; r < F.n; ++r) {
        double pr = 1.0;
#pragma unroll
        for (int a = 0; a < D; ++a) pr *= cos(F.par[r][2] * y[a] + F.par[r][3]);
        const double v = F.par[r][0] + F.par[r][1] * pr;
        const int t = F.mat[r];
#pragma unroll
        for (int m = 1; m < kMaxMat; ++m)
            if (m == t) f[m] += v;
        f[0] -= v;
    }
#pragma unroll
    for (int m = 0; m < kMaxMat; ++m) wf[m] = w * f[m];
}

__device__ __forceinline__ int material_at(double y0, double y1, int nreg, const double *lo, const double *hi,
                                           const int32_t *mat)
{
    int m = 0;
    for (int r = 0; r < nreg; ++r)
        if (y0 >= lo[2 * r] && y0 <= hi[2 * r] && y1 >= lo[2 * r + 1] && y1 <= hi[2 * r + 1]) m = mat[r];
    return m;
}

__device__ __forceinline__ int64_t find_col(const int64_t *row_off, const int32_t *col, int64_t i, int32_t j)
{
    int64_t lo = row_off[i], hi = row_off[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t cm = col[mid];
        if (cm == j) return mid;
        if (cm < j) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

struct IntegArgs {
    int64_t n;
    const double *x, *R, *V, *rho;
    const int64_t *nb_off;
    const int32_t *nb_idx;
    const int32_t *nv;
    const double *verts;
    const int32_t *tags;
    const int64_t *row_off;
    const int32_t *col;
    int64_t nnz;
    int G;
    int nreg;
    const double *reg_lo, *reg_hi;
    const int32_t *reg_mat;
    double *blocks;
    double *E;
    const int64_t *bq_off;
    double *bq_y, *bq_w, *bq_N;
    int32_t *bq_face, *bq_nact, *bq_act;
    unsigned long long *counters;
    int amax;       // candidate capacity staged in LDS
    int tile_rows;  // pair rows per Gram tile
    FieldSet fields;
};

// Candidate count per cell (to size LDS).
__global__ void cand_count_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ R,
                                  const double *__restrict__ rho, const int64_t *__restrict__ nb_off,
                                  const int32_t *__restrict__ nb_idx, int32_t *__restrict__ cnt)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double xc0 = x[2 * c], xc1 = x[2 * c + 1], rc = rho[c];
    int k = 1;
    for (int64_t p = nb_off[c]; p < nb_off[c + 1]; ++p) {
        int32_t j = nb_idx[p];
        double d0 = x[2 * (int64_t)j] - xc0, d1 = x[2 * (int64_t)j + 1] - xc1;
        double lim = R[j] + rc;
        if (d0 * d0 + d1 * d1 < lim * lim) k++;
    }
    cnt[c] = k;
}

// Thread 0 of a cell's workgroup: the functions whose support can reach
// cell c (the generator first, then the overlap neighbours within R_j +
// rho_c) into the LDS arrays; A = -1 when more than g.amax.
__device__ void stage_cell2(const IntegArgs &g, int64_t c, double xc0, double xc1, double *sx, double *sR,
                            double *sV, int32_t *sidx, int *sA)
{
    const int amax = g.amax;
    int A = 0;
    double rc = g.rho[c];
    sidx[A] = (int32_t)c; sx[0] = xc0; sx[1] = xc1; sR[0] = g.R[c]; sV[0] = g.V[c]; A = 1;
    for (int64_t p = g.nb_off[c]; p < g.nb_off[c + 1]; ++p) {
        int32_t j = g.nb_idx[p];
        double d0 = g.x[2 * (int64_t)j] - xc0, d1 = g.x[2 * (int64_t)j + 1] - xc1;
        double lim = g.R[j] + rc;
        if (d0 * d0 + d1 * d1 < lim * lim) {
            if (A >= amax) { A = -1; break; }
            sidx[A] = j;
            sx[2 * A] = g.x[2 * (int64_t)j];
            sx[2 * A + 1] = g.x[2 * (int64_t)j + 1];
            sR[A] = g.R[j];
            sV[A] = g.V[j];
            A++;
        }
    }
    if (A < 0) atomicAdd(&g.counters[kOverflow], 1ull);
    *sA = A;
}

template <int ORD, bool FIELDS>
__global__ __launch_bounds__(kThreads) void integrate2d_kernel(IntegArgs g)
{
    extern __shared__ double lds[];
    __shared__ int sA;
    const int G = g.G;
    const int NB = 3 * G + 3;
    const int amax = g.amax;
    double *sx = lds;
    double *sR = sx + 2 * amax;
    double *sV = sR + amax;
    int32_t *sidx = (int32_t *)(sV + amax);
    double *gram = sV + amax + (amax + 1) / 2;   // after the int32 indices
    const int64_t c = blockIdx.x;
    const double xc0 = g.x[2 * c], xc1 = g.x[2 * c + 1];
    const double hs = 0.5 * g.R[c];
    if (threadIdx.x == 0) stage_cell2(g, c, xc0, xc1, sx, sR, sV, sidx, &sA);
    __syncthreads();
    const int A = sA;
    if (A <= 0) return;
    const int nvc = g.nv[c];
    const int nq = nvc * kTriRule;
    const double *cv = g.verts + c * kCellCap2D * 2;
    constexpr int B = Basis2<ORD>::B;

    for (int a0 = 0; a0 < A; a0 += g.tile_rows) {
        const int a1 = min(A, a0 + g.tile_rows);
        const int TR = a1 - a0;
        const int TT = TR * A;
        for (int t = threadIdx.x; t < NB * TT; t += kThreads) gram[t] = 0.0;
        __syncthreads();
        for (int t = threadIdx.x; t < nq; t += kThreads) {
            int k = t / kTriRule, r = t - k * kTriRule;
            int kn = (k + 1 == nvc) ? 0 : k + 1;
            double e10 = cv[2 * k] - xc0, e11 = cv[2 * k + 1] - xc1;
            double e20 = cv[2 * kn] - xc0, e21 = cv[2 * kn + 1] - xc1;
            double detJ = e10 * e21 - e11 * e20;
            if (!(detJ > 0.0)) continue;
            double y0 = xc0 + e10 * c_tri_pts[r][0] + e20 * c_tri_pts[r][1];
            double y1 = xc1 + e11 * c_tri_pts[r][0] + e21 * c_tri_pts[r][1];
            double w = c_tri_w[r] * detJ;
            double C[B], dC0[B], dC1[B];
            uint64_t mask;
            int o = rk_prepare<ORD>(y0, y1, A, sx, sR, sV, hs, C, dC0, dC1, &mask);
            if (o < 0) continue;
            if (a0 == 0 && o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
            int mat = material_at(y0, y1, g.nreg, g.reg_lo, g.reg_hi, g.reg_mat);
            double wf[kMaxMat];
            if (FIELDS) {
                const double yy[2] = {y0, y1};
                material_weights<2>(yy, mat, w, g.fields, wf);
            }
            uint64_t ma = mask & ((a1 >= 64 ? ~0ull : ((1ull << a1) - 1)) & ~((1ull << a0) - 1));
            // the lanes of a wave (neighbouring quadrature points) walk the
            // active columns from different starting columns, so that their
            // LDS atomics rarely meet on one address (they would serialise)
            const int bs = (int)(threadIdx.x & 63) % A;
            const uint64_t below = (1ull << bs) - 1;
            while (ma) {
                int a = __builtin_ctzll(ma);
                ma &= ma - 1;
                double Na, dNa0, dNa1;
                rk_value<ORD>(y0, y1, a, sx, sR, sV, hs, C, dC0, dC1, &Na, &dNa0, &dNa1);
                double wa = w * Na, wa0 = w * dNa0, wa1 = w * dNa1;
                double *gr = gram + (a - a0) * A;
                uint64_t mhi = mask & ~below, mlo = mask & below;   // columns >= bs first, then the rest
                while (mhi | mlo) {
                    uint64_t &mb = mhi ? mhi : mlo;
                    int b = __builtin_ctzll(mb);
                    mb &= mb - 1;
                    double Nb, dNb0, dNb1;
                    rk_value<ORD>(y0, y1, b, sx, sR, sV, hs, C, dC0, dC1, &Nb, &dNb0, &dNb1);
                    if (!FIELDS) {
                        atomicAdd(&gr[(3 * mat + 0) * TT + b], wa * Nb);
                        atomicAdd(&gr[(3 * mat + 1) * TT + b], wa0 * Nb);
                        atomicAdd(&gr[(3 * mat + 2) * TT + b], wa1 * Nb);
                    } else {
#pragma unroll
                        for (int m = 0; m < kMaxMat; ++m) {
                            if (m >= G || wf[m] == 0.0) continue;
                            atomicAdd(&gr[(3 * m + 0) * TT + b], wf[m] * Na * Nb);
                            atomicAdd(&gr[(3 * m + 1) * TT + b], wf[m] * dNa0 * Nb);
                            atomicAdd(&gr[(3 * m + 2) * TT + b], wf[m] * dNa1 * Nb);
                        }
                    }
                    atomicAdd(&gr[(3 * G + 0) * TT + b], wa0 * dNb0);
                    atomicAdd(&gr[(3 * G + 1) * TT + b], wa0 * dNb1);
                    atomicAdd(&gr[(3 * G + 2) * TT + b], wa1 * dNb1);
                }
            }
        }
        __syncthreads();
        // Scatter the tile.  K^yx[a][b] = K^xy[b][a] is added from the tile
        // that holds row b of K^xy, i.e. as the transpose of this tile.
        const int64_t nnz = g.nnz;
        for (int t = threadIdx.x; t < TT; t += kThreads) {
            int al = t / A, b = t - al * A;
            int a = a0 + al;
            bool nz = false;
            for (int q = 0; q < NB; ++q) nz |= (gram[q * TT + t] != 0.0);
            if (!nz) continue;
            int64_t pos = find_col(g.row_off, g.col, sidx[a], sidx[b]);
            if (pos < 0) { atomicAdd(&g.counters[kMissing], 1ull); continue; }
            for (int m = 0; m < G; ++m)
                for (int q = 0; q < 3; ++q) {
                    double v = gram[(3 * m + q) * TT + t];
                    if (v != 0.0) atomicAdd(&g.blocks[(int64_t)(3 * m + q) * nnz + pos], v);
                }
            const int kb = 3 * G;
            atomicAdd(&g.blocks[(int64_t)(kb + 0) * nnz + pos], gram[(3 * G + 0) * TT + t]);
            atomicAdd(&g.blocks[(int64_t)(kb + 1) * nnz + pos], gram[(3 * G + 1) * TT + t]);
            atomicAdd(&g.blocks[(int64_t)(kb + 3) * nnz + pos], gram[(3 * G + 2) * TT + t]);
            // transpose part: K^yx[b][a] += K^xy[a][b]
            int64_t pos_t = find_col(g.row_off, g.col, sidx[b], sidx[a]);
            if (pos_t < 0) { atomicAdd(&g.counters[kMissing], 1ull); continue; }
            atomicAdd(&g.blocks[(int64_t)(kb + 2) * nnz + pos_t], gram[(3 * G + 1) * TT + t]);
        }
        __syncthreads();
    }

    // Boundary edges on domain faces: line rule mapped from [-1, 1] with
    // K = half the edge length (App. A); surface blocks and the boundary
    // point table used for the inflow term.
    int nbe = 0;
    for (int k = 0; k < nvc; ++k) {
        int tg = g.tags[c * kCellCap2D + k];
        if (tg <= -1 && tg >= -4) nbe++;
    }
    const int64_t nnz = g.nnz;
    for (int t = threadIdx.x; t < nbe * kSegRule; t += kThreads) {
        int e = t / kSegRule, q = t - e * kSegRule;
        int k = 0, seen = -1;
        for (k = 0; k < nvc; ++k) {
            int tg = g.tags[c * kCellCap2D + k];
            if (tg <= -1 && tg >= -4) {
                seen++;
                if (seen == e) break;
            }
        }
        int face = -1 - g.tags[c * kCellCap2D + k];
        int kn = (k + 1 == nvc) ? 0 : k + 1;
        double p0 = cv[2 * k], p1 = cv[2 * k + 1], q0 = cv[2 * kn], q1 = cv[2 * kn + 1];
        double s = 0.5 * (c_seg_pts[q] + 1.0);
        double y0 = p0 + (q0 - p0) * s, y1 = p1 + (q1 - p1) * s;
        double len = sqrt((q0 - p0) * (q0 - p0) + (q1 - p1) * (q1 - p1));
        double w = c_seg_w[q] * 0.5 * len;
        int64_t bq = g.bq_off[c] + t;
        g.bq_y[2 * bq] = y0;
        g.bq_y[2 * bq + 1] = y1;
        g.bq_face[bq] = face;
        g.bq_w[bq] = w;
        double C[B], dC0[B], dC1[B];
        uint64_t mask;
        int o = rk_prepare<ORD>(y0, y1, A, sx, sR, sV, hs, C, dC0, dC1, &mask);
        int na = 0;
        if (o >= 0) {
            if (o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
            uint64_t ma = mask;
            while (ma) {
                int a = __builtin_ctzll(ma);
                ma &= ma - 1;
                double Na, d0, d1;
                rk_value<ORD>(y0, y1, a, sx, sR, sV, hs, C, dC0, dC1, &Na, &d0, &d1);
                if (na < kBqAct) {
                    g.bq_act[bq * kBqAct + na] = sidx[a];
                    g.bq_N[bq * kBqAct + na] = Na;
                } else {
                    atomicAdd(&g.counters[kOverflow], 1ull);
                }
                na++;
                uint64_t mb = mask;
                while (mb) {
                    int b = __builtin_ctzll(mb);
                    mb &= mb - 1;
                    double Nb, e0, e1;
                    rk_value<ORD>(y0, y1, b, sx, sR, sV, hs, C, dC0, dC1, &Nb, &e0, &e1);
                    int64_t pos = find_col(g.row_off, g.col, sidx[a], sidx[b]);
                    if (pos < 0) { atomicAdd(&g.counters[kMissing], 1ull); continue; }
                    atomicAdd(&g.blocks[(int64_t)(3 * G + 4 + face) * nnz + pos], w * Na * Nb);
                }
            }
        }
        g.bq_nact[bq] = na < kBqAct ? na : kBqAct;
    }

    // Point values at the generator: E[c, j] = N_j(x_c).
    if (threadIdx.x == 0) {
        double C[B], dC0[B], dC1[B];
        uint64_t mask;
        int o = rk_prepare<ORD>(xc0, xc1, A, sx, sR, sV, hs, C, dC0, dC1, &mask);
        if (o >= 0) {
            if (o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
            uint64_t ma = mask;
            while (ma) {
                int a = __builtin_ctzll(ma);
                ma &= ma - 1;
                double Na, d0, d1;
                rk_value<ORD>(xc0, xc1, a, sx, sR, sV, hs, C, dC0, dC1, &Na, &d0, &d1);
                int64_t pos = find_col(g.row_off, g.col, (int32_t)c, sidx[a]);
                if (pos >= 0) g.E[pos] = Na;
                else atomicAdd(&g.counters[kMissing], 1ull);
            }
        }
    }
}

// ---- 3D integration ---------------------------------------------------------
//
// As in 2D, one workgroup per cell, with the functions that can reach the
// cell staged in LDS.  The cell's faces are fan-triangulated from their
// vertex 0 and joined to the generator, giving the tetrahedra
// (x_c, v_0, v_k, v_k+1) that carry the 8-point conical-product rule.  The
// moment matrix is kept as a packed lower triangle and factored once: the
// leading b x b block of its Cholesky factor is the factor of the moment
// matrix of the lower orders, so the pivots decide the order used (the
// highest whose pivots all exceed 1e-6 of its largest diagonal entry).  The
// gradient correction dC = -M^-1 (dM C) is formed from dM C accumulated
// directly in a second pass over the functions, never from dM itself.

__constant__ double c_tet_pts[kTetRule][3];
__constant__ double c_tet_w[kTetRule];
__constant__ double c_tri3_pts[kTri3Rule][2];
__constant__ double c_tri3_w[kTri3Rule];

template <int ORD>
struct Basis3 {
    static constexpr int B = ORD == 0 ? 1 : (ORD == 1 ? 4 : 10);
};

__host__ __device__ constexpr int bsize3(int o) { return o == 0 ? 1 : (o == 1 ? 4 : 10); }

// Unique monomials of degree <= ORD in z: [1, z0, z1, z2, z0z0, z0z1, z0z2,
// z1z1, z1z2, z2z2] and their derivatives D[g] = dP/dz_g.
template <int ORD>
__device__ __forceinline__ void basis3(const double (&z)[3], double (&P)[Basis3<ORD>::B],
                                       double (&D)[3][Basis3<ORD>::B])
{
    P[0] = 1.0;
#pragma unroll
    for (int g = 0; g < 3; ++g) D[g][0] = 0.0;
    if (ORD >= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P[1 + a] = z[a];
#pragma unroll
            for (int g = 0; g < 3; ++g) D[g][1 + a] = (g == a) ? 1.0 : 0.0;
        }
    }
    if (ORD >= 2) {
        int k = 4;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = a; c < 3; ++c) {
                P[k] = z[a] * z[c];
#pragma unroll
                for (int g = 0; g < 3; ++g) D[g][k] = (g == a ? z[c] : 0.0) + (g == c ? z[a] : 0.0);
                k++;
            }
    }
}

__device__ __forceinline__ constexpr int tri_idx(int r, int s) { return r * (r + 1) / 2 + s; }

// Solve L L^T out = rhs on the leading b x b block of the packed factor.
template <int B>
__device__ __forceinline__ void chol_solve_packed(int b, const double (&L)[B * (B + 1) / 2], const double (&rhs)[B],
                                                  double (&out)[B])
{
    double t[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
        if (k >= b) { t[k] = 0.0; continue; }
        double s = rhs[k];
#pragma unroll
        for (int p = 0; p < B; ++p)
            if (p < k) s -= L[tri_idx(k, p)] * t[p];
        t[k] = s / L[tri_idx(k, k)];
    }
#pragma unroll
    for (int k = B - 1; k >= 0; --k) {
        if (k >= b) { out[k] = 0.0; continue; }
        double s = t[k];
#pragma unroll
        for (int p = 0; p < B; ++p)
            if (p > k && p < b) s -= L[tri_idx(p, k)] * out[p];
        out[k] = s / L[tri_idx(k, k)];
    }
}

// RK correction at y from the staged candidates; returns the order used
// (-1: no function covers y).  C and dC are zero beyond the order's size.
template <int ORD>
__device__ int rk_prepare3(const double (&y)[3], int A, const double *sx, const double *sR, const double *sV,
                           double hs, double (&C)[Basis3<ORD>::B], double (&dC)[3][Basis3<ORD>::B])
{
    constexpr int B = Basis3<ORD>::B;
    constexpr int NP = B * (B + 1) / 2;
    double L[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) L[k] = 0.0;
    bool any = false;
    const double ihs = 1.0 / hs;
    for (int a = 0; a < A; ++a) {
        double r[3] = {y[0] - sx[3 * a], y[1] - sx[3 * a + 1], y[2] - sx[3 * a + 2]};
        double h = 0.5 * sR[a];
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (!(r2 < 4.0 * h * h)) continue;
        double dfac;
        double W = spline(r2, h, &dfac);
        if (W == 0.0) continue;
        any = true;
        double z[3] = {r[0] * ihs, r[1] * ihs, r[2] * ihs};
        double P[B], D[3][B];
        basis3<ORD>(z, P, D);
        double v = sV[a];
#pragma unroll
        for (int p = 0; p < B; ++p)
#pragma unroll
            for (int q = 0; q <= p; ++q) L[tri_idx(p, q)] += v * P[p] * P[q] * W;
    }
    if (!any) return -1;
    double diag[B], piv[B];
#pragma unroll
    for (int k = 0; k < B; ++k) diag[k] = L[tri_idx(k, k)];
    // kfail = number of leading pivots that are positive; past a failed pivot
    // the factor is continued with a unit diagonal and never used
    int kfail = 0;
    bool alive = true;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        double s = L[tri_idx(k, k)];
#pragma unroll
        for (int p = 0; p < B; ++p)
            if (p < k) s -= L[tri_idx(k, p)] * L[tri_idx(k, p)];
        piv[k] = s;
        alive = alive && (s > 0.0);
        kfail += alive ? 1 : 0;
        L[tri_idx(k, k)] = alive ? sqrt(s) : 1.0;
#pragma unroll
        for (int rr = 0; rr < B; ++rr) {
            if (rr <= k) continue;
            double t = L[tri_idx(rr, k)];
#pragma unroll
            for (int p = 0; p < B; ++p)
                if (p < k) t -= L[tri_idx(rr, p)] * L[tri_idx(k, p)];
            L[tri_idx(rr, k)] = t / L[tri_idx(k, k)];
        }
    }
    int o = -1;
#pragma unroll
    for (int oo = ORD; oo >= 0; --oo) {
        if (o >= 0) break;
        const int b = bsize3(oo);
        if (b > kfail) continue;
        double dmax = 0.0;
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (k < b) dmax = fmax(dmax, diag[k]);
        if (!(dmax > 0.0)) continue;
        bool ok = true;
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (k < b) ok = ok && (piv[k] > 1e-6 * dmax);
        if (ok) o = oo;
    }
    if (o < 0) return -1;
    const int b = bsize3(o);
    double e0[B];
#pragma unroll
    for (int k = 0; k < B; ++k) e0[k] = (k == 0) ? 1.0 : 0.0;
    chol_solve_packed<B>(b, L, e0, C);
    // dM_g C = sum_j V_j [ (D_g P^T + P D_g^T) C W / hs + P (P.C) dW_g ]
    double rg[3][B];
#pragma unroll
    for (int g = 0; g < 3; ++g)
#pragma unroll
        for (int k = 0; k < B; ++k) rg[g][k] = 0.0;
    for (int a = 0; a < A; ++a) {
        double r[3] = {y[0] - sx[3 * a], y[1] - sx[3 * a + 1], y[2] - sx[3 * a + 2]};
        double h = 0.5 * sR[a];
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (!(r2 < 4.0 * h * h)) continue;
        double dfac;
        double W = spline(r2, h, &dfac);
        if (W == 0.0) continue;
        double z[3] = {r[0] * ihs, r[1] * ihs, r[2] * ihs};
        double P[B], D[3][B];
        basis3<ORD>(z, P, D);
        double v = sV[a];
        double PC = 0.0;
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (k < b) PC += P[k] * C[k];
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            double DC = 0.0;
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (k < b) DC += D[g][k] * C[k];
            double dW = dfac * r[g];
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (k < b) rg[g][k] += v * ((D[g][k] * PC + P[k] * DC) * ihs * W + P[k] * PC * dW);
        }
    }
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        double t[B];
#pragma unroll
        for (int k = 0; k < B; ++k) t[k] = -rg[g][k];
        chol_solve_packed<B>(b, L, t, dC[g]);
    }
    return o;
}

template <int ORD>
__device__ __forceinline__ bool rk_value3(const double (&y)[3], int a, const double *sx, const double *sR,
                                          const double *sV, double hs, const double (&C)[Basis3<ORD>::B],
                                          const double (&dC)[3][Basis3<ORD>::B], double *N, double (&dN)[3])
{
    constexpr int B = Basis3<ORD>::B;
    double r[3] = {y[0] - sx[3 * a], y[1] - sx[3 * a + 1], y[2] - sx[3 * a + 2]};
    double h = 0.5 * sR[a];
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    if (!(r2 < 4.0 * h * h)) return false;
    double dfac;
    double W = spline(r2, h, &dfac);
    if (W == 0.0) return false;
    const double ihs = 1.0 / hs;
    double z[3] = {r[0] * ihs, r[1] * ihs, r[2] * ihs};
    double P[B], D[3][B];
    basis3<ORD>(z, P, D);
    double PC = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) PC += P[k] * C[k];
    double v = sV[a];
    *N = v * PC * W;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        double t1 = 0.0, t2 = 0.0;
#pragma unroll
        for (int k = 0; k < B; ++k) {
            t1 += D[g][k] * ihs * C[k];
            t2 += P[k] * dC[g][k];
        }
        dN[g] = v * ((t1 + t2) * W + PC * (dfac * r[g]));
    }
    return true;
}

__device__ __forceinline__ int material_at3(const double (&y)[3], int nreg, const double *lo, const double *hi,
                                            const int32_t *mat)
{
    int m = 0;
    for (int r = 0; r < nreg; ++r)
        if (y[0] >= lo[3 * r] && y[0] <= hi[3 * r] && y[1] >= lo[3 * r + 1] && y[1] <= hi[3 * r + 1] &&
            y[2] >= lo[3 * r + 2] && y[2] <= hi[3 * r + 2])
            m = mat[r];
    return m;
}

struct Integ3Args {
    int64_t n;
    const double *x, *R, *V, *rho;
    const int64_t *nb_off;
    const int32_t *nb_idx;
    const int32_t *nf, *fnv, *ftags;
    const double *fverts;
    const int64_t *row_off;
    const int32_t *col;
    int64_t nnz;
    int G;
    int nreg;
    const double *reg_lo, *reg_hi;
    const int32_t *reg_mat;
    double *blocks;
    double *E;
    const int64_t *bq_off;
    double *bq_y, *bq_w, *bq_N;
    int32_t *bq_face, *bq_nact, *bq_act;
    unsigned long long *counters;
    int amax;
    int tile_rows;
    FieldSet fields;
};

__global__ void cand_count3_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ R,
                                   const double *__restrict__ rho, const int64_t *__restrict__ nb_off,
                                   const int32_t *__restrict__ nb_idx, int32_t *__restrict__ cnt)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double rc = rho[c];
    int k = 1;
    for (int64_t p = nb_off[c]; p < nb_off[c + 1]; ++p) {
        int64_t j = nb_idx[p];
        double d0 = x[3 * j] - x[3 * c], d1 = x[3 * j + 1] - x[3 * c + 1], d2 = x[3 * j + 2] - x[3 * c + 2];
        double lim = R[j] + rc;
        if (d0 * d0 + d1 * d1 + d2 * d2 < lim * lim) k++;
    }
    cnt[c] = k;
}

// Thread 0 of a cell's workgroup: the functions whose support can reach
// cell c (the generator first, then the overlap neighbours within R_j + rho_c)
// into the LDS arrays (A = -1 when more than g.amax), and the prefix counts
// of the cell's fan tetrahedra and of its boundary triangles per face.
__device__ void stage_cell3(const Integ3Args &g, int64_t c, const double (&xc)[3], double *sx, double *sR, double *sV,
                            int32_t *sidx, int *sA, int *tet_pre, int *bnd_pre, int *sntet, int *snbt)
{
    const int amax = g.amax;
    const int nfc = g.nf[c];
    int A = 0;
    double rc = g.rho[c];
    sidx[0] = (int32_t)c; sx[0] = xc[0]; sx[1] = xc[1]; sx[2] = xc[2]; sR[0] = g.R[c]; sV[0] = g.V[c];
    A = 1;
    for (int64_t p = g.nb_off[c]; p < g.nb_off[c + 1]; ++p) {
        int64_t j = g.nb_idx[p];
        double d0 = g.x[3 * j] - xc[0], d1 = g.x[3 * j + 1] - xc[1], d2 = g.x[3 * j + 2] - xc[2];
        double lim = g.R[j] + rc;
        if (d0 * d0 + d1 * d1 + d2 * d2 < lim * lim) {
            if (A >= amax) { A = -1; break; }
            sidx[A] = (int32_t)j;
            sx[3 * A] = g.x[3 * j]; sx[3 * A + 1] = g.x[3 * j + 1]; sx[3 * A + 2] = g.x[3 * j + 2];
            sR[A] = g.R[j];
            sV[A] = g.V[j];
            A++;
        }
    }
    if (A < 0) atomicAdd(&g.counters[kOverflow], 1ull);
    *sA = A;
    int nt = 0, nb = 0;
    tet_pre[0] = 0;
    bnd_pre[0] = 0;
    for (int f = 0; f < nfc; ++f) {
        int m = g.fnv[c * kFaceCap3 + f];
        int tg = g.ftags[c * kFaceCap3 + f];
        nt += m - 2;
        if (tg <= -1 && tg >= -6) nb += m - 2;
        tet_pre[f + 1] = nt;
        bnd_pre[f + 1] = nb;
    }
    *sntet = nt;
    *snbt = nb;
}

// The cell's boundary triangles on domain faces (4-point rule): the surface
// blocks and the boundary point table of the inflow term; then the point
// values at the generator, E[c, j] = N_j(x_c).  All threads of the workgroup.
template <int ORD>
__device__ void integ3_boundary(const Integ3Args &g, int64_t c, int A, const double *sx, const double *sR,
                                const double *sV, const int32_t *sidx, const double (&xc)[3], double hs,
                                const double *fvc, int snbt, const int *bnd_pre)
{
    constexpr int B = Basis3<ORD>::B;
    const int G = g.G;
    const int64_t nnz = g.nnz;
    // boundary triangles on domain faces: 4-point rule, surface blocks and
    // the boundary point table used for the inflow term
    const int nbq = snbt * kTri3Rule;
    const int sb = 4 * G + 9;
    for (int t = threadIdx.x; t < nbq; t += blockDim.x) {
        const int tr = t / kTri3Rule, q = t - tr * kTri3Rule;
        int f = 0;
        while (bnd_pre[f + 1] <= tr) f++;
        const int k = 1 + tr - bnd_pre[f];
        const int face = -1 - g.ftags[c * kFaceCap3 + f];
        const double *A0 = fvc + (f * kFaceVerts3) * 3;
        const double *B0 = fvc + (f * kFaceVerts3 + k) * 3;
        const double *C0 = fvc + (f * kFaceVerts3 + k + 1) * 3;
        double g1[3], g2[3], nn[3];
        for (int d = 0; d < 3; ++d) { g1[d] = B0[d] - A0[d]; g2[d] = C0[d] - A0[d]; }
        nn[0] = g1[1] * g2[2] - g1[2] * g2[1];
        nn[1] = g1[2] * g2[0] - g1[0] * g2[2];
        nn[2] = g1[0] * g2[1] - g1[1] * g2[0];
        const double area2 = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
        double y[3];
        for (int d = 0; d < 3; ++d) y[d] = A0[d] + g1[d] * c_tri3_pts[q][0] + g2[d] * c_tri3_pts[q][1];
        const double w = c_tri3_w[q] * area2;
        const int64_t bq = g.bq_off[c] + t;
        for (int d = 0; d < 3; ++d) g.bq_y[3 * bq + d] = y[d];
        g.bq_face[bq] = face;
        g.bq_w[bq] = w;
        double C[B], dC[3][B];
        int o = rk_prepare3<ORD>(y, A, sx, sR, sV, hs, C, dC);
        int na = 0;
        if (o >= 0) {
            if (o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
            for (int a = 0; a < A; ++a) {
                double Na, d_[3];
                if (!rk_value3<ORD>(y, a, sx, sR, sV, hs, C, dC, &Na, d_)) continue;
                if (na < kBqAct3) {
                    g.bq_act[bq * kBqAct3 + na] = sidx[a];
                    g.bq_N[bq * kBqAct3 + na] = Na;
                } else {
                    atomicAdd(&g.counters[kOverflow], 1ull);
                }
                na++;
                for (int b = 0; b < A; ++b) {
                    double Nb, e_[3];
                    if (!rk_value3<ORD>(y, b, sx, sR, sV, hs, C, dC, &Nb, e_)) continue;
                    const int64_t pos = find_col(g.row_off, g.col, sidx[a], sidx[b]);
                    if (pos < 0) { atomicAdd(&g.counters[kMissing], 1ull); continue; }
                    atomicAdd(&g.blocks[(int64_t)(sb + face) * nnz + pos], w * Na * Nb);
                }
            }
        }
        g.bq_nact[bq] = na < kBqAct3 ? na : kBqAct3;
    }

    // point values at the generator: E[c, j] = N_j(x_c)
    if (threadIdx.x == 0) {
        double C[B], dC[3][B];
        int o = rk_prepare3<ORD>(xc, A, sx, sR, sV, hs, C, dC);
        if (o >= 0) {
            if (o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
            for (int a = 0; a < A; ++a) {
                double Na, d_[3];
                if (!rk_value3<ORD>(xc, a, sx, sR, sV, hs, C, dC, &Na, d_)) continue;
                const int64_t pos = find_col(g.row_off, g.col, (int32_t)c, sidx[a]);
                if (pos >= 0) g.E[pos] = Na;
                else atomicAdd(&g.counters[kMissing], 1ull);
            }
        }
    }
}

template <int ORD, bool FIELDS>
__global__ __launch_bounds__(kThreads3) void integrate3d_kernel(Integ3Args g)
{
    extern __shared__ double lds[];
    __shared__ int sA, sntet, snbt;
    __shared__ int tet_pre[kFaceCap3 + 1], bnd_pre[kFaceCap3 + 1];
    const int G = g.G;
    const int NB = 4 * G + 6;
    const int amax = g.amax;
    double *sx = lds;
    double *sR = sx + 3 * amax;
    double *sV = sR + amax;
    int32_t *sidx = (int32_t *)(sV + amax);
    double *gram = sV + amax + (amax + 1) / 2;
    const int64_t c = blockIdx.x;
    const double xc[3] = {g.x[3 * c], g.x[3 * c + 1], g.x[3 * c + 2]};
    const double hs = 0.5 * g.R[c];
    if (threadIdx.x == 0) stage_cell3(g, c, xc, sx, sR, sV, sidx, &sA, tet_pre, bnd_pre, &sntet, &snbt);
    __syncthreads();
    const int A = sA;
    if (A <= 0) return;
    constexpr int B = Basis3<ORD>::B;
    const int nq = sntet * kTetRule;
    const double *fvc = g.fverts + c * kFaceCap3 * kFaceVerts3 * 3;
    const int64_t nnz = g.nnz;

    // The cell's quadrature points are taken blockDim.x at a time, one per
    // thread (a 3D cell has a few hundred, so usually all at once).  Each
    // thread computes its point's RK correction once and keeps it in registers
    // for every tile of Gram rows below; a tile's rows that do not cover the
    // point are skipped by their support test before any other work.
    for (int q0 = 0; q0 < nq; q0 += blockDim.x) {
        const int t = q0 + threadIdx.x;
        bool valid = false;
        double y[3] = {xc[0], xc[1], xc[2]};
        double w = 0.0;
        double C[B], dC[3][B];
        int mat = 0;
        double wf[kMaxMat];
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) C[k2] = dC[0][k2] = dC[1][k2] = dC[2][k2] = 0.0;
#pragma unroll
        for (int m2 = 0; m2 < kMaxMat; ++m2) wf[m2] = 0.0;
        if (t < nq) {
            const int te = t / kTetRule, q = t - te * kTetRule;
            int f = 0;
            while (tet_pre[f + 1] <= te) f++;
            const int k = 1 + te - tet_pre[f];
            const double *v0 = fvc + (f * kFaceVerts3) * 3;
            const double *vk = fvc + (f * kFaceVerts3 + k) * 3;
            const double *vk1 = fvc + (f * kFaceVerts3 + k + 1) * 3;
            double e1[3], e2[3], e3[3], cr[3];
            for (int d = 0; d < 3; ++d) { e1[d] = v0[d] - xc[d]; e2[d] = vk[d] - xc[d]; e3[d] = vk1[d] - xc[d]; }
            cr[0] = e2[1] * e3[2] - e2[2] * e3[1];
            cr[1] = e2[2] * e3[0] - e2[0] * e3[2];
            cr[2] = e2[0] * e3[1] - e2[1] * e3[0];
            const double detJ = e1[0] * cr[0] + e1[1] * cr[1] + e1[2] * cr[2];
            if (detJ > 0.0) {
                for (int d = 0; d < 3; ++d)
                    y[d] = xc[d] + e1[d] * c_tet_pts[q][0] + e2[d] * c_tet_pts[q][1] + e3[d] * c_tet_pts[q][2];
                w = c_tet_w[q] * detJ;
                const int o = rk_prepare3<ORD>(y, A, sx, sR, sV, hs, C, dC);
                if (o >= 0) {
                    valid = true;
                    if (o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
                    mat = material_at3(y, g.nreg, g.reg_lo, g.reg_hi, g.reg_mat);
                    if (FIELDS) material_weights<3>(y, mat, w, g.fields, wf);
                }
            }
        }
        for (int a0 = 0; a0 < A; a0 += g.tile_rows) {
            const int a1 = min(A, a0 + g.tile_rows);
            const int TR = a1 - a0;
            const int TT = TR * A;
            for (int t2 = threadIdx.x; t2 < NB * TT; t2 += blockDim.x) gram[t2] = 0.0;
            __syncthreads();
            if (valid) {
                // the lanes of a wave (neighbouring quadrature points) start the
                // column walk at different columns, so that their LDS atomics
                // never meet on one address (they would serialise)
                const int bstart = (int)(threadIdx.x & 63) % A;
                if constexpr (!FIELDS) {
                    // the tile rows' values at y once (registers), then every
                    // column's values once, added against all active rows
                    constexpr int TRR = kTileRows3;
                    double ta[TRR], td0[TRR], td1[TRR], td2[TRR];
                    unsigned amask = 0;
#pragma unroll
                    for (int al = 0; al < TRR; ++al) {
                        ta[al] = td0[al] = td1[al] = td2[al] = 0.0;
                        double Na, dNa[3];
                        if (a0 + al < a1 && rk_value3<ORD>(y, a0 + al, sx, sR, sV, hs, C, dC, &Na, dNa)) {
                            ta[al] = Na; td0[al] = dNa[0]; td1[al] = dNa[1]; td2[al] = dNa[2];
                            amask |= 1u << al;
                        }
                    }
                    if (amask)
                    for (int bi = 0; bi < A; ++bi) {
                        const int b = bstart + bi < A ? bstart + bi : bstart + bi - A;
                        double Nb, dNb[3];
                        if (!rk_value3<ORD>(y, b, sx, sR, sV, hs, C, dC, &Nb, dNb)) continue;
                        const double wNb = w * Nb, wd0 = w * dNb[0], wd1 = w * dNb[1], wd2 = w * dNb[2];
#pragma unroll
                        for (int al = 0; al < TRR; ++al) {
                            if (!((amask >> al) & 1u)) continue;
                            double *gr = gram + al * A;
                            atomicAdd(&gr[(4 * mat + 0) * TT + b], ta[al] * wNb);
                            atomicAdd(&gr[(4 * mat + 1) * TT + b], td0[al] * wNb);
                            atomicAdd(&gr[(4 * mat + 2) * TT + b], td1[al] * wNb);
                            atomicAdd(&gr[(4 * mat + 3) * TT + b], td2[al] * wNb);
                            atomicAdd(&gr[(4 * G + 0) * TT + b], td0[al] * wd0);
                            atomicAdd(&gr[(4 * G + 1) * TT + b], td0[al] * wd1);
                            atomicAdd(&gr[(4 * G + 2) * TT + b], td0[al] * wd2);
                            atomicAdd(&gr[(4 * G + 3) * TT + b], td1[al] * wd1);
                            atomicAdd(&gr[(4 * G + 4) * TT + b], td1[al] * wd2);
                            atomicAdd(&gr[(4 * G + 5) * TT + b], td2[al] * wd2);
                        }
                    }
                } else {
                    // with material fields (per-material weights per point) the
                    // rows are taken one at a time, each column re-evaluated
                    for (int a = a0; a < a1; ++a) {
                        double Na, dNa[3];
                        if (!rk_value3<ORD>(y, a, sx, sR, sV, hs, C, dC, &Na, dNa)) continue;
                        const double wa0 = w * dNa[0], wa1 = w * dNa[1], wa2 = w * dNa[2];
                        double *gr = gram + (a - a0) * A;
                        for (int bi = 0; bi < A; ++bi) {
                            const int b = bstart + bi < A ? bstart + bi : bstart + bi - A;
                            double Nb, dNb[3];
                            if (!rk_value3<ORD>(y, b, sx, sR, sV, hs, C, dC, &Nb, dNb)) continue;
#pragma unroll
                            for (int m = 0; m < kMaxMat; ++m) {
                                if (m >= G || wf[m] == 0.0) continue;
                                atomicAdd(&gr[(4 * m + 0) * TT + b], wf[m] * Na * Nb);
                                atomicAdd(&gr[(4 * m + 1) * TT + b], wf[m] * dNa[0] * Nb);
                                atomicAdd(&gr[(4 * m + 2) * TT + b], wf[m] * dNa[1] * Nb);
                                atomicAdd(&gr[(4 * m + 3) * TT + b], wf[m] * dNa[2] * Nb);
                            }
                            atomicAdd(&gr[(4 * G + 0) * TT + b], wa0 * dNb[0]);
                            atomicAdd(&gr[(4 * G + 1) * TT + b], wa0 * dNb[1]);
                            atomicAdd(&gr[(4 * G + 2) * TT + b], wa0 * dNb[2]);
                            atomicAdd(&gr[(4 * G + 3) * TT + b], wa1 * dNb[1]);
                            atomicAdd(&gr[(4 * G + 4) * TT + b], wa1 * dNb[2]);
                            atomicAdd(&gr[(4 * G + 5) * TT + b], wa2 * dNb[2]);
                        }
                    }
                }
            }
            __syncthreads();
            // scatter: K^ab for a <= b from the tile, K^ba[j][i] = K^ab[i][j] as its transpose
            const int kb = 4 * G;
            for (int t2 = threadIdx.x; t2 < TT; t2 += blockDim.x) {
                const int t = t2;
                const int al = t / A, b = t - al * A;
                const int a = a0 + al;
                bool nz = false;
                for (int q = 0; q < NB; ++q) nz |= (gram[q * TT + t] != 0.0);
                if (!nz) continue;
                const int64_t pos = find_col(g.row_off, g.col, sidx[a], sidx[b]);
                if (pos < 0) { atomicAdd(&g.counters[kMissing], 1ull); continue; }
                for (int m = 0; m < G; ++m)
                    for (int q = 0; q < 4; ++q) {
                        double v = gram[(4 * m + q) * TT + t];
                        if (v != 0.0) atomicAdd(&g.blocks[(int64_t)(4 * m + q) * nnz + pos], v);
                    }
                // tile order xx, xy, xz, yy, yz, zz -> block kb + 3 alpha + beta
                const int ab[6] = {0, 1, 2, 4, 5, 8};
                for (int q = 0; q < 6; ++q)
                    atomicAdd(&g.blocks[(int64_t)(kb + ab[q]) * nnz + pos], gram[(4 * G + q) * TT + t]);
                const int64_t pos_t = find_col(g.row_off, g.col, sidx[b], sidx[a]);
                if (pos_t < 0) { atomicAdd(&g.counters[kMissing], 1ull); continue; }
                const int ba[3] = {3, 6, 7};          // yx, zx, zy
                const int src[3] = {1, 2, 4};         // from xy, xz, yz
                for (int q = 0; q < 3; ++q)
                    atomicAdd(&g.blocks[(int64_t)(kb + ba[q]) * nnz + pos_t], gram[(4 * G + src[q]) * TT + t]);
            }
            __syncthreads();
        }
    }

    integ3_boundary<ORD>(g, c, A, sx, sR, sV, sidx, xc, hs, fvc, snbt, bnd_pre);
}

// Quadrature points per cell (fan tetrahedra of the cell's faces times the
// rule) and, when outb is given, boundary points per cell (the triangles of
// its faces on the domain boundary times the boundary rule).
__global__ void cell_points3_kernel(int64_t n, const int32_t *__restrict__ nf, const int32_t *__restrict__ fnv,
                                    const int32_t *__restrict__ ftags, int32_t *__restrict__ out,
                                    int32_t *__restrict__ outb)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    int nt = 0, nb = 0;
    for (int f = 0; f < nf[c]; ++f) {
        const int m = fnv[c * kFaceCap3 + f] - 2;
        const int tg = ftags[c * kFaceCap3 + f];
        nt += m;
        if (tg <= -1 && tg >= -6) nb += m;
    }
    out[c] = nt * kTetRule;
    if (outb) outb[c] = nb * kTri3Rule;
}

// ---- 3D, one material without fields: Gram products on the matrix cores ----
//
// The volume blocks of a cell (Sec. 3.2, Alg. 1) are sums over the cell's
// quadrature points q of w_q f_i(y_q) f_j(y_q), where i = 4a + u runs over
// the candidate functions a and the values u of each (N_a, dN_a/dx, dN_a/dy,
// dN_a/dz).  With the panel F[q][i] = sqrt(w_q) f_i(y_q) this is the
// symmetric product G = F^T F: a dense (4A x Q)(Q x 4A) contraction per cell.
// A first kernel writes the panels of a batch of cells (one point per thread,
// its RK correction computed once); a second forms the upper triangle of G in
// 64 x 64 tiles with FP64 MFMA (one tile per wave, accumulators in registers)
// and adds every entry to its CSR block.  The quadrature weights are positive
// (conical product rule, positive Jacobians), so sqrt(w) is real.

struct GramArgs {
    double *F;          // [slots][slot] panels, row stride ipad
    int64_t slot;       // doubles per slot: the volume panel (rows x ipad), the surface panel,
                        // the position table, the row starts
    int64_t soff;       // offset of the surface panel in a slot: [boundary points][amax]
    int64_t toff;       // offset of the position table: int32 [amax][amax], then int64 [amax]
    int ipad;           // row stride: 4 amax rounded up to 64
    int amax;
    int32_t *meta;      // [slots][2]: A, quadrature points (A = 0: nothing to add)
    unsigned *queue;    // one task counter per XCD, 64 bytes apart (zeroed by the panel kernel)
};

// CSR positions of every pair of a cell's candidates, relative to the row
// start (-1: not in the pattern), into tab [amax][amax] (int32), then the row
// starts (int64 [amax]): each candidate's row merged with the candidates in
// global order (the overlap list is ascending; the generator, candidate 0,
// goes in at its place).  All threads of the workgroup.
__device__ void gram_positions(const int64_t *__restrict__ row_off, const int32_t *__restrict__ col,
                               const int32_t *sidx, int A, int64_t c, int amax, double *tab)
{
    int32_t *rel = (int32_t *)tab;
    int64_t *rstart = (int64_t *)(tab + ((int64_t)amax * amax + 1) / 2);
    int lo = 1, hi = A;   // first candidate after the generator in global order
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sidx[mid] < (int32_t)c) lo = mid + 1;
        else hi = mid;
    }
    const int p0 = lo - 1;
    for (int a = threadIdx.x; a < A; a += blockDim.x) {
        const int64_t r0 = row_off[sidx[a]], r1 = row_off[sidx[a] + 1];
        rstart[a] = r0;
        int32_t *ra = rel + (int64_t)a * amax;
        int64_t p = r0;
        for (int k = 0; k < A; ++k) {
            const int b = k < p0 ? k + 1 : (k == p0 ? 0 : k);
            const int32_t j = sidx[b];
            while (p < r1 && col[p] < j) ++p;
            ra[b] = (p < r1 && col[p] == j) ? (int32_t)(p - r0) : -1;
        }
    }
}

// Boundary terms of a cell for the panel kernel (the same quantities as
// integ3_boundary).  Every boundary point (one per thread) writes its row of
// the boundary table and its weighted values sqrt(w) N_a into the surface
// panel Sp; then, for each of the cell's faces on the domain boundary, the
// workgroup forms the face's sums over its points for every pair of functions
// nonzero there, and adds each sum to the face's surface block at (a, b) and
// (b, a) -- one CSR lookup per pair and face rather than per pair and point.
// The point values at the generator are spread over the candidates.
template <int ORD>
__device__ void integ3_boundary_panel(const Integ3Args &g, int64_t c, int A, const double *sx, const double *sR,
                                      const double *sV, const int32_t *sidx, const double (&xc)[3], double hs,
                                      const double *fvc, int snbt, const int *bnd_pre, double *Sp, int ss,
                                      int32_t *sflag, int32_t *slist)
{
    constexpr int B = Basis3<ORD>::B;
    __shared__ double sC[4 * B];
    __shared__ int s_o, s_m;
    const int64_t nnz = g.nnz;
    const int nbq = snbt * kTri3Rule;
    const int sb = 4 * g.G + 9;
    for (int t = threadIdx.x; t < nbq; t += blockDim.x) {
        const int tr = t / kTri3Rule, q = t - tr * kTri3Rule;
        int f = 0;
        while (bnd_pre[f + 1] <= tr) f++;
        const int k = 1 + tr - bnd_pre[f];
        const int face = -1 - g.ftags[c * kFaceCap3 + f];
        const double *A0 = fvc + (f * kFaceVerts3) * 3;
        const double *B0 = fvc + (f * kFaceVerts3 + k) * 3;
        const double *C0 = fvc + (f * kFaceVerts3 + k + 1) * 3;
        double g1[3], g2[3], nn[3];
        for (int d = 0; d < 3; ++d) { g1[d] = B0[d] - A0[d]; g2[d] = C0[d] - A0[d]; }
        nn[0] = g1[1] * g2[2] - g1[2] * g2[1];
        nn[1] = g1[2] * g2[0] - g1[0] * g2[2];
        nn[2] = g1[0] * g2[1] - g1[1] * g2[0];
        const double area2 = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
        double y[3];
        for (int d = 0; d < 3; ++d) y[d] = A0[d] + g1[d] * c_tri3_pts[q][0] + g2[d] * c_tri3_pts[q][1];
        const double w = c_tri3_w[q] * area2;
        const int64_t bq = g.bq_off[c] + t;
        for (int d = 0; d < 3; ++d) g.bq_y[3 * bq + d] = y[d];
        g.bq_face[bq] = face;
        g.bq_w[bq] = w;
        double C[B], dC[3][B];
        const int o = rk_prepare3<ORD>(y, A, sx, sR, sV, hs, C, dC);
        const double sw = w > 0.0 ? sqrt(w) : 0.0;
        double *srow = Sp + (int64_t)t * ss;
        int na = 0;
        if (o >= 0 && o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
        for (int a = 0; a < A; ++a) {
            double Na, d_[3];
            if (o < 0 || !rk_value3<ORD>(y, a, sx, sR, sV, hs, C, dC, &Na, d_)) {
                srow[a] = 0.0;
                continue;
            }
            if (na < kBqAct3) {
                g.bq_act[bq * kBqAct3 + na] = sidx[a];
                g.bq_N[bq * kBqAct3 + na] = Na;
            } else {
                atomicAdd(&g.counters[kOverflow], 1ull);
            }
            na++;
            srow[a] = sw * Na;
        }
        g.bq_nact[bq] = na < kBqAct3 ? na : kBqAct3;
    }
    if (threadIdx.x == 0) {
        double C[B], dC[3][B];
        const int o = rk_prepare3<ORD>(xc, A, sx, sR, sV, hs, C, dC);
        if (o >= 0 && o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
        s_o = o;
        for (int k2 = 0; k2 < B; ++k2) {
            sC[k2] = C[k2];
            sC[B + k2] = dC[0][k2];
            sC[2 * B + k2] = dC[1][k2];
            sC[3 * B + k2] = dC[2][k2];
        }
    }
    __syncthreads();   // the surface panel rows and the generator's correction
    // point values at the generator: E[c, j] = N_j(x_c)
    if (s_o >= 0) {
        double C[B], dC[3][B];
        for (int k2 = 0; k2 < B; ++k2) {
            C[k2] = sC[k2];
            dC[0][k2] = sC[B + k2];
            dC[1][k2] = sC[2 * B + k2];
            dC[2][k2] = sC[3 * B + k2];
        }
        for (int a = threadIdx.x; a < A; a += blockDim.x) {
            double Na, d_[3];
            if (!rk_value3<ORD>(xc, a, sx, sR, sV, hs, C, dC, &Na, d_)) continue;
            const int64_t pos = find_col(g.row_off, g.col, (int32_t)c, sidx[a]);
            if (pos >= 0) g.E[pos] = Na;
            else atomicAdd(&g.counters[kMissing], 1ull);
        }
    }
    const int nfc = g.nf[c];
    for (int f = 0; f < nfc; ++f) {
        if (bnd_pre[f + 1] == bnd_pre[f]) continue;   // not on the domain boundary
        const int q0 = kTri3Rule * bnd_pre[f], q1 = kTri3Rule * bnd_pre[f + 1];
        const int face = -1 - g.ftags[c * kFaceCap3 + f];
        double *blk = g.blocks + (int64_t)(sb + face) * nnz;
        for (int a = threadIdx.x; a < A; a += blockDim.x) {
            bool nz = false;
            for (int qq = q0; qq < q1; ++qq) nz = nz || Sp[(int64_t)qq * ss + a] != 0.0;
            sflag[a] = nz ? 1 : 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int m = 0;
            for (int a = 0; a < A; ++a)
                if (sflag[a]) slist[m++] = a;
            s_m = m;
        }
        __syncthreads();
        const int m = s_m;
        for (int p = threadIdx.x; p < m * m; p += blockDim.x) {
            const int i = p / m, j = p - i * m;
            if (j < i) continue;
            const int a = slist[i], b = slist[j];
            double sum = 0.0;
            for (int qq = q0; qq < q1; ++qq) sum += Sp[(int64_t)qq * ss + a] * Sp[(int64_t)qq * ss + b];
            if (sum == 0.0) continue;
            const int64_t pab = find_col(g.row_off, g.col, sidx[a], sidx[b]);
            if (pab < 0) atomicAdd(&g.counters[kMissing], 1ull);
            else atomicAdd(&blk[pab], sum);
            if (a == b) continue;
            const int64_t pba = find_col(g.row_off, g.col, sidx[b], sidx[a]);
            if (pba < 0) atomicAdd(&g.counters[kMissing], 1ull);
            else atomicAdd(&blk[pba], sum);
        }
        __syncthreads();   // the flags and the list are reused by the next face
    }
}


// Panels of cells c0 + blockIdx.x: row q (q < nq rounded up to 4) holds
// sqrt(w_q) (N_a, dN_a) for the candidates a < A at columns 4a..4a+3 and zeros
// up to the last 64-column tile; rows past nq are zero.  Then the cell's
// boundary terms and point values (integ3_boundary_panel).
template <int ORD>
__global__ __launch_bounds__(kThreads3) void integrate3d_panels_kernel(Integ3Args g, GramArgs q, int64_t c0)
{
    extern __shared__ double lds[];
    __shared__ int sA, sntet, snbt;
    __shared__ int tet_pre[kFaceCap3 + 1], bnd_pre[kFaceCap3 + 1];
    constexpr int B = Basis3<ORD>::B;
    const int amax = g.amax;
    double *sx = lds;
    double *sR = sx + 3 * amax;
    double *sV = sR + amax;
    int32_t *sidx = (int32_t *)(sV + amax);
    int32_t *sflag = sidx + amax;
    int32_t *slist = sflag + amax;
    const int slot = blockIdx.x;
    const int64_t c = c0 + slot;
    const double xc[3] = {g.x[3 * c], g.x[3 * c + 1], g.x[3 * c + 2]};
    const double hs = 0.5 * g.R[c];
    if (threadIdx.x == 0) stage_cell3(g, c, xc, sx, sR, sV, sidx, &sA, tet_pre, bnd_pre, &sntet, &snbt);
    __syncthreads();
    const int A = sA;
    int32_t *meta = q.meta + 2 * (int64_t)slot;
    // the product kernel's task counters start at zero for every batch
    if (blockIdx.x == 0 && threadIdx.x < 8) q.queue[16 * threadIdx.x] = 0u;
    if (A <= 0) {
        if (threadIdx.x == 0) { meta[0] = 0; meta[1] = 0; }
        return;
    }
    const int nq = sntet * kTetRule;
    const int nq4 = (nq + 3) & ~3;
    const int width = ((4 * A + 63) >> 6) << 6;
    if (threadIdx.x == 0) { meta[0] = A; meta[1] = nq; }
    const double *fvc = g.fverts + c * kFaceCap3 * kFaceVerts3 * 3;
    double *Fs = q.F + (int64_t)slot * q.slot;
    gram_positions(g.row_off, g.col, sidx, A, c, amax, Fs + q.toff);
    for (int t = threadIdx.x; t < nq4; t += blockDim.x) {
        double y[3] = {xc[0], xc[1], xc[2]};
        double w = 0.0;
        double C[B], dC[3][B];
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) C[k2] = dC[0][k2] = dC[1][k2] = dC[2][k2] = 0.0;
        if (t < nq) {
            const int te = t / kTetRule, qq = t - te * kTetRule;
            int f = 0;
            while (tet_pre[f + 1] <= te) f++;
            const int k = 1 + te - tet_pre[f];
            const double *v0 = fvc + (f * kFaceVerts3) * 3;
            const double *vk = fvc + (f * kFaceVerts3 + k) * 3;
            const double *vk1 = fvc + (f * kFaceVerts3 + k + 1) * 3;
            double e1[3], e2[3], e3[3], cr[3];
            for (int d = 0; d < 3; ++d) { e1[d] = v0[d] - xc[d]; e2[d] = vk[d] - xc[d]; e3[d] = vk1[d] - xc[d]; }
            cr[0] = e2[1] * e3[2] - e2[2] * e3[1];
            cr[1] = e2[2] * e3[0] - e2[0] * e3[2];
            cr[2] = e2[0] * e3[1] - e2[1] * e3[0];
            const double detJ = e1[0] * cr[0] + e1[1] * cr[1] + e1[2] * cr[2];
            if (detJ > 0.0) {
                for (int d = 0; d < 3; ++d)
                    y[d] = xc[d] + e1[d] * c_tet_pts[qq][0] + e2[d] * c_tet_pts[qq][1] + e3[d] * c_tet_pts[qq][2];
                w = c_tet_w[qq] * detJ;
                const int o = rk_prepare3<ORD>(y, A, sx, sR, sV, hs, C, dC);
                if (o < 0) w = 0.0;
                else if (o < ORD) atomicAdd(&g.counters[kFallbacks], 1ull);
            }
        }
        const double sw = w > 0.0 ? sqrt(w) : 0.0;
        double *row = Fs + (int64_t)t * q.ipad;
        for (int a = 0; a < A; ++a) {
            double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
            double Na, dNa[3];
            if (sw > 0.0 && rk_value3<ORD>(y, a, sx, sR, sV, hs, C, dC, &Na, dNa)) {
                v0 = sw * Na; v1 = sw * dNa[0]; v2 = sw * dNa[1]; v3 = sw * dNa[2];
            }
            double2 *o = (double2 *)(row + 4 * a);
            o[0] = make_double2(v0, v1);
            o[1] = make_double2(v2, v3);
        }
        for (int i = 4 * A; i < width; i += 2) *(double2 *)(row + i) = make_double2(0.0, 0.0);
    }
    integ3_boundary_panel<ORD>(g, c, A, sx, sR, sV, sidx, xc, hs, fvc, snbt, bnd_pre, Fs + q.soff, amax, sflag,
                               slist);
}

typedef double gram_acc_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t shfl64(int64_t v, int src)
{
    const int lo = __shfl((int)(uint32_t)(uint64_t)v, src);
    const int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Block index of the entry (value u of row function, value v of column
// function) at the row's CSR position (one material): 0 for N N, u for
// dN_u N, and 1 + DIM + DIM (u-1) + (v-1) for dN_u dN_v (u, v = 1..DIM for
// x, y, z).
template <int DIM>
__device__ __forceinline__ int gram_block(int u, int v)
{
    return v == 0 ? u : 1 + DIM + DIM * (u - 1) + (v - 1);
}

// One 64 x 64 tile (I, J), I <= J, of a cell's G: 16 x 16 candidate pairs.
// MFMA 16x16x4 (FP64): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] of
// the operands and D[l / 16 + 4 r][l % 16] in accumulator register r.
template <bool DIAG>
__device__ __forceinline__ void gram_tile(const double *__restrict__ Fs, int ipad, int nk, int I, int J, int lane,
                                          gram_acc_t (&acc)[4][4])
{
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = gram_acc_t{0.0, 0.0, 0.0, 0.0};
    const double *pa = Fs + (int64_t)(lane >> 4) * ipad + I * 64 + (lane & 15);
    const double *pb = Fs + (int64_t)(lane >> 4) * ipad + J * 64 + (lane & 15);
    const int64_t step = 4 * (int64_t)ipad;
    double av[4], bv[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        av[bi] = pa[bi * 16];
        bv[bi] = DIAG ? 0.0 : pb[bi * 16];
    }
    for (int ks = 0; ks < nk; ++ks) {
        double an[4], bn[4];
        const bool more = ks + 1 < nk;
        pa += step;
        pb += step;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
            an[bi] = more ? pa[bi * 16] : 0.0;
            bn[bi] = (!DIAG && more) ? pb[bi * 16] : 0.0;
        }
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                if (DIAG && bi > bj) continue;   // wholly below the diagonal
                acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], DIAG ? av[bj] : bv[bj], acc[bi][bj],
                                                                  0, 0, 0);
            }
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
            av[bi] = an[bi];
            bv[bi] = bn[bi];
        }
    }
}

// Persistent workgroups, each serving the task queue of the XCD it runs on
// (workgroups are dealt round-robin over the 8 XCDs): queue x holds the tiles
// of the batch's slots x, x + 8, ..., slot by slot, so that the waves of one
// XCD work on few cells at a time and find their panels in its L2.  A wave
// takes the next tile (I, J), I <= J, reads the CSR positions of its 256
// candidate pairs both ways from the slot's table (8 per lane, kept in
// registers), forms the tile, and adds each entry of the upper triangle to its
// block (twice when the mirrored entry belongs to another block or position).
// Every wave leaves once its queue is drained.
template <int DIM>
__device__ __forceinline__ void gram_products(const GramArgs &q, double *blocks, int64_t nnz,
                                              unsigned long long *counters, int nslot, int ntmax)
{
    const int x = blockIdx.x & 7;
    const int lane = threadIdx.x & 63;
    const int nsx = nslot > x ? (nslot - x + 7) / 8 : 0;
    const unsigned total = (unsigned)nsx * (unsigned)ntmax;
    const int amax = q.amax;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(&q.queue[16 * x], 1u);
        t = (unsigned)__shfl((int)t, 0);
        if (t >= total) break;
        const int slot = x + 8 * (int)(t / (unsigned)ntmax);
        int rt = (int)(t % (unsigned)ntmax);
        const int A = q.meta[2 * slot], nq = q.meta[2 * slot + 1];
        if (A <= 0 || nq <= 0) continue;
        const int T = (4 * A + 63) >> 6;
        if (rt >= T * (T + 1) / 2) continue;
        int I = 0;
        while (rt >= T - I) { rt -= T - I; ++I; }
        const int J = I + rt;
        const int nk = (nq + 3) >> 2;
        const double *Fs = q.F + (int64_t)slot * q.slot;
        const int32_t *rel = (const int32_t *)(Fs + q.toff);
        const int64_t *rstart = (const int64_t *)(Fs + q.toff + ((int64_t)amax * amax + 1) / 2);
        // pair p = 16 a' + b' (a = 16 I + a', b = 16 J + b'): entries 0..255
        // are pos(a, b), 256..511 pos(b, a); lane l holds entries l + 64 s
        int64_t pos[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int p = (lane + 64 * s) & 255;
            const int a = 16 * I + (p >> 4), b = 16 * J + (p & 15);
            pos[s] = -1;
            if (a < A && b < A) {
                const int ra = s < 4 ? a : b, rb = s < 4 ? b : a;
                const int32_t o = rel[(int64_t)ra * amax + rb];
                if (o >= 0) pos[s] = rstart[ra] + o;
            }
        }
        gram_acc_t acc[4][4];
        if (I == J) gram_tile<true>(Fs, q.ipad, nk, I, J, lane, acc);
        else gram_tile<false>(Fs, q.ipad, nk, I, J, lane, acc);
        // lane l holds value u = l / 16 of row function a = 16 I + 4 bi + r and
        // value v = l % 4 of column function b = 16 J + 4 bj + (l % 16) / 4;
        // pair entry 16 (4 bi + r) + b' sits in pos[bi] (pos[4 + bi]) of lane
        // 16 r + b'
        const int u = lane >> 4, v = lane & 3, c4 = (lane & 15) >> 2;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                if (I == J && bi > bj) continue;   // uniform: wholly below the diagonal
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int src = 16 * r + 4 * bj + c4;
                    const int64_t pab = shfl64(pos[bi], src), pba = shfl64(pos[4 + bi], src);
                    const int a = 16 * I + 4 * bi + r, b = 16 * J + 4 * bj + c4;
                    if (a >= A || b >= A) continue;
                    const double val = acc[bi][bj][r];
                    if (val == 0.0) continue;
                    const int i = 4 * a + u, j = 4 * b + v;
                    if (i > j) continue;   // the mirror entry (in this tile when I == J) adds it
                    const bool fwd = i == j || u >= 1 || v == 0;
                    const bool bwd = i != j && (v >= 1 || u == 0);
                    if (fwd) {
                        if (pab < 0) atomicAdd(&counters[kMissing], 1ull);
                        else atomicAdd(&blocks[(int64_t)gram_block<DIM>(u, v) * nnz + pab], val);
                    }
                    if (bwd) {
                        if (pba < 0) atomicAdd(&counters[kMissing], 1ull);
                        else atomicAdd(&blocks[(int64_t)gram_block<DIM>(v, u) * nnz + pba], val);
                    }
                }
            }
    }
}

__global__ __launch_bounds__(256, 2) void gram3_kernel(GramArgs q, double *blocks, int64_t nnz,
                                                       unsigned long long *counters, int nslot, int ntmax)
{
    gram_products<3>(q, blocks, nnz, counters, nslot, ntmax);
}

hipError_t upload_rules3(hipStream_t s)
{
    const Rules &r = rules();
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tet_pts), r.tet_pts, sizeof(r.tet_pts), 0,
                                          hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tet_w), r.tet_w, sizeof(r.tet_w), 0, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tri3_pts), r.tri3_pts, sizeof(r.tri3_pts), 0,
                                   hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tri3_w), r.tri3_w, sizeof(r.tri3_w), 0, hipMemcpyHostToDevice, s);
    return e;
}

}  // namespace

template <int ORD, class Args>
hipError_t launch_integ(void (*plain)(Args), void (*fields)(Args), bool use_fields, dim3 grid, size_t shmem,
                        const Args &g, hipStream_t s, int threads = kThreads)
{
    void (*k)(Args) = use_fields ? fields : plain;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    k<<<grid, threads, shmem, s>>>(g);
    return hipGetLastError();
}

static FieldSet field_set(const Problem &P)
{
    FieldSet F;
    F.n = P.n_fields;
    F.nshell = P.n_shells;
    for (int r = 0; r < kMaxFields; ++r) {
        for (int q = 0; q < 4; ++q) F.par[r][q] = P.field_par[r][q];
        F.mat[r] = P.field_mat[r];
        for (int q = 0; q < 5; ++q) F.shell[r][q] = P.shell_par[r][q];
        F.shell_mat[r] = P.shell_mat[r];
    }
    return F;
}

// The Gram panel region of the integration workspace carved for a batch of
// cells: per slot the volume panel (quadrature points rounded up to 4 rows of
// 4 amax values rounded up to 64), the surface panel [boundary points][amax],
// the position table; then the slots' metadata and the product kernel's
// queue counters.  *nb = cells per batch (0: not even one slot fits).
static hipError_t gram_layout(Problem &P, int amax, int nqmax, int nbqmax, GramArgs *q, int64_t *nb)
{
    const int ipad = ((4 * amax + 63) / 64) * 64;
    const int64_t rows = (nqmax + 3) & ~3;
    const int64_t soff = rows * ipad;
    const int64_t toff = soff + (int64_t)nbqmax * amax;
    const size_t panel = sizeof(double) * ((size_t)toff + ((size_t)amax * amax + 1) / 2 + (size_t)amax);
    const size_t per = panel + 2 * sizeof(int32_t);
    const size_t region = P.gram_ws.count;
    *nb = region > 2048 ? std::min<int64_t>(P.n, (int64_t)((region - 2048) / per)) : 0;
    if (*nb < 1) return hipSuccess;
    char *base = P.gram_ws.p;
    q->F = (double *)base;
    q->slot = (int64_t)(panel / sizeof(double));
    q->soff = soff;
    q->toff = toff;
    q->ipad = ipad;
    q->amax = amax;
    const size_t moff = (panel * *nb + 255) & ~(size_t)255;
    q->meta = (int32_t *)(base + moff);
    q->queue = (unsigned *)(base + ((moff + 2 * sizeof(int32_t) * *nb + 255) & ~(size_t)255));
    return hipSuccess;
}

hipError_t launch_integrate2d(Problem &P, hipStream_t s)
{
    // Candidate capacity from the largest candidate set.
    hipError_t e;
    cand_count_kernel<<<(int)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.x.p, P.R.p, P.rho.p, P.nb_off.p, P.nb_idx.p,
                                                                 P.tmp_cand.p);
    std::vector<int32_t> h(P.n);
    e = hipMemcpyAsync(h.data(), P.tmp_cand.p, sizeof(int32_t) * P.n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    int amax = 1;
    for (int32_t v : h) amax = v > amax ? v : amax;
    P.cand_max = amax;
    if (amax > kCandMax2D) return hipErrorInvalidValue;   // reported as capacity by the caller

    int dev = 0;
    int lds_max = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
    const int NB = 3 * P.n_mat + 3;
    size_t fixed = sizeof(double) * (4 * amax + (amax + 1) / 2) + 64;
    size_t budget = (lds_max > 0 ? (size_t)lds_max : 65536) - fixed;
    int tile_rows = (int)(budget / (sizeof(double) * NB * amax));
    if (tile_rows > amax) tile_rows = amax;
    if (tile_rows < 1) return hipErrorInvalidValue;
    size_t shmem = fixed + sizeof(double) * (size_t)NB * tile_rows * amax;

    IntegArgs g;
    g.n = P.n; g.x = P.x.p; g.R = P.R.p; g.V = P.V.p; g.rho = P.rho.p;
    g.nb_off = P.nb_off.p; g.nb_idx = P.nb_idx.p; g.nv = P.nv.p; g.verts = P.verts.p; g.tags = P.tags.p;
    g.row_off = P.row_off.p; g.col = P.col.p; g.nnz = P.nnz; g.G = P.n_mat; g.nreg = P.n_regions;
    g.reg_lo = P.reg_lo.p; g.reg_hi = P.reg_hi.p; g.reg_mat = P.reg_mat.p; g.blocks = P.blocks.p; g.E = P.E.p;
    g.bq_off = P.bq_off.p; g.bq_y = P.bq_y.p; g.bq_w = P.bq_w.p; g.bq_N = P.bq_N.p; g.bq_face = P.bq_face.p;
    g.bq_nact = P.bq_nact.p; g.bq_act = P.bq_act.p; g.counters = P.counters.p; g.amax = amax;
    g.tile_rows = tile_rows;
    g.fields = field_set(P);
    if ((e = upload_rules(s)) != hipSuccess) return e;
    dim3 grid((unsigned)P.n);
    switch (P.rk_order) {
    case 0:
        e = launch_integ<0>(integrate2d_kernel<0, false>, integrate2d_kernel<0, true>, P.n_fields > 0 || P.n_shells > 0, grid, shmem, g, s);
        if (e != hipSuccess) return e;
        break;
    case 1:
        e = launch_integ<1>(integrate2d_kernel<1, false>, integrate2d_kernel<1, true>, P.n_fields > 0 || P.n_shells > 0, grid, shmem, g, s);
        if (e != hipSuccess) return e;
        break;
    default:
        e = launch_integ<2>(integrate2d_kernel<2, false>, integrate2d_kernel<2, true>, P.n_fields > 0 || P.n_shells > 0, grid, shmem, g, s);
        if (e != hipSuccess) return e;
        break;
    }
    return hipGetLastError();
}

hipError_t launch_integrate3d(Problem &P, hipStream_t s)
{
    hipError_t e;
    cand_count3_kernel<<<(int)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.x.p, P.R.p, P.rho.p, P.nb_off.p, P.nb_idx.p,
                                                                  P.tmp_cand.p);
    std::vector<int32_t> h(P.n);
    e = hipMemcpyAsync(h.data(), P.tmp_cand.p, sizeof(int32_t) * P.n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    int amax = 1;
    for (int32_t v : h) amax = v > amax ? v : amax;
    P.cand_max = amax;
    if (amax > kCandMax3D) return hipErrorInvalidValue;   // reported as capacity by the caller

    int dev = 0;
    int lds_max = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
    const int NB = 4 * P.n_mat + 6;
    size_t fixed = sizeof(double) * (5 * amax + (amax + 1) / 2) + 64 + 2 * sizeof(int) * (kFaceCap3 + 1) + 16;
    size_t budget = (lds_max > 0 ? (size_t)lds_max : 65536) - fixed;
    int tile_rows = (int)(budget / (sizeof(double) * NB * amax));
    if (tile_rows > amax) tile_rows = amax;
    // without material fields the rows' values live in registers
    if (!(P.n_fields > 0 || P.n_shells > 0) && tile_rows > kTileRows3) tile_rows = kTileRows3;
    if (tile_rows < 1) return hipErrorInvalidValue;
    size_t shmem = sizeof(double) * (5 * amax + (amax + 1) / 2) + sizeof(double) * (size_t)NB * tile_rows * amax;

    Integ3Args g;
    g.n = P.n; g.x = P.x.p; g.R = P.R.p; g.V = P.V.p; g.rho = P.rho.p;
    g.nb_off = P.nb_off.p; g.nb_idx = P.nb_idx.p; g.nf = P.nf.p; g.fnv = P.fnv.p; g.ftags = P.ftags.p;
    g.fverts = P.fverts.p; g.row_off = P.row_off.p; g.col = P.col.p; g.nnz = P.nnz; g.G = P.n_mat;
    g.nreg = P.n_regions; g.reg_lo = P.reg_lo.p; g.reg_hi = P.reg_hi.p; g.reg_mat = P.reg_mat.p;
    g.blocks = P.blocks.p; g.E = P.E.p; g.bq_off = P.bq_off.p; g.bq_y = P.bq_y.p; g.bq_w = P.bq_w.p;
    g.bq_N = P.bq_N.p; g.bq_face = P.bq_face.p; g.bq_nact = P.bq_nact.p; g.bq_act = P.bq_act.p;
    g.counters = P.counters.p; g.amax = amax; g.tile_rows = tile_rows;
    g.fields = field_set(P);
    if ((e = upload_rules(s)) != hipSuccess) return e;
    dim3 grid((unsigned)P.n);
    if (P.n_mat == 1 && !(P.n_fields > 0 || P.n_shells > 0)) {
        // one material without fields: panels of as many cells as the
        // workspace region holds, then their Gram products on the matrix cores
        // (the atomic kernel below when not even one panel fits)
        int32_t *nbq_cell = (int32_t *)P.tmp_scnt.p;   // free until the surface counts after integration
        cell_points3_kernel<<<(unsigned)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.nf.p, P.fnv.p, P.ftags.p,
                                                                          P.tmp_cand.p, nbq_cell);
        std::vector<int32_t> hb(P.n);
        e = hipMemcpyAsync(h.data(), P.tmp_cand.p, sizeof(int32_t) * P.n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hb.data(), nbq_cell, sizeof(int32_t) * P.n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        int nqmax = 1, nbqmax = 0;
        for (int32_t v : h) nqmax = v > nqmax ? v : nqmax;
        for (int32_t v : hb) nbqmax = v > nbqmax ? v : nbqmax;
        GramArgs q;
        int64_t nb = 0;
        if ((e = gram_layout(P, amax, nqmax, nbqmax, &q, &nb)) != hipSuccess) return e;
        if (nb >= 1) {
            int ncu = 0;
            if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
            const int tmax = q.ipad / 64;
            const int ntmax = tmax * (tmax + 1) / 2;
            const unsigned gblocks = (unsigned)(((std::max(ncu, 8) * 2) + 7) / 8 * 8);
            const size_t cand = sizeof(double) * (5 * amax + (amax + 1) / 2) + 2 * sizeof(int32_t) * amax;
            void (*kp)(Integ3Args, GramArgs, int64_t) =
                P.rk_order == 0 ? integrate3d_panels_kernel<0>
                                : (P.rk_order == 1 ? integrate3d_panels_kernel<1> : integrate3d_panels_kernel<2>);
            for (int64_t c0 = 0; c0 < P.n; c0 += nb) {
                const int64_t nc = std::min<int64_t>(nb, P.n - c0);
                kp<<<(unsigned)nc, kThreads3, cand, s>>>(g, q, c0);
                gram3_kernel<<<gblocks, 256, 0, s>>>(q, g.blocks, g.nnz, g.counters, (int)nc, ntmax);
            }
            return hipGetLastError();
        }
    }
    switch (P.rk_order) {
    case 0:
        e = launch_integ<0>(integrate3d_kernel<0, false>, integrate3d_kernel<0, true>, P.n_fields > 0 || P.n_shells > 0, grid, shmem, g, s, kThreads3);
        if (e != hipSuccess) return e;
        break;
    case 1:
        e = launch_integ<1>(integrate3d_kernel<1, false>, integrate3d_kernel<1, true>, P.n_fields > 0 || P.n_shells > 0, grid, shmem, g, s, kThreads3);
        if (e != hipSuccess) return e;
        break;
    default:
        e = launch_integ<2>(integrate3d_kernel<2, false>, integrate3d_kernel<2, true>, P.n_fields > 0 || P.n_shells > 0, grid, shmem, g, s, kThreads3);
        if (e != hipSuccess) return e;
        break;
    }
    return hipGetLastError();
}

}  // namespace mlpg
