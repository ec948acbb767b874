// Geometry kernels: overlap connectivity (Sec. 3.4), Voronoi-like cells in
// 2D (Sec. 3.1, Fig. 1) and the sparse pattern of the bilinear forms.
#include "internal.hpp"

namespace mlpg {

namespace {

constexpr int kTile = 256;

// |x_i - x_j| <= R_i + R_j in plain IEEE double with no contraction, so that
// every implementation of the same definition draws the same lists.
__device__ __forceinline__ bool overlap_test(int dim, const double *xi, const double *xj, double ri, double rj)
{
#pragma clang fp contract(off)
    double d2 = 0.0;
    for (int a = 0; a < dim; ++a) {
        double t = xj[a] - xi[a];
        d2 = d2 + t * t;
    }
    double s = ri + rj;
    return d2 <= s * s;
}

// One thread per point i, all j streamed through LDS tiles.  mode 0 counts,
// mode 1 writes the list in increasing j.
template <int MODE>
__global__ __launch_bounds__(kTile) void neighbors_kernel(int dim, int64_t n, const double *__restrict__ x,
                                                          const double *__restrict__ R, int64_t *__restrict__ counts,
                                                          const int64_t *__restrict__ off, int32_t *__restrict__ idx)
{
    __shared__ double tx[kTile * 3];
    __shared__ double tr[kTile];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double xi[3] = {0, 0, 0}, ri = 0.0;
    if (i < n) {
        for (int a = 0; a < dim; ++a) xi[a] = x[i * dim + a];
        ri = R[i];
    }
    int64_t cnt = 0;
    int64_t p = (MODE == 1 && i < n) ? off[i] : 0;
    for (int64_t base = 0; base < n; base += kTile) {
        __syncthreads();
        int64_t j = base + threadIdx.x;
        if (j < n) {
            for (int a = 0; a < dim; ++a) tx[threadIdx.x * 3 + a] = x[j * dim + a];
            tr[threadIdx.x] = R[j];
        }
        __syncthreads();
        if (i < n) {
            int lim = (int)((n - base) < kTile ? (n - base) : kTile);
            for (int t = 0; t < lim; ++t) {
                int64_t jj = base + t;
                if (jj == i) continue;
                if (overlap_test(dim, xi, &tx[t * 3], ri, tr[t])) {
                    if (MODE == 0) cnt++;
                    else idx[p++] = (int32_t)jj;
                }
            }
        }
    }
    if (MODE == 0 && i < n) counts[i] = cnt;
}

// Exclusive prefix sum of n counts into off[0..n] with a single workgroup:
// each thread sums a contiguous chunk, the chunk totals are scanned in LDS,
// then every chunk is written.
__global__ __launch_bounds__(1024) void scan_kernel(const int64_t *__restrict__ counts, int64_t *__restrict__ off,
                                                    int64_t n)
{
    __shared__ int64_t sums[1024];
    int t = threadIdx.x;
    int64_t chunk = (n + 1023) / 1024;
    int64_t lo = t * chunk, hi = lo + chunk < n ? lo + chunk : n;
    int64_t s = 0;
    for (int64_t k = lo; k < hi; ++k) s += counts[k];
    sums[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t v = (t >= d) ? sums[t - d] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    int64_t run = sums[t] - s;
    for (int64_t k = lo; k < hi; ++k) {
        off[k] = run;
        run += counts[k];
    }
    if (t == 1023) off[n] = sums[1023];
}

// Keep {y : nrm . y - off <= 0}; returns the new vertex count or -1 on overflow.
__device__ int clip_poly(int nv, const double *v, const int32_t *tg, double *ov, int32_t *otg, double n0, double n1,
                         double off, int32_t newtag)
{
    int no = 0;
    for (int k = 0; k < nv; ++k) {
        int kn = (k + 1 == nv) ? 0 : k + 1;
        double px = v[2 * k], py = v[2 * k + 1], qx = v[2 * kn], qy = v[2 * kn + 1];
        double sp = n0 * px + n1 * py - off;
        double sq = n0 * qx + n1 * qy - off;
        if (sp <= 0.0) {
            if (no >= kCellCap2D) return -1;
            ov[2 * no] = px;
            ov[2 * no + 1] = py;
            otg[no++] = tg[k];
            if (sq > 0.0) {
                double t = sp / (sp - sq);
                if (no >= kCellCap2D) return -1;
                ov[2 * no] = px + t * (qx - px);
                ov[2 * no + 1] = py + t * (qy - py);
                otg[no++] = newtag;
            }
        } else if (sq <= 0.0) {
            double t = sp / (sp - sq);
            if (no >= kCellCap2D) return -1;
            ov[2 * no] = px + t * (qx - px);
            ov[2 * no + 1] = py + t * (qy - py);
            otg[no++] = tg[k];
        }
    }
    return no;
}

// One thread per cell: kernel box intersected with the domain, clipped by the
// bisector half-plane of every overlap neighbour.  A neighbour farther than
// twice the current vertex radius cannot cut the polygon and is skipped.
__global__ __launch_bounds__(128) void clip2d_kernel(int64_t n, const double *__restrict__ x,
                                                     const double *__restrict__ R,
                                                     const int64_t *__restrict__ nb_off,
                                                     const int32_t *__restrict__ nb_idx, double lo0, double lo1,
                                                     double hi0, double hi1, int32_t *__restrict__ nv_out,
                                                     double *__restrict__ verts, int32_t *__restrict__ tags,
                                                     double *__restrict__ V, double *__restrict__ rho,
                                                     int32_t *__restrict__ flags, int64_t *__restrict__ bq_count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[2 * kCellCap2D], b[2 * kCellCap2D];
    int32_t ta[kCellCap2D], tb[kCellCap2D];
    const double xi0 = x[2 * i], xi1 = x[2 * i + 1], r = R[i];
    double l0 = xi0 - r, h0 = xi0 + r, l1 = xi1 - r, h1 = xi1 + r;
    int32_t tl0 = kTagBox, th0 = kTagBox, tl1 = kTagBox, th1 = kTagBox;
    if (l0 <= lo0) { l0 = lo0; tl0 = -1; }
    if (h0 >= hi0) { h0 = hi0; th0 = -2; }
    if (l1 <= lo1) { l1 = lo1; tl1 = -3; }
    if (h1 >= hi1) { h1 = hi1; th1 = -4; }
    a[0] = l0; a[1] = l1; ta[0] = tl1;
    a[2] = h0; a[3] = l1; ta[1] = th0;
    a[4] = h0; a[5] = h1; ta[2] = th1;
    a[6] = l0; a[7] = h1; ta[3] = tl0;
    int nv = 4;
    double r2max = 0.0;
    for (int k = 0; k < 4; ++k) {
        double d0 = a[2 * k] - xi0, d1 = a[2 * k + 1] - xi1;
        r2max = fmax(r2max, d0 * d0 + d1 * d1);
    }
    double *cur = a, *nxt = b;
    int32_t *tcur = ta, *tnxt = tb;
    int flag = 0;
    for (int64_t p = nb_off[i]; p < nb_off[i + 1]; ++p) {
        int32_t j = nb_idx[p];
        double dx0 = x[2 * (int64_t)j] - xi0, dx1 = x[2 * (int64_t)j + 1] - xi1;
        double dd = dx0 * dx0 + dx1 * dx1;
        if (0.25 * dd * (1.0 - 1e-12) >= r2max) continue;
        double m0 = 0.5 * (xi0 + x[2 * (int64_t)j]), m1 = 0.5 * (xi1 + x[2 * (int64_t)j + 1]);
        double off = dx0 * m0 + dx1 * m1;
        int no = clip_poly(nv, cur, tcur, nxt, tnxt, dx0, dx1, off, j);
        if (no < 0) { flag = 1; break; }
        nv = no;
        double *t = cur; cur = nxt; nxt = t;
        int32_t *tt = tcur; tcur = tnxt; tnxt = tt;
        r2max = 0.0;
        for (int k = 0; k < nv; ++k) {
            double d0 = cur[2 * k] - xi0, d1 = cur[2 * k + 1] - xi1;
            r2max = fmax(r2max, d0 * d0 + d1 * d1);
        }
        if (nv < 3) break;
    }
    int64_t nbe = 0;
    if (flag || nv < 3) {
        nv_out[i] = 0;
        V[i] = 0.0;
        rho[i] = 0.0;
        flags[i] = 1;
    } else {
        double area = 0.0;
        for (int k = 0; k < nv; ++k) {
            int kn = (k + 1 == nv) ? 0 : k + 1;
            double p0 = cur[2 * k] - xi0, p1 = cur[2 * k + 1] - xi1;
            double q0 = cur[2 * kn] - xi0, q1 = cur[2 * kn + 1] - xi1;
            area += 0.5 * (p0 * q1 - p1 * q0);
            verts[(i * kCellCap2D + k) * 2] = cur[2 * k];
            verts[(i * kCellCap2D + k) * 2 + 1] = cur[2 * k + 1];
            tags[i * kCellCap2D + k] = tcur[k];
            if (tcur[k] <= -1 && tcur[k] >= -4) nbe++;
        }
        nv_out[i] = nv;
        V[i] = area;
        rho[i] = sqrt(r2max);
        flags[i] = (r2max > r * r) ? 2 : 0;
    }
    bq_count[i] = nbe * kSegRule;
}

// Pattern row i: i inserted into its sorted overlap list.
__global__ void pattern_kernel(int64_t n, const int64_t *__restrict__ nb_off, const int32_t *__restrict__ nb_idx,
                               int64_t *__restrict__ row_off, int32_t *__restrict__ col,
                               int64_t *__restrict__ diag_pos)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    row_off[i] = (i < n ? nb_off[i] : nb_off[n]) + i;
    if (i == n) return;
    int64_t o = nb_off[i] + i;
    bool placed = false;
    for (int64_t p = nb_off[i]; p < nb_off[i + 1]; ++p) {
        int32_t j = nb_idx[p];
        if (!placed && j > i) {
            diag_pos[i] = o;
            col[o++] = (int32_t)i;
            placed = true;
        }
        col[o++] = j;
    }
    if (!placed) {
        diag_pos[i] = o;
        col[o++] = (int32_t)i;
    }
}

}  // namespace

hipError_t launch_neighbors_count(int dim, int64_t n, const double *x, const double *R, int64_t *counts, hipStream_t s)
{
    int grid = (int)((n + kTile - 1) / kTile);
    neighbors_kernel<0><<<grid, kTile, 0, s>>>(dim, n, x, R, counts, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_neighbors_fill(int dim, int64_t n, const double *x, const double *R, const int64_t *off,
                                 int32_t *idx, hipStream_t s)
{
    int grid = (int)((n + kTile - 1) / kTile);
    neighbors_kernel<1><<<grid, kTile, 0, s>>>(dim, n, x, R, nullptr, off, idx);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int64_t *counts, int64_t *off, int64_t n, hipStream_t s)
{
    scan_kernel<<<1, 1024, 0, s>>>(counts, off, n);
    return hipGetLastError();
}

hipError_t launch_clip2d(Problem &P, hipStream_t s, int32_t *flags, int64_t *bq_count)
{
    int grid = (int)((P.n + 127) / 128);
    clip2d_kernel<<<grid, 128, 0, s>>>(P.n, P.x.p, P.R.p, P.nb_off.p, P.nb_idx.p, P.dom_lo[0], P.dom_lo[1],
                                       P.dom_hi[0], P.dom_hi[1], P.nv.p, P.verts.p, P.tags.p, P.V.p, P.rho.p, flags,
                                       bq_count);
    return hipGetLastError();
}

hipError_t launch_pattern(Problem &P, hipStream_t s)
{
    int grid = (int)((P.n + 1 + 255) / 256);
    pattern_kernel<<<grid, 256, 0, s>>>(P.n, P.nb_off.p, P.nb_idx.p, P.row_off.p, P.col.p, P.diag_pos.p);
    return hipGetLastError();
}

}  // namespace mlpg
