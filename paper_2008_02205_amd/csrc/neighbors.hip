// Overlap connectivity by cell lists (Sec. 3.4, Eq. mlpg-connectivity):
// j != i is a neighbour of i when |x_i - x_j| <= R_i + R_j.
//
// The points' bounding box is cut into a uniform grid of cells of side at
// least 2 max_i R_i, so that two overlapping points sit in the same or in
// adjacent cells.  Points are binned (counts, exclusive scan, scatter; the
// order inside a cell is whatever the scatter's atomics give); every point
// then tests the points of the 3^dim cells around its own.  The count pass
// writes the list lengths, which do not depend on that order; the fill pass
// writes each list and sorts it (Shell sort with the gaps 701, 301, 132, 57,
// 23, 10, 4, 1 of Ciura, 2001), so the lists come out in increasing j exactly
// as a brute-force search over all pairs would draw them.
//
// Scratch (NbScratch): the bounding box, each point's cell, each cell's
// count and start, and the points in cell order.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace mlpg {

namespace {

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

struct NbGrid {
    double lo[3], inv_h;
    int dims[3];
    int dim;
};

// The cell of coordinate x along axis a, clamped to the grid (a NaN lands in
// cell 0: every index stays in range whatever the input).
__device__ __forceinline__ int cell_coord(const NbGrid &g, double x, int a)
{
    const double t = (x - g.lo[a]) * g.inv_h;
    if (t >= 0.0 && t < (double)g.dims[a]) return (int)t;
    return t >= (double)g.dims[a] ? g.dims[a] - 1 : 0;
}

// Bounding box and the largest radius: bb[0..2] min, bb[3..5] max, bb[6] max R.
__global__ __launch_bounds__(1024) void bbox_kernel(int dim, int64_t n, const double *__restrict__ x,
                                                    const double *__restrict__ R, double *__restrict__ bb)
{
    __shared__ double red[7][1024];
    double v[7];
    for (int a = 0; a < 3; ++a) {
        v[a] = 1e300;
        v[3 + a] = -1e300;
    }
    v[6] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        for (int a = 0; a < dim; ++a) {
            const double c = x[i * dim + a];
            v[a] = fmin(v[a], c);
            v[3 + a] = fmax(v[3 + a], c);
        }
        v[6] = fmax(v[6], R[i]);
    }
    for (int q = 0; q < 7; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int q = 0; q < 7; ++q) {
                const double o = red[q][threadIdx.x + st];
                double &m = red[q][threadIdx.x];
                m = (q < 3) ? fmin(m, o) : fmax(m, o);
            }
        __syncthreads();
    }
    if (threadIdx.x < 7) bb[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t count)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = 0u;
}

__global__ void nb_bin_kernel(int64_t n, NbGrid g, const double *__restrict__ x, int32_t *__restrict__ cell,
                              uint32_t *__restrict__ cnt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int a = 0; a < g.dim; ++a) c = c * g.dims[a] + cell_coord(g, x[i * g.dim + a], a);
    cell[i] = c;
    atomicAdd(&cnt[c], 1u);
}

// exclusive scan of the 32-bit cell counts into 64-bit starts (one workgroup)
__global__ __launch_bounds__(1024) void nb_scan_kernel(const uint32_t *__restrict__ cnt, int64_t *__restrict__ off,
                                                       int64_t m)
{
    __shared__ int64_t sums[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (m + 1023) / 1024;
    const int64_t lo = t * chunk, hi = lo + chunk < m ? lo + chunk : m;
    int64_t s = 0;
    for (int64_t k = lo; k < hi; ++k) s += cnt[k];
    sums[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? sums[t - d] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    int64_t run = sums[t] - s;
    for (int64_t k = lo; k < hi; ++k) {
        off[k] = run;
        run += cnt[k];
    }
    if (t == 1023) off[m] = sums[1023];
}

__global__ void nb_scatter_kernel(int64_t n, const int32_t *__restrict__ cell, const int64_t *__restrict__ off,
                                  uint32_t *__restrict__ cursor, int32_t *__restrict__ pts)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    const uint32_t k = atomicAdd(&cursor[c], 1u);
    pts[off[c] + k] = (int32_t)i;
}

// MODE 0: counts[i] = number of neighbours; MODE 1: the neighbours into
// idx[off[i] ..] (cell order), then sorted.
template <int MODE>
__global__ __launch_bounds__(256) void nb_search_kernel(int64_t n, NbGrid g, const double *__restrict__ x,
                                                        const double *__restrict__ R,
                                                        const int64_t *__restrict__ coff,
                                                        const int32_t *__restrict__ pts, int64_t *__restrict__ counts,
                                                        const int64_t *__restrict__ off, int32_t *__restrict__ idx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int dim = g.dim;
    double xi[3] = {0, 0, 0};
    int ci[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        xi[a] = x[i * dim + a];
        ci[a] = cell_coord(g, xi[a], a);
    }
    const double ri = R[i];
    int64_t cnt = 0;
    int64_t p = MODE == 1 ? off[i] : 0;
    const int64_t pend = MODE == 1 ? off[i + 1] : 0;   // the row's slots: never written past
    const int lo2 = dim == 3 ? -1 : 0, hi2 = dim == 3 ? 1 : 0;
    for (int d0 = -1; d0 <= 1; ++d0) {
        const int c0 = ci[0] + d0;
        if (c0 < 0 || c0 >= g.dims[0]) continue;
        for (int d1 = -1; d1 <= 1; ++d1) {
            const int c1 = ci[1] + d1;
            if (c1 < 0 || c1 >= g.dims[1]) continue;
            for (int d2 = lo2; d2 <= hi2; ++d2) {
                const int c2 = ci[2] + d2;
                if (dim == 3 && (c2 < 0 || c2 >= g.dims[2])) continue;
                const int c = dim == 3 ? (c0 * g.dims[1] + c1) * g.dims[2] + c2 : c0 * g.dims[1] + c1;
                for (int64_t q = coff[c]; q < coff[c + 1]; ++q) {
                    const int32_t j = pts[q];
                    if (j == i) continue;
                    double xj[3] = {0, 0, 0};
                    for (int a = 0; a < dim; ++a) xj[a] = x[(int64_t)j * dim + a];
                    if (overlap_test(dim, xi, xj, ri, R[j])) {
                        if (MODE == 0) cnt++;
                        else if (p < pend) idx[p++] = j;
                    }
                }
            }
        }
    }
    if (MODE == 0) {
        counts[i] = cnt;
        return;
    }
    // Shell sort of the row (Ciura's gaps)
    const int64_t a0 = off[i];
    const int64_t len = p - a0;
    const int gaps[8] = {701, 301, 132, 57, 23, 10, 4, 1};
    for (int gi = 0; gi < 8; ++gi) {
        const int64_t gp = gaps[gi];
        if (gp >= len) continue;
        for (int64_t u = gp; u < len; ++u) {
            const int32_t v = idx[a0 + u];
            int64_t w = u;
            while (w >= gp && idx[a0 + w - gp] > v) {
                idx[a0 + w] = idx[a0 + w - gp];
                w -= gp;
            }
            idx[a0 + w] = v;
        }
    }
}

inline unsigned grid_of(int64_t count, int threads) { return (unsigned)((count + threads - 1) / threads); }

// Binning shared by both passes; returns the grid and fills the scratch.
hipError_t nb_bin(int dim, int64_t n, const double *x, const double *R, const NbScratch &sc, NbGrid *g_out,
                  hipStream_t s)
{
    bbox_kernel<<<1, 1024, 0, s>>>(dim, n, x, R, sc.bbox);
    double bb[7];
    hipError_t e;
    if ((e = hipMemcpyAsync(bb, sc.bbox, sizeof(bb), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    NbGrid g;
    g.dim = dim;
    // cells of side 2 max R (a hair more, so that rounding cannot push an
    // overlapping pair two cells apart), enlarged while the grid is too big
    double h = 2.0 * bb[6] * (1.0 + 1e-12);
    double ext = 0.0;
    for (int a = 0; a < dim; ++a) ext = std::max(ext, bb[3 + a] - bb[a]);
    if (!(h > 0.0)) h = ext > 0.0 ? ext : 1.0;
    if (!std::isfinite(h) || !std::isfinite(ext)) return hipErrorInvalidValue;
    for (;;) {
        int64_t m = 1;
        bool big = false;
        for (int a = 0; a < dim; ++a) {
            const double d = std::floor((bb[3 + a] - bb[a]) / h) + 1.0;
            if (d > 1e9) big = true;
            g.dims[a] = big ? 1 : (int)d;
            m *= g.dims[a];
        }
        if (!big && m <= sc.max_cells) break;
        h *= 2.0;
    }
    for (int a = 0; a < 3; ++a) g.lo[a] = a < dim ? bb[a] : 0.0;
    for (int a = dim; a < 3; ++a) g.dims[a] = 1;
    g.inv_h = 1.0 / h;
    int64_t m = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    zero_u32_kernel<<<grid_of(m, 256), 256, 0, s>>>(sc.cnt, m);
    nb_bin_kernel<<<grid_of(n, 256), 256, 0, s>>>(n, g, x, sc.cell, sc.cnt);
    nb_scan_kernel<<<1, 1024, 0, s>>>(sc.cnt, sc.coff, m);
    zero_u32_kernel<<<grid_of(m, 256), 256, 0, s>>>(sc.cnt, m);
    nb_scatter_kernel<<<grid_of(n, 256), 256, 0, s>>>(n, sc.cell, sc.coff, sc.cnt, sc.pts);
    *g_out = g;
    return hipGetLastError();
}

}  // namespace

int64_t nb_max_cells(int64_t n) { return std::max<int64_t>(n, 4096); }

hipError_t launch_neighbors_count(int dim, int64_t n, const double *x, const double *R, int64_t *counts,
                                  const NbScratch &sc, hipStream_t s)
{
    NbGrid g;
    hipError_t e = nb_bin(dim, n, x, R, sc, &g, s);
    if (e != hipSuccess) return e;
    nb_search_kernel<0><<<grid_of(n, 256), 256, 0, s>>>(n, g, x, R, sc.coff, sc.pts, counts, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_neighbors_fill(int dim, int64_t n, const double *x, const double *R, const int64_t *off,
                                 int32_t *idx, const NbScratch &sc, hipStream_t s)
{
    NbGrid g;
    hipError_t e = nb_bin(dim, n, x, R, sc, &g, s);
    if (e != hipSuccess) return e;
    nb_search_kernel<1><<<grid_of(n, 256), 256, 0, s>>>(n, g, x, R, sc.coff, sc.pts, nullptr, off, idx);
    return hipGetLastError();
}

size_t nb_scratch_bytes(int64_t n, int64_t max_cells)
{
    return Arena::align(8 * 8) + Arena::align(4 * (size_t)n) + Arena::align(4 * (size_t)max_cells) +
           Arena::align(8 * (size_t)(max_cells + 1)) + Arena::align(4 * (size_t)n);
}

NbScratch nb_scratch_at(void *base, int64_t n, int64_t max_cells)
{
    NbScratch sc;
    char *p = (char *)base;
    sc.bbox = (double *)p;
    p += Arena::align(8 * 8);
    sc.cell = (int32_t *)p;
    p += Arena::align(4 * (size_t)n);
    sc.cnt = (uint32_t *)p;
    p += Arena::align(4 * (size_t)max_cells);
    sc.coff = (int64_t *)p;
    p += Arena::align(8 * (size_t)(max_cells + 1));
    sc.pts = (int32_t *)p;
    sc.max_cells = max_cells;
    return sc;
}

}  // namespace mlpg
