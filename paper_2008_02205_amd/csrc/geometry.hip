// Geometry kernels: overlap connectivity (Sec. 3.4), Voronoi-like cells in
// 2D and 3D (Sec. 3.1, Fig. 1) and the sparse pattern of the bilinear forms.
#include "internal.hpp"

namespace mlpg {

namespace {

// Exclusive prefix sum of n counts into off[0..n] with a single workgroup:
// each thread sums a contiguous chunk, the chunk totals are scanned in LDS,
// then every chunk is written.  counts and off may be the same array (each
// thread reads an entry of its own chunk before overwriting it).
__global__ __launch_bounds__(1024) void scan_kernel(const int64_t *counts, int64_t *off, int64_t n)
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
        const int64_t c = counts[k];
        off[k] = run;
        run += c;
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

// ---- 3D cells ---------------------------------------------------------------
//
// One wavefront per cell, one lane per face.  The cell is the kernel box
// intersected with the domain, clipped by the bisector plane of every
// overlap neighbour (Sec. 3.1 in three dimensions).  Each clip: every lane
// clips its face polygon (kept side n.y - off <= 0; a crossing edge is cut at
// the point computed from its kept end, so the two faces sharing the edge
// produce the same point), surviving faces are compacted in order, and the
// cut points form the new face: lexicographic order, duplicates dropped,
// then ordered by the diamond pseudo-angle about their centroid in the frame
// u = n x e_k, v = n x u (counter-clockwise seen from outside).  A plane that
// keeps every vertex changes nothing.  Neighbours are taken nearest first, so
// the clipping stops at the first one whose bisector lies beyond the farthest
// vertex (no later plane can cut); the intersection of the half-spaces does
// not depend on the order, only the rounding of the vertices does.  No FP contraction, so that the
// same arithmetic gives the same vertices anywhere it is evaluated.
constexpr int kClipCuts = 160;
constexpr int kNbSort = 1024;   // neighbour lists up to this length are sorted by distance

__device__ __forceinline__ double dot3d(const double *a, const double *b)
{
#pragma clang fp contract(off)
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void cross3d(const double *a, const double *b, double *c)
{
#pragma clang fp contract(off)
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ bool lex_less3d(const double *a, const double *b)
{
    if (a[0] != b[0]) return a[0] < b[0];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[2] < b[2];
}

__device__ __forceinline__ bool eq3d(const double *a, const double *b)
{
    return a[0] == b[0] && a[1] == b[1] && a[2] == b[2];
}

__device__ __forceinline__ double diamond(double dx, double dy)
{
#pragma clang fp contract(off)
    if (dy >= 0.0) return dx >= 0.0 ? dy / (dx + dy) : 1.0 - dx / (-dx + dy);
    return dx < 0.0 ? 2.0 - dy / (-dx - dy) : 3.0 + dx / (dx - dy);
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__global__ __launch_bounds__(64) void clip3d_kernel(int64_t n, const double *__restrict__ x,
                                                    const double *__restrict__ R,
                                                    const int64_t *__restrict__ nb_off,
                                                    const int32_t *__restrict__ nb_idx, double lo0, double lo1,
                                                    double lo2, double hi0, double hi1, double hi2,
                                                    int32_t *__restrict__ nf_out, int32_t *__restrict__ fnv_out,
                                                    int32_t *__restrict__ ftag_out, double *__restrict__ fv_out,
                                                    double *__restrict__ V, double *__restrict__ rho,
                                                    int32_t *__restrict__ flags, int64_t *__restrict__ bq_count)
{
#pragma clang fp contract(off)
    __shared__ double sv[kFaceCap3][kFaceVerts3][3];   // current faces
    __shared__ double tv[kFaceCap3][kFaceVerts3][3];   // clipped faces, at their old index
    __shared__ int snv[kFaceCap3], stag[kFaceCap3], tnv[kFaceCap3], ttag[kFaceCap3];
    __shared__ double cuts[kClipCuts][3], uniq[kClipCuts][3], ang[kClipCuts];
    __shared__ int first[kClipCuts];
    __shared__ double gsh[3];
    __shared__ int s_ncut, s_flag;
    __shared__ double sd[kNbSort];
    __shared__ int32_t sj[kNbSort];

    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    const double r = R[i];
    const double dlo[3] = {lo0, lo1, lo2}, dhi[3] = {hi0, hi1, hi2};
    double blo[3], bhi[3];
    int32_t bt[6];
    for (int a = 0; a < 3; ++a) {
        blo[a] = xi[a] - r;
        bhi[a] = xi[a] + r;
        bt[2 * a] = kTagBox;
        bt[2 * a + 1] = kTagBox;
        if (blo[a] <= dlo[a]) { blo[a] = dlo[a]; bt[2 * a] = -1 - 2 * a; }
        if (bhi[a] >= dhi[a]) { bhi[a] = dhi[a]; bt[2 * a + 1] = -2 - 2 * a; }
    }
    // box faces -x,+x,-y,+y,-z,+z; corner bit b picks lo (0) or hi (1)
    if (lane < 6) {
        const int f = lane;
        const int ax = f >> 1, side = f & 1;
        const int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
        // corners in the (o1, o2) plane, counter-clockwise seen from outside
        const int c1[4] = {0, 1, 1, 0}, c2[4] = {0, 0, 1, 1};
        for (int k = 0; k < 4; ++k) {
            int kk = side ? k : (k == 0 ? 0 : 4 - k);   // reversed on the low side
            double p[3];
            p[ax] = side ? bhi[ax] : blo[ax];
            p[o1] = c1[kk] ? bhi[o1] : blo[o1];
            p[o2] = c2[kk] ? bhi[o2] : blo[o2];
            for (int a = 0; a < 3; ++a) sv[f][k][a] = p[a];
        }
        snv[f] = 4;
        stag[f] = bt[f];
    }
    if (lane == 0) s_flag = 0;
    int nf = 6;
    __syncthreads();
    double r2 = 0.0;
    if (lane < nf)
        for (int k = 0; k < snv[lane]; ++k) {
            double d[3] = {sv[lane][k][0] - xi[0], sv[lane][k][1] - xi[1], sv[lane][k][2] - xi[2]};
            r2 = fmax(r2, dot3d(d, d));
        }
    double r2max = wave_max(r2);

    // neighbours nearest first (ties by index), by a bitonic sort in LDS; a
    // list longer than the sort buffer is taken in index order instead
    const int64_t p0 = nb_off[i];
    const int cnt = (int)(nb_off[i + 1] - p0);
    const bool sorted = cnt <= kNbSort;
    if (sorted) {
        int N = 64;
        while (N < cnt) N <<= 1;
        for (int k = lane; k < N; k += 64) {
            if (k < cnt) {
                const int32_t jj = nb_idx[p0 + k];
                const double d[3] = {x[3 * (int64_t)jj] - xi[0], x[3 * (int64_t)jj + 1] - xi[1],
                                     x[3 * (int64_t)jj + 2] - xi[2]};
                sd[k] = dot3d(d, d);
                sj[k] = jj;
            } else {
                sd[k] = HUGE_VAL;
                sj[k] = INT32_MAX;
            }
        }
        __syncthreads();
        for (int size = 2; size <= N; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = lane; t < N / 2; t += 64) {
                    const int a = 2 * stride * (t / stride) + (t % stride), b = a + stride;
                    const bool up = (a & size) == 0;
                    const bool gt = sd[a] > sd[b] || (sd[a] == sd[b] && sj[a] > sj[b]);
                    if (gt == up) {
                        const double td = sd[a]; sd[a] = sd[b]; sd[b] = td;
                        const int32_t tj = sj[a]; sj[a] = sj[b]; sj[b] = tj;
                    }
                }
                __syncthreads();
            }
    }

    for (int k = 0; k < cnt; ++k) {
        const int32_t j = sorted ? sj[k] : nb_idx[p0 + k];
        const double xj[3] = {x[3 * (int64_t)j], x[3 * (int64_t)j + 1], x[3 * (int64_t)j + 2]};
        const double nrm[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
        const double dd = dot3d(nrm, nrm);
        if (0.25 * dd * (1.0 - 1e-12) >= r2max) {
            if (sorted) break;   // every later neighbour is at least as far
            continue;
        }
        const double mid[3] = {0.5 * (xi[0] + xj[0]), 0.5 * (xi[1] + xj[1]), 0.5 * (xi[2] + xj[2])};
        const double off = dot3d(nrm, mid);
        bool outside = false;
        if (lane < nf)
            for (int k = 0; k < snv[lane]; ++k) outside |= (dot3d(nrm, sv[lane][k]) - off > 0.0);
        if (__ballot(outside) == 0) continue;
        if (lane == 0) s_ncut = 0;
        __syncthreads();
        // clip this lane's face into tv[lane]
        if (lane < nf) {
            const int nv = snv[lane];
            int no = 0;
            for (int k = 0; k < nv; ++k) {
                const double *A = sv[lane][k];
                const double *B = sv[lane][k + 1 == nv ? 0 : k + 1];
                const double sa = dot3d(nrm, A) - off, sb = dot3d(nrm, B) - off;
                if (sa <= 0.0) {
                    if (no < kFaceVerts3) {
                        tv[lane][no][0] = A[0]; tv[lane][no][1] = A[1]; tv[lane][no][2] = A[2];
                    }
                    no++;
                    if (sa == 0.0) {
                        int c = atomicAdd(&s_ncut, 1);
                        if (c < kClipCuts) { cuts[c][0] = A[0]; cuts[c][1] = A[1]; cuts[c][2] = A[2]; }
                    }
                }
                if ((sa < 0.0 && sb > 0.0) || (sa > 0.0 && sb < 0.0)) {
                    const double *I = sa < 0.0 ? A : B, *O = sa < 0.0 ? B : A;
                    const double si = sa < 0.0 ? sa : sb, so = sa < 0.0 ? sb : sa;
                    const double t = si / (si - so);
                    const double c0 = I[0] + t * (O[0] - I[0]), c1 = I[1] + t * (O[1] - I[1]),
                                 c2 = I[2] + t * (O[2] - I[2]);
                    if (no < kFaceVerts3) { tv[lane][no][0] = c0; tv[lane][no][1] = c1; tv[lane][no][2] = c2; }
                    no++;
                    int c = atomicAdd(&s_ncut, 1);
                    if (c < kClipCuts) { cuts[c][0] = c0; cuts[c][1] = c1; cuts[c][2] = c2; }
                }
            }
            if (no > kFaceVerts3) s_flag = 1;
            tnv[lane] = no < kFaceVerts3 ? no : kFaceVerts3;   // the clip fails below when it overflowed
            ttag[lane] = stag[lane];
        }
        __syncthreads();
        // compact the surviving faces in order
        const bool keep = lane < nf && tnv[lane] >= 3;
        const uint64_t km = __ballot(keep);
        const int nk = __popcll(km);
        if (keep) {
            const int d = __popcll(km & ((1ull << lane) - 1));
            for (int k = 0; k < tnv[lane]; ++k)
                for (int a = 0; a < 3; ++a) sv[d][k][a] = tv[lane][k][a];
            snv[d] = tnv[lane];
            stag[d] = ttag[lane];
        }
        const int nc = s_ncut;
        if (nc > kClipCuts) s_flag = 1;
        const int ncu = nc < kClipCuts ? nc : kClipCuts;
        // the new face: unique cut points in lexicographic order
        for (int k = lane; k < ncu; k += 64) {
            int dup = 0;
            for (int m = 0; m < k; ++m) dup += eq3d(cuts[m], cuts[k]);
            first[k] = dup == 0;
        }
        __syncthreads();
        for (int k = lane; k < ncu; k += 64)
            if (first[k]) {
                int pos = 0;
                for (int m = 0; m < ncu; ++m) pos += (first[m] && lex_less3d(cuts[m], cuts[k]));
                uniq[pos][0] = cuts[k][0]; uniq[pos][1] = cuts[k][1]; uniq[pos][2] = cuts[k][2];
            }
        int nu = 0;
        for (int m = 0; m < ncu; ++m) nu += first[m];
        __syncthreads();
        nf = nk;
        if (nu >= 3) {
            if (nf >= kFaceCap3 || nu > kFaceVerts3) {
                s_flag = 1;
            } else {
                if (lane == 0) {
                    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
                    for (int a = 0; a < nu; ++a) { g0 += uniq[a][0]; g1 += uniq[a][1]; g2 += uniq[a][2]; }
                    gsh[0] = g0 / nu; gsh[1] = g1 / nu; gsh[2] = g2 / nu;
                }
                __syncthreads();
                int ax = 0;
                for (int d = 1; d < 3; ++d)
                    if (fabs(nrm[d]) < fabs(nrm[ax])) ax = d;
                double e[3] = {0.0, 0.0, 0.0}, u[3], v[3];
                e[ax] = 1.0;
                cross3d(nrm, e, u);
                cross3d(nrm, u, v);
                for (int k = lane; k < nu; k += 64) {
                    double rr[3] = {uniq[k][0] - gsh[0], uniq[k][1] - gsh[1], uniq[k][2] - gsh[2]};
                    ang[k] = diamond(dot3d(u, rr), dot3d(v, rr));
                }
                __syncthreads();
                for (int k = lane; k < nu; k += 64) {
                    int rank = 0;
                    for (int m = 0; m < nu; ++m) rank += (ang[m] < ang[k] || (ang[m] == ang[k] && m < k));
                    sv[nf][rank][0] = uniq[k][0]; sv[nf][rank][1] = uniq[k][1]; sv[nf][rank][2] = uniq[k][2];
                }
                if (lane == 0) { snv[nf] = nu; stag[nf] = j; }
                nf++;
            }
        }
        __syncthreads();
        if (s_flag) break;
        r2 = 0.0;
        if (lane < nf)
            for (int k = 0; k < snv[lane]; ++k) {
                double d[3] = {sv[lane][k][0] - xi[0], sv[lane][k][1] - xi[1], sv[lane][k][2] - xi[2]};
                r2 = fmax(r2, dot3d(d, d));
            }
        r2max = wave_max(r2);
    }
    __syncthreads();
    const bool failed = s_flag != 0 || nf < 4;
    if (failed) {
        if (lane == 0) {
            nf_out[i] = 0; V[i] = 0.0; rho[i] = 0.0; flags[i] = 1; bq_count[i] = 0;
        }
        return;
    }
    if (lane < nf) {
        const int nv = snv[lane];
        fnv_out[i * kFaceCap3 + lane] = nv;
        ftag_out[i * kFaceCap3 + lane] = stag[lane];
        double *o = fv_out + ((i * kFaceCap3 + lane) * kFaceVerts3) * 3;
        for (int k = 0; k < nv; ++k)
            for (int a = 0; a < 3; ++a) o[3 * k + a] = sv[lane][k][a];
    }
    if (lane == 0) {
        // volume: tetrahedra (x_i, v_0, v_k, v_k+1) of each face fan, in face order
        double vol = 0.0;
        int64_t nbt = 0;
        for (int f = 0; f < nf; ++f) {
            const int nv = snv[f];
            const double e1[3] = {sv[f][0][0] - xi[0], sv[f][0][1] - xi[1], sv[f][0][2] - xi[2]};
            for (int k = 1; k + 1 < nv; ++k) {
                double e2[3], e3[3], c[3];
                for (int a = 0; a < 3; ++a) { e2[a] = sv[f][k][a] - xi[a]; e3[a] = sv[f][k + 1][a] - xi[a]; }
                cross3d(e2, e3, c);
                vol += dot3d(e1, c) / 6.0;
            }
            if (stag[f] <= -1 && stag[f] >= -6) nbt += nv - 2;
        }
        nf_out[i] = nf;
        V[i] = vol;
        rho[i] = sqrt(r2max);
        flags[i] = (r2max > r * r) ? 2 : 0;
        bq_count[i] = nbt * kTri3Rule;
    }
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

// Caller-supplied overlap lists: row offsets within [0, total] and
// non-decreasing from 0, indices in [0, n), never i itself, strictly
// increasing along a row.  A row whose offsets are out of range is not read.
// Sets bit 1 (offsets) or bit 2 (indices) of *bad.
__global__ void check_lists_kernel(int64_t n, int64_t total, const int64_t *__restrict__ off,
                                   const int32_t *__restrict__ idx, unsigned long long *bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = off[i], b = off[i + 1];
    if ((i == 0 && a != 0) || a < 0 || b < a || b > total) {
        atomicOr(bad, 1ull);
        return;
    }
    int64_t prev = -1;
    for (int64_t p = a; p < b; ++p) {
        const int64_t j = idx[p];
        if (j < 0 || j >= n || j == i || j <= prev) {
            atomicOr(bad, 2ull);
            return;
        }
        prev = j;
    }
}

}  // namespace

hipError_t launch_check_lists(int64_t n, int64_t total, const int64_t *off, const int32_t *idx,
                              unsigned long long *bad, hipStream_t s)
{
    check_lists_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, total, off, idx, bad);
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

hipError_t launch_clip3d(Problem &P, hipStream_t s, int32_t *flags, int64_t *bq_count)
{
    clip3d_kernel<<<(unsigned)P.n, 64, 0, s>>>(P.n, P.x.p, P.R.p, P.nb_off.p, P.nb_idx.p, P.dom_lo[0], P.dom_lo[1],
                                              P.dom_lo[2], P.dom_hi[0], P.dom_hi[1], P.dom_hi[2], P.nf.p, P.fnv.p,
                                              P.ftags.p, P.fverts.p, P.V.p, P.rho.p, flags, bq_count);
    return hipGetLastError();
}

hipError_t launch_pattern(Problem &P, hipStream_t s)
{
    int grid = (int)((P.n + 1 + 255) / 256);
    pattern_kernel<<<grid, 256, 0, s>>>(P.n, P.nb_off.p, P.nb_idx.p, P.row_off.p, P.col.p, P.diag_pos.p);
    return hipGetLastError();
}

}  // namespace mlpg
