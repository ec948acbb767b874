/*
 * Plain FP64 CPU oracle for the meshless-local Petrov-Galerkin (MLPG)
 * discrete-ordinates transport method with Voronoi-cell integration
 * (Bassett & Owen, arXiv 2008.02205).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It is written to be read against the paper:
 * straightforward loops in the order the paper states the method, no blocking
 * or fusion, FP64 throughout.
 *
 * Contents (paper section in brackets):
 *   - overlap connectivity (Sec. 3.4, Eq. mlpg-connectivity)
 *   - Voronoi-like cells: kernel-extent box clipped by bisector half-planes
 *     (Sec. 3.1, Fig. 1), fan subdivision into triangles / tetrahedra (Fig. 2)
 *   - cubic-spline kernel and its gradient (Sec. 2.1)
 *   - reproducing-kernel functions U_j and their gradients from the moment
 *     matrix M, C = M^-1 G, dC = -M^-1 dM C (Sec. 2.2, Eq. rk-matrix)
 *   - meshless integration with quadrature outermost (Sec. 3.2, Alg. 1,
 *     App. A maps) into direction-independent sparse blocks
 *   - operators L, T, MS, D and r of Sec. 4.2 applied per ordinate
 *   - per-ordinate GMRES for L^-1 and the outer GMRES on
 *     (I - D L^-1 MS) Phi = b_phi (Eq. krylov-operator), backward Euler
 *     (Sec. 4.1) and recovery Psi = L^-1 MS Phi + b_psi.
 *
 * Readings where the paper is silent (kernel shape, scaled monomials, row
 * scaling by V_i, fallback order for a singular moment matrix, tau) are the
 * ones listed in the design notes; each is restated where it is used.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXB 10   /* largest monomial basis: quadratic in 3D */
#define ORC_MAXD 3

/* ------------------------------------------------------------------------ */
/* Overlap connectivity (Sec. 3.4): j is a neighbour of i when the supports
 * of W_i and W_j intersect, |x_i - x_j| <= R_i + R_j.  Brute force over all
 * pairs; lists exclude i itself and are in increasing index order.         */
/* ------------------------------------------------------------------------ */
static int overlaps(int dim, const double *xi, const double *xj, double ri, double rj)
{
    double d2 = 0.0;
    for (int a = 0; a < dim; ++a) {
        double t = xj[a] - xi[a];
        d2 = d2 + t * t;
    }
    double s = ri + rj;
    return d2 <= s * s;
}

int64_t orc_neighbors_count(int dim, int64_t n, const double *x, const double *R, int64_t *off)
{
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && overlaps(dim, x + i * dim, x + j * dim, R[i], R[j])) c++;
        off[i + 1] = off[i] + c;
    }
    return off[n];
}

void orc_neighbors_fill(int dim, int64_t n, const double *x, const double *R, const int64_t *off,
                        int32_t *idx)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = off[i];
        for (int64_t j = 0; j < n; ++j)
            if (j != i && overlaps(dim, x + i * dim, x + j * dim, R[i], R[j])) idx[p++] = (int32_t)j;
    }
}

/* ------------------------------------------------------------------------ */
/* Voronoi-like cells in 2D (Sec. 3.1).  The initial polygon is the box
 * [x_i - R_i, x_i + R_i]^2 (it encloses the kernel extent), intersected with
 * the domain box; it is then clipped by the half-plane on x_i's side of the
 * bisector of x_i and every overlap neighbour x_j.  Each edge carries a tag:
 *   tag >= 0            : edge lies on the bisector with neighbour tag
 *   tag = -1 - a        : edge lies on domain face a (0:-x 1:+x 2:-y 3:+y)
 *   tag = ORC_TAG_BOX   : edge of the kernel box not on the domain
 * Vertices are counter-clockwise; edge k runs from vertex k to k+1.        */
/* ------------------------------------------------------------------------ */
#define ORC_TAG_BOX (-100)

static int clip_polygon(int nv, const double *v, const int32_t *tag, double *ov, int32_t *otag,
                        const double *nrm, double off, int32_t newtag, int cap)
{
    /* keep { y : nrm . y - off <= 0 } (points on the line are kept) */
    int no = 0;
    for (int k = 0; k < nv; ++k) {
        const double *P = v + 2 * k;
        const double *Q = v + 2 * ((k + 1) % nv);
        double sp = nrm[0] * P[0] + nrm[1] * P[1] - off;
        double sq = nrm[0] * Q[0] + nrm[1] * Q[1] - off;
        if (sp <= 0.0) {
            if (no >= cap) return -1;
            ov[2 * no] = P[0]; ov[2 * no + 1] = P[1];
            otag[no++] = tag[k];       /* from P onward along edge k */
            if (sq > 0.0) {
                double t = sp / (sp - sq);
                if (no >= cap) return -1;
                ov[2 * no] = P[0] + t * (Q[0] - P[0]);
                ov[2 * no + 1] = P[1] + t * (Q[1] - P[1]);
                otag[no++] = newtag;   /* ... and from the cut point on along the bisector */
            }
        } else if (sq <= 0.0) {
            double t = sp / (sp - sq);
            if (no >= cap) return -1;
            ov[2 * no] = P[0] + t * (Q[0] - P[0]);
            ov[2 * no + 1] = P[1] + t * (Q[1] - P[1]);
            otag[no++] = tag[k];       /* from this cut point to Q lies on edge k */
        }
    }
    return no;
}

int64_t orc_cells2d(int64_t n, const double *x, const double *R, const int64_t *off, const int32_t *idx,
                    const double *dom_lo, const double *dom_hi, int cap, int32_t *nv_out,
                    double *verts, int32_t *tags, double *V, double *rho)
{
    double *a = (double *)malloc(sizeof(double) * 2 * cap), *b = (double *)malloc(sizeof(double) * 2 * cap);
    int32_t *ta = (int32_t *)malloc(sizeof(int32_t) * cap), *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = x + 2 * i;
        double lo0 = xi[0] - R[i], hi0 = xi[0] + R[i], lo1 = xi[1] - R[i], hi1 = xi[1] + R[i];
        int32_t t_lo0 = ORC_TAG_BOX, t_hi0 = ORC_TAG_BOX, t_lo1 = ORC_TAG_BOX, t_hi1 = ORC_TAG_BOX;
        if (lo0 <= dom_lo[0]) { lo0 = dom_lo[0]; t_lo0 = -1; }
        if (hi0 >= dom_hi[0]) { hi0 = dom_hi[0]; t_hi0 = -2; }
        if (lo1 <= dom_lo[1]) { lo1 = dom_lo[1]; t_lo1 = -3; }
        if (hi1 >= dom_hi[1]) { hi1 = dom_hi[1]; t_hi1 = -4; }
        /* CCW: (lo0,lo1) -> (hi0,lo1) -> (hi0,hi1) -> (lo0,hi1) */
        a[0] = lo0; a[1] = lo1; ta[0] = t_lo1;
        a[2] = hi0; a[3] = lo1; ta[1] = t_hi0;
        a[4] = hi0; a[5] = hi1; ta[2] = t_hi1;
        a[6] = lo0; a[7] = hi1; ta[3] = t_lo0;
        int nv = 4;
        for (int64_t p = off[i]; p < off[i + 1] && nv > 0; ++p) {
            int32_t j = idx[p];
            const double *xj = x + 2 * j;
            double nrm[2] = {xj[0] - xi[0], xj[1] - xi[1]};
            double mid[2] = {0.5 * (xi[0] + xj[0]), 0.5 * (xi[1] + xj[1])};
            double o = nrm[0] * mid[0] + nrm[1] * mid[1];
            int no = clip_polygon(nv, a, ta, b, tb, nrm, o, j, cap);
            if (no < 0) { nv = -1; break; }
            nv = no;
            double *s = a; a = b; b = s;
            int32_t *st = ta; ta = tb; tb = st;
        }
        if (nv < 3) {
            bad++;
            nv_out[i] = 0; V[i] = 0.0; rho[i] = 0.0;
            continue;
        }
        nv_out[i] = nv;
        double area = 0.0, r2 = 0.0;
        for (int k = 0; k < nv; ++k) {
            const double *P = a + 2 * k, *Q = a + 2 * ((k + 1) % nv);
            area += 0.5 * ((P[0] - xi[0]) * (Q[1] - xi[1]) - (P[1] - xi[1]) * (Q[0] - xi[0]));
            double d0 = P[0] - xi[0], d1 = P[1] - xi[1];
            if (d0 * d0 + d1 * d1 > r2) r2 = d0 * d0 + d1 * d1;
            verts[(i * cap + k) * 2] = P[0];
            verts[(i * cap + k) * 2 + 1] = P[1];
            tags[i * cap + k] = ta[k];
        }
        V[i] = area;
        rho[i] = sqrt(r2);
    }
    free(a); free(b); free(ta); free(tb);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Voronoi-like cells in 3D (Sec. 3.1, the three-dimensional case).  The
 * polyhedron starts as the box [x_i - R_i, x_i + R_i]^3 intersected with the
 * domain box and is clipped by the half-space on x_i's side of the bisector
 * plane of x_i and every overlap neighbour x_j.  It is stored as a list of
 * convex faces; each face is a polygon whose vertices run counter-clockwise
 * seen from outside the cell, and carries a tag as in 2D:
 *   tag >= 0 : face on the bisector with neighbour tag
 *   tag = -1 - a : face on domain face a (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z)
 *   tag = ORC_TAG_BOX : face of the kernel box not on the domain.
 * One clip: every face is clipped as a polygon (vertices with n.y - off <= 0
 * are kept; a crossing edge is cut at the point computed from its kept end),
 * faces left with fewer than three vertices are dropped, and the cut points
 * (together with kept vertices lying exactly on the plane) form the new face
 * on the plane.  Its vertices are put in lexicographic order, duplicates are
 * removed, and they are ordered by angle around the plane normal about their
 * centroid; the angle is the "diamond" pseudo-angle (a monotone function of
 * the angle using only arithmetic).  A plane that leaves every vertex kept
 * changes nothing.  Neighbours are applied nearest first (ties by index):
 * the cell does not depend on the order, but the faces' vertex order, and
 * with it the fan of tetrahedra the quadrature uses, does, so the order is
 * part of the definition.                                                  */
/* ------------------------------------------------------------------------ */
#define ORC_FCAP3 64
#define ORC_VCAP3 32

typedef struct {
    int nf;
    int nv[ORC_FCAP3];
    int32_t tag[ORC_FCAP3];
    double v[ORC_FCAP3][ORC_VCAP3][3];
} orc_poly3;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static int lex_less3(const double *a, const double *b)
{
    if (a[0] != b[0]) return a[0] < b[0];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[2] < b[2];
}

/* pseudo-angle in [0, 4) of (dx, dy), increasing with the polar angle */
static double diamond_angle(double dx, double dy)
{
    if (dy >= 0.0) return dx >= 0.0 ? dy / (dx + dy) : 1.0 - dx / (-dx + dy);
    return dx < 0.0 ? 2.0 - dy / (-dx - dy) : 3.0 + dx / (dx - dy);
}

static void box_poly3(orc_poly3 *P, const double *lo, const double *hi, const int32_t *t)
{
    /* corner (b0,b1,b2) with b = 0 for lo, 1 for hi; faces -x,+x,-y,+y,-z,+z */
    static const int fc[6][4][3] = {
        {{0, 0, 0}, {0, 0, 1}, {0, 1, 1}, {0, 1, 0}}, {{1, 0, 0}, {1, 1, 0}, {1, 1, 1}, {1, 0, 1}},
        {{0, 0, 0}, {1, 0, 0}, {1, 0, 1}, {0, 0, 1}}, {{0, 1, 0}, {0, 1, 1}, {1, 1, 1}, {1, 1, 0}},
        {{0, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, 0, 0}}, {{0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}}};
    P->nf = 6;
    for (int f = 0; f < 6; ++f) {
        P->nv[f] = 4;
        P->tag[f] = t[f];
        for (int k = 0; k < 4; ++k)
            for (int a = 0; a < 3; ++a) P->v[f][k][a] = fc[f][k][a] ? hi[a] : lo[a];
    }
}

/* Clip P by { y : nrm . y - off <= 0 }; the new face gets newtag.  Returns 0,
 * or -1 when a capacity is exceeded.  tmp is scratch of the same size.     */
static int clip_poly3(orc_poly3 *P, orc_poly3 *tmp, const double *nrm, double off, int32_t newtag)
{
    int any_out = 0;
    for (int f = 0; f < P->nf; ++f)
        for (int k = 0; k < P->nv[f]; ++k)
            if (dot3(nrm, P->v[f][k]) - off > 0.0) any_out = 1;
    if (!any_out) return 0;
    double cuts[4 * ORC_VCAP3][3];
    int ncut = 0;
    tmp->nf = 0;
    for (int f = 0; f < P->nf; ++f) {
        int nv = P->nv[f], no = 0;
        double(*out)[3] = tmp->v[tmp->nf];
        for (int k = 0; k < nv; ++k) {
            const double *A = P->v[f][k], *B = P->v[f][(k + 1) % nv];
            double sa = dot3(nrm, A) - off, sb = dot3(nrm, B) - off;
            if (sa <= 0.0) {
                if (no >= ORC_VCAP3) return -1;
                memcpy(out[no++], A, sizeof(double) * 3);
                if (sa == 0.0) {
                    if (ncut >= 4 * ORC_VCAP3) return -1;
                    memcpy(cuts[ncut++], A, sizeof(double) * 3);
                }
            }
            if ((sa < 0.0 && sb > 0.0) || (sa > 0.0 && sb < 0.0)) {
                const double *I = sa < 0.0 ? A : B, *O = sa < 0.0 ? B : A;   /* kept end, removed end */
                double si = sa < 0.0 ? sa : sb, so = sa < 0.0 ? sb : sa;
                double t = si / (si - so);
                double c[3] = {I[0] + t * (O[0] - I[0]), I[1] + t * (O[1] - I[1]), I[2] + t * (O[2] - I[2])};
                if (no >= ORC_VCAP3 || ncut >= 4 * ORC_VCAP3) return -1;
                memcpy(out[no++], c, sizeof(c));
                memcpy(cuts[ncut++], c, sizeof(c));
            }
        }
        if (no >= 3) {
            tmp->nv[tmp->nf] = no;
            tmp->tag[tmp->nf] = P->tag[f];
            tmp->nf++;
        }
    }
    /* the new face: sort the cut points, drop duplicates, order by angle */
    for (int a = 1; a < ncut; ++a)
        for (int b = a; b > 0 && lex_less3(cuts[b], cuts[b - 1]); --b) {
            double s[3];
            memcpy(s, cuts[b], sizeof(s));
            memcpy(cuts[b], cuts[b - 1], sizeof(s));
            memcpy(cuts[b - 1], s, sizeof(s));
        }
    int nu = 0;
    for (int a = 0; a < ncut; ++a)
        if (nu == 0 || memcmp(cuts[a], cuts[nu - 1], sizeof(double) * 3) != 0) memcpy(cuts[nu++], cuts[a], sizeof(double) * 3);
    if (nu >= 3) {
        if (tmp->nf >= ORC_FCAP3 || nu > ORC_VCAP3) return -1;
        double g[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < nu; ++a)
            for (int d = 0; d < 3; ++d) g[d] += cuts[a][d];
        for (int d = 0; d < 3; ++d) g[d] /= nu;
        int ax = 0;   /* axis least aligned with the normal (first on ties) */
        for (int d = 1; d < 3; ++d)
            if (fabs(nrm[d]) < fabs(nrm[ax])) ax = d;
        double e[3] = {0.0, 0.0, 0.0}, u[3], v[3];
        e[ax] = 1.0;
        cross3(nrm, e, u);
        cross3(nrm, u, v);
        double ang[4 * ORC_VCAP3];
        for (int a = 0; a < nu; ++a) {
            double r[3] = {cuts[a][0] - g[0], cuts[a][1] - g[1], cuts[a][2] - g[2]};
            ang[a] = diamond_angle(dot3(u, r), dot3(v, r));
        }
        /* stable insertion sort by angle (ties keep lexicographic order) */
        int ord[4 * ORC_VCAP3];
        for (int a = 0; a < nu; ++a) ord[a] = a;
        for (int a = 1; a < nu; ++a)
            for (int b = a; b > 0 && ang[ord[b]] < ang[ord[b - 1]]; --b) {
                int s = ord[b]; ord[b] = ord[b - 1]; ord[b - 1] = s;
            }
        for (int a = 0; a < nu; ++a) memcpy(tmp->v[tmp->nf][a], cuts[ord[a]], sizeof(double) * 3);
        tmp->nv[tmp->nf] = nu;
        tmp->tag[tmp->nf] = newtag;
        tmp->nf++;
    }
    memcpy(P, tmp, sizeof(*P));
    return 0;
}

typedef struct {
    double d2;
    int32_t j;
} nb_dist;

static int cmp_nb_dist(const void *a, const void *b)
{
    const nb_dist *p = (const nb_dist *)a, *q = (const nb_dist *)b;
    if (p->d2 != q->d2) return p->d2 < q->d2 ? -1 : 1;
    return (p->j > q->j) - (p->j < q->j);
}

/* Cells of the points listed in ids[0..m) (all points when ids is NULL and
 * m = n).  Outputs per listed cell k: nf[k] faces, fnv[k][f], fverts[k][f][v][3],
 * ftags[k][f], volume V[k] (sum of the tetrahedra x_i, v_0, v_k, v_k+1 of
 * every face fan) and rho[k] = max |v - x_i|.  fcap/vcap are the caller's
 * capacities.  Returns the number of cells that failed (capacity).          */
int64_t orc_cells3d(int64_t n, const double *x, const double *R, const int64_t *off, const int32_t *idx,
                    const double *dom_lo, const double *dom_hi, int64_t m, const int64_t *ids, int fcap,
                    int vcap, int32_t *nf_out, int32_t *fnv, double *fverts, int32_t *ftags, double *V,
                    double *rho)
{
    (void)n;
    orc_poly3 *P = (orc_poly3 *)malloc(sizeof(orc_poly3)), *T = (orc_poly3 *)malloc(sizeof(orc_poly3));
    nb_dist *ord = NULL;
    int64_t ordcap = 0;
    int64_t bad = 0;
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = ids ? ids[k] : k;
        const double *xi = x + 3 * i;
        double lo[3], hi[3];
        int32_t t[6];
        for (int a = 0; a < 3; ++a) {
            lo[a] = xi[a] - R[i]; hi[a] = xi[a] + R[i];
            t[2 * a] = ORC_TAG_BOX; t[2 * a + 1] = ORC_TAG_BOX;
            if (lo[a] <= dom_lo[a]) { lo[a] = dom_lo[a]; t[2 * a] = -1 - 2 * a; }
            if (hi[a] >= dom_hi[a]) { hi[a] = dom_hi[a]; t[2 * a + 1] = -2 - 2 * a; }
        }
        box_poly3(P, lo, hi, t);
        /* neighbours nearest first, ties by index */
        int64_t cnt = off[i + 1] - off[i];
        if (cnt > ordcap) {
            ordcap = cnt;
            ord = (nb_dist *)realloc(ord, sizeof(nb_dist) * ordcap);
        }
        for (int64_t p = 0; p < cnt; ++p) {
            int32_t j = idx[off[i] + p];
            double d[3] = {x[3 * (int64_t)j] - xi[0], x[3 * (int64_t)j + 1] - xi[1], x[3 * (int64_t)j + 2] - xi[2]};
            ord[p].d2 = dot3(d, d);
            ord[p].j = j;
        }
        qsort(ord, (size_t)cnt, sizeof(nb_dist), cmp_nb_dist);
        int ok = 1;
        for (int64_t p = 0; p < cnt; ++p) {
            int32_t j = ord[p].j;
            const double *xj = x + 3 * (int64_t)j;
            double nrm[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
            double mid[3] = {0.5 * (xi[0] + xj[0]), 0.5 * (xi[1] + xj[1]), 0.5 * (xi[2] + xj[2])};
            if (clip_poly3(P, T, nrm, dot3(nrm, mid), j) != 0) { ok = 0; break; }
        }
        if (ok && (P->nf > fcap)) ok = 0;
        for (int f = 0; ok && f < P->nf; ++f)
            if (P->nv[f] > vcap) ok = 0;
        if (!ok || P->nf < 4) {
            bad++;
            nf_out[k] = 0; V[k] = 0.0; rho[k] = 0.0;
            continue;
        }
        double vol = 0.0, r2 = 0.0;
        nf_out[k] = P->nf;
        for (int f = 0; f < P->nf; ++f) {
            fnv[k * fcap + f] = P->nv[f];
            ftags[k * fcap + f] = P->tag[f];
            for (int q = 0; q < P->nv[f]; ++q) {
                double d[3] = {P->v[f][q][0] - xi[0], P->v[f][q][1] - xi[1], P->v[f][q][2] - xi[2]};
                if (dot3(d, d) > r2) r2 = dot3(d, d);
                memcpy(fverts + ((k * fcap + f) * vcap + q) * 3, P->v[f][q], sizeof(double) * 3);
            }
            double e1[3] = {P->v[f][0][0] - xi[0], P->v[f][0][1] - xi[1], P->v[f][0][2] - xi[2]};
            for (int q = 1; q + 1 < P->nv[f]; ++q) {
                double e2[3], e3[3], c[3];
                for (int a = 0; a < 3; ++a) { e2[a] = P->v[f][q][a] - xi[a]; e3[a] = P->v[f][q + 1][a] - xi[a]; }
                cross3(e2, e3, c);
                vol += dot3(e1, c) / 6.0;
            }
        }
        V[k] = vol;
        rho[k] = sqrt(r2);
    }
    free(P); free(T); free(ord);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Cubic B-spline base kernel (reading of the unnamed W^b of Sec. 2.1),
 * q = |y - x_j| / h_j with h_j = R_j / 2, support q < 2.  The
 * normalisation constant cancels in the RK functions and is omitted.
 * Returns W and fills dW = grad_y W.                                        */
/* ------------------------------------------------------------------------ */
static double kernel_w(int dim, const double *y, const double *xj, double Rj, double *dW)
{
    double h = 0.5 * Rj;
    double r[ORC_MAXD], r2 = 0.0;
    for (int a = 0; a < dim; ++a) { r[a] = y[a] - xj[a]; r2 += r[a] * r[a]; }
    double q = sqrt(r2) / h;
    double w, dwq_over_q;  /* W(q) and W'(q)/q */
    if (q < 1.0) {
        w = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
        dwq_over_q = -3.0 + 2.25 * q;
    } else if (q < 2.0) {
        double t = 2.0 - q;
        w = 0.25 * t * t * t;
        dwq_over_q = -0.75 * t * t / q;
    } else {
        w = 0.0;
        dwq_over_q = 0.0;
    }
    /* grad_y W = W'(q) dq/dy = W'(q) (y - x_j) / (q h^2) */
    for (int a = 0; a < dim; ++a) dW[a] = dwq_over_q * r[a] / (h * h);
    return w;
}

/* Monomial basis P(z) = [1, z^a, z^a z^b (a <= b)] of total degree <= order,
 * and its derivatives dP/dz^g.  Returns the basis size.                    */
static int basis_size(int dim, int order)
{
    if (order == 0) return 1;
    if (order == 1) return 1 + dim;
    return (dim + 1) * (dim + 2) / 2;
}

static void basis_eval(int dim, int order, const double *z, double *P, double dP[][ORC_MAXB])
{
    int b = basis_size(dim, order);
    for (int k = 0; k < b; ++k) {
        P[k] = 0.0;
        for (int g = 0; g < dim; ++g) dP[g][k] = 0.0;
    }
    P[0] = 1.0;
    if (order >= 1)
        for (int a = 0; a < dim; ++a) {
            P[1 + a] = z[a];
            dP[a][1 + a] = 1.0;
        }
    if (order >= 2) {
        int k = 1 + dim;
        for (int a = 0; a < dim; ++a)
            for (int c = a; c < dim; ++c) {
                P[k] = z[a] * z[c];
                dP[a][k] += z[c];
                dP[c][k] += z[a];
                k++;
            }
    }
}

/* Cholesky factorisation M = L L^T in place (lower triangle).  Returns 0 on
 * success, -1 when a pivot falls below rel_tol * max diag(M).               */
static int cholesky(int b, double M[][ORC_MAXB], double rel_tol)
{
    double dmax = 0.0;
    for (int k = 0; k < b; ++k) if (M[k][k] > dmax) dmax = M[k][k];
    if (!(dmax > 0.0)) return -1;
    for (int k = 0; k < b; ++k) {
        double s = M[k][k];
        for (int p = 0; p < k; ++p) s -= M[k][p] * M[k][p];
        if (!(s > rel_tol * dmax)) return -1;
        M[k][k] = sqrt(s);
        for (int r = k + 1; r < b; ++r) {
            double t = M[r][k];
            for (int p = 0; p < k; ++p) t -= M[r][p] * M[k][p];
            M[r][k] = t / M[k][k];
        }
    }
    return 0;
}

static void chol_solve(int b, double L[][ORC_MAXB], const double *rhs, double *out)
{
    double t[ORC_MAXB];
    for (int k = 0; k < b; ++k) {
        double s = rhs[k];
        for (int p = 0; p < k; ++p) s -= L[k][p] * t[p];
        t[k] = s / L[k][k];
    }
    for (int k = b - 1; k >= 0; --k) {
        double s = t[k];
        for (int p = k + 1; p < b; ++p) s -= L[p][k] * out[p];
        out[k] = s / L[k][k];
    }
}

/* RK functions at point y (Sec. 2.2).  Candidates cand[0..nc) are the points
 * whose kernel might cover y; those with W_j(y) = 0 get N = dN = 0.  The
 * monomials are taken in the scaled argument z = (y - x_j) / hs; this
 * diagonal change of basis leaves U_j unchanged and only improves the
 * conditioning of M.  Output N_j = V_j U_j and dN_j = V_j grad U_j.  When a
 * Cholesky pivot of M falls below 1e-6 of the largest diagonal entry, the
 * order drops by one and the evaluation is repeated (reading for the singular
 * case the paper leaves open; the bound keeps the condition number of M near
 * 1e6 so that the RK functions stay accurate to about 1e-10).  Returns the
 * order used, or -1 when even order 0 fails (no kernel covers y).          */
#define ORC_PIVOT_TOL 1e-6

static int rk_eval_act(int dim, int order, const double *y, int nc, const int32_t *cand, const double *x,
                       const double *R, const double *V, double hs, double *N, double *dN, unsigned char *act)
{
    for (int ord = order; ord >= 0; --ord) {
        int b = basis_size(dim, ord);
        double M[ORC_MAXB][ORC_MAXB], dM[ORC_MAXD][ORC_MAXB][ORC_MAXB];
        memset(M, 0, sizeof(M));
        memset(dM, 0, sizeof(dM));
        for (int c = 0; c < nc; ++c) {
            const double *xj = x + (int64_t)cand[c] * dim;
            double dW[ORC_MAXD];
            double W = kernel_w(dim, y, xj, R[cand[c]], dW);
            if (W == 0.0) continue;
            double z[ORC_MAXD], P[ORC_MAXB], dPz[ORC_MAXD][ORC_MAXB];
            for (int a = 0; a < dim; ++a) z[a] = (y[a] - xj[a]) / hs;
            basis_eval(dim, ord, z, P, dPz);
            double Vj = V[cand[c]];
            for (int r = 0; r < b; ++r)
                for (int s = 0; s < b; ++s) {
                    M[r][s] += Vj * P[r] * P[s] * W;
                    for (int g = 0; g < dim; ++g)
                        dM[g][r][s] += Vj * ((dPz[g][r] / hs * P[s] + P[r] * dPz[g][s] / hs) * W +
                                             P[r] * P[s] * dW[g]);
                }
        }
        double L[ORC_MAXB][ORC_MAXB];
        memcpy(L, M, sizeof(M));
        if (cholesky(b, L, ORC_PIVOT_TOL) != 0) continue;
        double G[ORC_MAXB] = {0}, C[ORC_MAXB], dC[ORC_MAXD][ORC_MAXB];
        G[0] = 1.0;
        chol_solve(b, L, G, C);                        /* C = M^-1 G        */
        for (int g = 0; g < dim; ++g) {                /* dC = -M^-1 dM C   */
            double t[ORC_MAXB];
            for (int r = 0; r < b; ++r) {
                double s = 0.0;
                for (int q = 0; q < b; ++q) s += dM[g][r][q] * C[q];
                t[r] = -s;
            }
            chol_solve(b, L, t, dC[g]);
        }
        for (int c = 0; c < nc; ++c) {
            const double *xj = x + (int64_t)cand[c] * dim;
            double dW[ORC_MAXD];
            double W = kernel_w(dim, y, xj, R[cand[c]], dW);
            if (W == 0.0) {
                N[c] = 0.0;
                for (int g = 0; g < dim; ++g) dN[c * dim + g] = 0.0;
                if (act) act[c] = 0;
                continue;
            }
            if (act) act[c] = 1;
            double z[ORC_MAXD], P[ORC_MAXB], dPz[ORC_MAXD][ORC_MAXB];
            for (int a = 0; a < dim; ++a) z[a] = (y[a] - xj[a]) / hs;
            basis_eval(dim, ord, z, P, dPz);
            double PC = 0.0;
            for (int r = 0; r < b; ++r) PC += P[r] * C[r];
            double Vj = V[cand[c]];
            N[c] = Vj * PC * W;                        /* U_j = P_j^T C W_j */
            for (int g = 0; g < dim; ++g) {
                double t1 = 0.0, t2 = 0.0;
                for (int r = 0; r < b; ++r) {
                    t1 += dPz[g][r] / hs * C[r];
                    t2 += P[r] * dC[g][r];
                }
                dN[c * dim + g] = Vj * ((t1 + t2) * W + PC * dW[g]);
            }
        }
        return ord;
    }
    for (int c = 0; c < nc; ++c) {
        N[c] = 0.0;
        for (int g = 0; g < dim; ++g) dN[c * dim + g] = 0.0;
        if (act) act[c] = 0;
    }
    return -1;
}

int orc_rk_eval(int dim, int order, const double *y, int nc, const int32_t *cand, const double *x,
                const double *R, const double *V, double hs, double *N, double *dN)
{
    return rk_eval_act(dim, order, y, nc, cand, x, R, V, hs, N, dN, NULL);
}

/* ------------------------------------------------------------------------ */
/* Meshless integration (Sec. 3.2, Alg. 1).  Blocks over the overlap pattern
 * (rows = test function i, columns = trial function j; row i of the pattern
 * holds i and its neighbours in increasing order):
 *   Mass_g[i,j] = <N_i, N_j>        over material-g quadrature points
 *   D^a_g[i,j]  = <d^a N_i, N_j>    over material-g quadrature points
 *   K^ab[i,j]   = <d^a N_i, d^b N_j>
 *   S_f[i,j]    = (N_i, N_j) on domain face f
 * with N_i = V_i U_i (the test function U_i scaled by V_i, so that Mass is
 * symmetric).  Block order: for g: Mass_g, D^0_g..D^{d-1}_g; then K^ab with
 * a-major order; then S_0..S_{2d-1}.                                        */
/* ------------------------------------------------------------------------ */
int orc_num_blocks(int dim, int n_mat) { return n_mat * (1 + dim) + dim * dim + 2 * dim; }

static int64_t find_pos(const int64_t *row_off, const int32_t *col, int64_t i, int32_t j)
{
    int64_t lo = row_off[i], hi = row_off[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] == j) return mid;
        if (col[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int material_at(int dim, const double *y, int n_regions, const double *reg_lo,
                       const double *reg_hi, const int32_t *reg_mat)
{
    int m = 0;
    for (int r = 0; r < n_regions; ++r) {
        int in = 1;
        for (int a = 0; a < dim; ++a)
            if (y[a] < reg_lo[r * dim + a] || y[a] > reg_hi[r * dim + a]) in = 0;
        if (in) m = reg_mat[r];
    }
    return m;
}

typedef struct {
    int dim, rk_order, n_mat;
    int64_t n;
    const double *x, *R, *V;
    const int64_t *nb_off;
    const int32_t *nb_idx;
    const int64_t *row_off;
    const int32_t *col;
    int64_t nnz;
    int n_regions;
    const double *reg_lo, *reg_hi;
    const int32_t *reg_mat;
    double *blocks;             /* [nblk][nnz] */
    int64_t fallbacks, missing;
    int n_fields;               /* smooth material fields (may be 0) */
    const double *field_par;    /* [n_fields][4]: a, b, k, phase */
    const int32_t *field_mat;   /* [n_fields] material that receives the field */
    int n_shells;               /* spherical shells (may be 0) */
    const double *shell_par;    /* [n_shells][dim + 2]: centre, inner radius, outer radius */
    const int32_t *shell_mat;   /* [n_shells] material inside the shell */
} integ_ctx;

/* Material fractions f[0..n_mat) at y.  Box regions give an indicator (last
 * match wins, material 0 elsewhere).  Each smooth field r then moves
 *   v_r(y) = a + b prod_alpha cos(k y_alpha + phase)
 * from material 0 to material field_mat[r], so the fractions still sum to
 * one.  With one material per cross-section component this represents the
 * spatially varying opacities of the manufactured problems (Sec. 5.1), whose
 * products of sines and cosines are cosines with a phase. */
static void material_fractions(const integ_ctx *ic, const double *y, double *f)
{
    for (int g = 0; g < ic->n_mat; ++g) f[g] = 0.0;
    int m = material_at(ic->dim, y, ic->n_regions, ic->reg_lo, ic->reg_hi, ic->reg_mat);
    /* shells (annuli in 2D, such as the asteroid of Sec. 5.4) after the boxes, last match wins */
    for (int r = 0; r < ic->n_shells; ++r) {
        const double *sp = ic->shell_par + (ic->dim + 2) * r;
        double d2 = 0.0;
        for (int a = 0; a < ic->dim; ++a) d2 += (y[a] - sp[a]) * (y[a] - sp[a]);
        const double d = sqrt(d2);
        if (d >= sp[ic->dim] && d <= sp[ic->dim + 1]) m = ic->shell_mat[r];
    }
    f[m] = 1.0;
    for (int r = 0; r < ic->n_fields; ++r) {
        const double *fp = ic->field_par + 4 * r;
        double pr = 1.0;
        for (int a = 0; a < ic->dim; ++a) pr *= cos(fp[2] * y[a] + fp[3]);
        const double v = fp[0] + fp[1] * pr;
        f[ic->field_mat[r]] += v;
        f[0] -= v;
    }
}

/* Candidate functions for a cell c: c itself and its overlap neighbours
 * (the doubled-radius argument of Sec. 3.4). */
static int cell_candidates(const integ_ctx *ic, int64_t c, int32_t *cand)
{
    int nc = 0;
    cand[nc++] = (int32_t)c;
    for (int64_t p = ic->nb_off[c]; p < ic->nb_off[c + 1]; ++p) cand[nc++] = ic->nb_idx[p];
    return nc;
}

/* Accumulate one volume quadrature point of weight w (already mapped by |J|). */
static void add_volume_point(integ_ctx *ic, int64_t c, const double *y, double w, int nc,
                             const int32_t *cand, const int64_t *pos, double *N, double *dN,
                             unsigned char *act)
{
    int dim = ic->dim;
    int ord = rk_eval_act(dim, ic->rk_order, y, nc, cand, ic->x, ic->R, ic->V, 0.5 * ic->R[c], N, dN, act);
    if (ord < 0) return;
    if (ord < ic->rk_order) ic->fallbacks++;
    double f[8];
    material_fractions(ic, y, f);
    int64_t nnz = ic->nnz;
    for (int a = 0; a < nc; ++a) {
        if (!act[a]) continue;
        for (int b = 0; b < nc; ++b) {
            if (!act[b]) continue;
            int64_t p = pos[a * nc + b];
            if (p < 0) { ic->missing++; continue; }
            for (int g = 0; g < ic->n_mat; ++g) {
                if (f[g] == 0.0) continue;
                const double wg = w * f[g];
                ic->blocks[(int64_t)(g * (1 + dim)) * nnz + p] += wg * N[a] * N[b];
                for (int al = 0; al < dim; ++al)
                    ic->blocks[(int64_t)(g * (1 + dim) + 1 + al) * nnz + p] += wg * dN[a * dim + al] * N[b];
            }
            int kb = ic->n_mat * (1 + dim);
            for (int al = 0; al < dim; ++al)
                for (int be = 0; be < dim; ++be)
                    ic->blocks[(int64_t)(kb + al * dim + be) * nnz + p] +=
                        w * dN[a * dim + al] * dN[b * dim + be];
        }
    }
}

typedef struct {
    int64_t count, cap;
    double *y;        /* [cap][dim] */
    int32_t *face;    /* [cap] */
    double *w;        /* [cap] */
    int kmax;
    int32_t *nact;    /* [cap] */
    int32_t *act;     /* [cap][kmax] */
    double *Nv;       /* [cap][kmax] */
} bq_out;

static void add_surface_point(integ_ctx *ic, int64_t c, const double *y, double w, int face, int nc,
                              const int32_t *cand, const int64_t *pos, double *N, double *dN,
                              unsigned char *act, bq_out *bo)
{
    int dim = ic->dim;
    int ord = rk_eval_act(dim, ic->rk_order, y, nc, cand, ic->x, ic->R, ic->V, 0.5 * ic->R[c], N, dN, act);
    if (ord < 0) return;
    if (ord < ic->rk_order) ic->fallbacks++;
    int64_t nnz = ic->nnz;
    int sb = ic->n_mat * (1 + dim) + dim * dim + face;
    for (int a = 0; a < nc; ++a) {
        if (!act[a]) continue;
        for (int b = 0; b < nc; ++b) {
            if (!act[b]) continue;
            int64_t p = pos[a * nc + b];
            if (p < 0) { ic->missing++; continue; }
            ic->blocks[(int64_t)sb * nnz + p] += w * N[a] * N[b];
        }
    }
    if (bo && bo->y) {
        int64_t k = bo->count;
        if (k < bo->cap) {
            for (int a = 0; a < dim; ++a) bo->y[k * dim + a] = y[a];
            bo->face[k] = face;
            bo->w[k] = w;
            int na = 0;
            for (int a = 0; a < nc && na < bo->kmax; ++a)
                if (act[a]) {
                    bo->act[k * bo->kmax + na] = cand[a];
                    bo->Nv[k * bo->kmax + na] = N[a];
                    na++;
                }
            bo->nact[k] = na;
        }
    }
    bo->count++;
}

/* 2D integration: each cell is split into the fan of triangles (x_c, v_k,
 * v_k+1) (Fig. 2); the reference triangle {xi >= 0, xi0 + xi1 <= 1} is mapped
 * by x = p0 + (p_a - p0) xi^a with |J| = twice the area (App. A).  Cell edges
 * on domain face f get the line rule mapped from [-1,1] with K = half the
 * edge length.  Also returns E[p] = N_j(x_i) on the pattern (the point values
 * of Eq. flux-expansion), evaluated with the cell of x_i.                   */
int64_t orc_integrate2d(integ_ctx *ic_in, int cap, const int32_t *nv, const double *verts,
                        const int32_t *tags, int nq_tri, const double *tri_pts, const double *tri_w,
                        int nq_seg, const double *seg_pts, const double *seg_w, double *E,
                        int64_t bq_cap, int kmax, double *bq_y, int32_t *bq_face, double *bq_w,
                        int32_t *bq_nact, int32_t *bq_act, double *bq_N, int64_t *stats)
{
    integ_ctx ic = *ic_in;
    ic.fallbacks = 0;
    ic.missing = 0;
    int64_t n = ic.n;
    int maxc = 1;
    for (int64_t c = 0; c < n; ++c) {
        int k = (int)(ic.nb_off[c + 1] - ic.nb_off[c]) + 1;
        if (k > maxc) maxc = k;
    }
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * maxc);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * maxc * maxc);
    double *N = (double *)malloc(sizeof(double) * maxc);
    double *dN = (double *)malloc(sizeof(double) * maxc * 2);
    unsigned char *act = (unsigned char *)malloc(maxc);
    bq_out bo = {0, bq_cap, bq_y, bq_face, bq_w, kmax, bq_nact, bq_act, bq_N};
    for (int64_t c = 0; c < n; ++c) {
        int nc = cell_candidates(&ic, c, cand);
        for (int a = 0; a < nc; ++a)
            for (int b = 0; b < nc; ++b) pos[a * nc + b] = find_pos(ic.row_off, ic.col, cand[a], cand[b]);
        const double *xc = ic.x + 2 * c;
        int m = nv[c];
        for (int k = 0; k < m; ++k) {
            const double *P = verts + (c * cap + k) * 2;
            const double *Q = verts + (c * cap + (k + 1) % m) * 2;
            double e1[2] = {P[0] - xc[0], P[1] - xc[1]}, e2[2] = {Q[0] - xc[0], Q[1] - xc[1]};
            double detJ = e1[0] * e2[1] - e1[1] * e2[0];   /* = 2 * area (CCW) */
            if (detJ > 0.0) {
                for (int q = 0; q < nq_tri; ++q) {
                    double y[2] = {xc[0] + e1[0] * tri_pts[2 * q] + e2[0] * tri_pts[2 * q + 1],
                                   xc[1] + e1[1] * tri_pts[2 * q] + e2[1] * tri_pts[2 * q + 1]};
                    add_volume_point(&ic, c, y, tri_w[q] * detJ, nc, cand, pos, N, dN, act);
                }
            }
            int t = tags[c * cap + k];
            if (t <= -1 && t >= -4) {
                int face = -1 - t;
                double len = sqrt((Q[0] - P[0]) * (Q[0] - P[0]) + (Q[1] - P[1]) * (Q[1] - P[1]));
                for (int q = 0; q < nq_seg; ++q) {
                    double s = 0.5 * (seg_pts[q] + 1.0);
                    double y[2] = {P[0] + (Q[0] - P[0]) * s, P[1] + (Q[1] - P[1]) * s};
                    add_surface_point(&ic, c, y, seg_w[q] * 0.5 * len, face, nc, cand, pos, N, dN, act, &bo);
                }
            }
        }
        /* point values at the generator x_c */
        if (E) {
            int ord = rk_eval_act(2, ic.rk_order, xc, nc, cand, ic.x, ic.R, ic.V, 0.5 * ic.R[c], N, dN, act);
            if (ord >= 0) {
                if (ord < ic.rk_order) ic.fallbacks++;
                for (int a = 0; a < nc; ++a) {
                    if (!act[a]) continue;
                    int64_t p = pos[0 * nc + a];
                    if (p < 0) { ic.missing++; continue; }
                    E[p] = N[a];
                }
            }
        }
    }
    free(cand); free(pos); free(N); free(dN); free(act);
    stats[0] = ic.fallbacks;
    stats[1] = ic.missing;
    stats[2] = bo.count;
    return bo.count;
}

/* 3D integration: every face of cell c is fan-triangulated from its vertex 0
 * and each triangle is joined to the generator x_c, giving the tetrahedra
 * (x_c, v_0, v_k, v_k+1) (Fig. 2 in three dimensions).  The reference
 * tetrahedron {xi >= 0, xi0 + xi1 + xi2 <= 1} maps by
 * x = x_c + (v_0 - x_c) xi0 + (v_k - x_c) xi1 + (v_k+1 - x_c) xi2, |J| = 6 x
 * volume (App. A).  Domain faces get the triangle rule on each fan triangle
 * (v_0, v_k, v_k+1) with |J| = twice its area.  E as in 2D.               */
int64_t orc_integrate3d(integ_ctx *ic_in, int fcap, int vcap, const int32_t *nf, const int32_t *fnv,
                        const double *fverts, const int32_t *ftags, int nq_tet, const double *tet_pts,
                        const double *tet_w, int nq_tri, const double *tri_pts, const double *tri_w, double *E,
                        int64_t bq_cap, int kmax, double *bq_y, int32_t *bq_face, double *bq_w,
                        int32_t *bq_nact, int32_t *bq_act, double *bq_N, int64_t *stats)
{
    integ_ctx ic = *ic_in;
    ic.fallbacks = 0;
    ic.missing = 0;
    int64_t n = ic.n;
    int maxc = 1;
    for (int64_t c = 0; c < n; ++c) {
        int k = (int)(ic.nb_off[c + 1] - ic.nb_off[c]) + 1;
        if (k > maxc) maxc = k;
    }
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * maxc);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * maxc * maxc);
    double *N = (double *)malloc(sizeof(double) * maxc);
    double *dN = (double *)malloc(sizeof(double) * maxc * 3);
    unsigned char *act = (unsigned char *)malloc(maxc);
    bq_out bo = {0, bq_cap, bq_y, bq_face, bq_w, kmax, bq_nact, bq_act, bq_N};
    for (int64_t c = 0; c < n; ++c) {
        int nc = cell_candidates(&ic, c, cand);
        for (int a = 0; a < nc; ++a)
            for (int b = 0; b < nc; ++b) pos[a * nc + b] = find_pos(ic.row_off, ic.col, cand[a], cand[b]);
        const double *xc = ic.x + 3 * c;
        for (int f = 0; f < nf[c]; ++f) {
            int m = fnv[c * fcap + f];
            const double *fv = fverts + (c * fcap + f) * vcap * 3;
            int t = ftags[c * fcap + f];
            for (int k = 1; k + 1 < m; ++k) {
                const double *A = fv, *B = fv + 3 * k, *Cv = fv + 3 * (k + 1);
                double e1[3], e2[3], e3[3], cr[3];
                for (int a = 0; a < 3; ++a) { e1[a] = A[a] - xc[a]; e2[a] = B[a] - xc[a]; e3[a] = Cv[a] - xc[a]; }
                cross3(e2, e3, cr);
                double detJ = dot3(e1, cr);
                if (detJ > 0.0) {
                    for (int q = 0; q < nq_tet; ++q) {
                        const double *xi = tet_pts + 3 * q;
                        double y[3];
                        for (int a = 0; a < 3; ++a) y[a] = xc[a] + e1[a] * xi[0] + e2[a] * xi[1] + e3[a] * xi[2];
                        add_volume_point(&ic, c, y, tet_w[q] * detJ, nc, cand, pos, N, dN, act);
                    }
                }
                if (t <= -1 && t >= -6) {
                    int face = -1 - t;
                    double g1[3], g2[3], nn[3];
                    for (int a = 0; a < 3; ++a) { g1[a] = B[a] - A[a]; g2[a] = Cv[a] - A[a]; }
                    cross3(g1, g2, nn);
                    double area2 = sqrt(dot3(nn, nn));
                    for (int q = 0; q < nq_tri; ++q) {
                        const double *xi = tri_pts + 2 * q;
                        double y[3];
                        for (int a = 0; a < 3; ++a) y[a] = A[a] + g1[a] * xi[0] + g2[a] * xi[1];
                        add_surface_point(&ic, c, y, tri_w[q] * area2, face, nc, cand, pos, N, dN, act, &bo);
                    }
                }
            }
        }
        if (E) {
            int ord = rk_eval_act(3, ic.rk_order, xc, nc, cand, ic.x, ic.R, ic.V, 0.5 * ic.R[c], N, dN, act);
            if (ord >= 0) {
                if (ord < ic.rk_order) ic.fallbacks++;
                for (int a = 0; a < nc; ++a) {
                    if (!act[a]) continue;
                    int64_t p = pos[0 * nc + a];
                    if (p < 0) { ic.missing++; continue; }
                    E[p] = N[a];
                }
            }
        }
    }
    free(cand); free(pos); free(N); free(dN); free(act);
    stats[0] = ic.fallbacks;
    stats[1] = ic.missing;
    stats[2] = bo.count;
    return bo.count;
}

/* ------------------------------------------------------------------------ */
/* Operators of Sec. 4.2, applied for one ordinate m from the blocks.
 *   (L psi)_i  = sum_j [ a0 <N_i,N_j> + a0 tau_i W.<dN_i,N_j>
 *                       + sum_f max(0, W.n_f) (N_i,N_j)_f - W.<dN_i,N_j>
 *                       + tau_i W^a W^b <d^a N_i, d^b N_j>
 *                       + <N_i sigma_t N_j> + tau_i W.<dN_i sigma_t N_j> ] psi_j
 *   (T psi)_i  = sum_j [ a0 <N_i,N_j> + a0 tau_i W.<dN_i,N_j> ] psi_j
 *   (MS phi)_i = 1/(4 pi) sum_j [ <N_i sigma_s N_j> + tau_i W.<dN_i sigma_s N_j> ] phi_j
 *   source     = sum_j [ <N_i,N_j> + tau_i W.<dN_i,N_j> ] q_j   (q expanded in the basis)
 * with W = Omega_m, a0 = 1/(c dt), and f running over the domain faces whose
 * outward normal n_f satisfies W.n_f > 0 (outflow).                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim, n_mat, n_ord;
    int64_t n, nnz;
    const int64_t *row_off;
    const int32_t *col;
    const double *blocks;
    const double *omega;   /* [M][dim] */
    const double *wq;      /* [M] */
    const double *sig_t, *sig_s;
    double a0;
    const double *tau;     /* [n] */
    /* boundary quadrature points for the inflow term */
    int64_t nbq;
    int kmax;
    const int32_t *bq_face;
    const double *bq_w;
    const int32_t *bq_nact, *bq_act;
    const double *bq_N;
    /* solver settings */
    double tol_in, tol_out;
    int restart_in, restart_out, max_in, max_out;
    /* right preconditioner of the inner solves: 0 point Jacobi, 1 patch
     * block Jacobi over the spatial patches below (needs x and the box) */
    int precond;
    const double *x;
    const double *dom_lo, *dom_hi;
} op_ctx;

static const double face_normal[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

static double blk(const op_ctx *o, int b, int64_t p) { return o->blocks[(int64_t)b * o->nnz + p]; }

static double L_entry(const op_ctx *o, int m, int64_t i, int64_t p)
{
    int dim = o->dim, G = o->n_mat;
    const double *W = o->omega + m * dim;
    double tau = o->tau[i];
    double mass = 0.0, WD = 0.0, sigmass = 0.0, sigWD = 0.0;
    for (int g = 0; g < G; ++g) {
        double mg = blk(o, g * (1 + dim), p);
        double dg = 0.0;
        for (int a = 0; a < dim; ++a) dg += W[a] * blk(o, g * (1 + dim) + 1 + a, p);
        mass += mg;
        WD += dg;
        sigmass += o->sig_t[g] * mg;
        sigWD += o->sig_t[g] * dg;
    }
    double WKW = 0.0;
    int kb = G * (1 + dim);
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) WKW += W[a] * W[b] * blk(o, kb + a * dim + b, p);
    double surf = 0.0;
    int sb = kb + dim * dim;
    for (int f = 0; f < 2 * dim; ++f) {
        double wn = 0.0;
        for (int a = 0; a < dim; ++a) wn += W[a] * face_normal[f][a];
        if (wn > 0.0) surf += wn * blk(o, sb + f, p);
    }
    return o->a0 * mass + o->a0 * tau * WD + surf - WD + tau * WKW + sigmass + tau * sigWD;
}

static void apply_L(const op_ctx *o, int m, const double *x, double *y)
{
    for (int64_t i = 0; i < o->n; ++i) {
        double s = 0.0;
        for (int64_t p = o->row_off[i]; p < o->row_off[i + 1]; ++p) s += L_entry(o, m, i, p) * x[o->col[p]];
        y[i] = s;
    }
}

/* The entries L_m[i, col[p]] of one ordinate, evaluated once (the same
 * L_entry values apply_L uses, kept for the length of one inner solve). */
static double *L_values(const op_ctx *o, int m)
{
    double *Lv = (double *)malloc(sizeof(double) * (o->nnz > 0 ? o->nnz : 1));
    for (int64_t i = 0; i < o->n; ++i)
        for (int64_t p = o->row_off[i]; p < o->row_off[i + 1]; ++p) Lv[p] = L_entry(o, m, i, p);
    return Lv;
}

/* y = L_m x from the stored entries of L_values: the sums of apply_L. */
static void apply_Lv(const op_ctx *o, const double *Lv, const double *x, double *y)
{
    for (int64_t i = 0; i < o->n; ++i) {
        double s = 0.0;
        for (int64_t p = o->row_off[i]; p < o->row_off[i + 1]; ++p) s += Lv[p] * x[o->col[p]];
        y[i] = s;
    }
}

/* kind 0: (Mass + tau W.D) x ; kind 1: 1/(4 pi) sigma_s-weighted version */
static void apply_MD(const op_ctx *o, int m, int kind, const double *x, double *y)
{
    int dim = o->dim, G = o->n_mat;
    const double *W = o->omega + m * dim;
    for (int64_t i = 0; i < o->n; ++i) {
        double s = 0.0;
        for (int64_t p = o->row_off[i]; p < o->row_off[i + 1]; ++p) {
            double e = 0.0;
            for (int g = 0; g < G; ++g) {
                double coef = kind == 0 ? 1.0 : o->sig_s[g] / (4.0 * M_PI);
                double dg = 0.0;
                for (int a = 0; a < dim; ++a) dg += W[a] * blk(o, g * (1 + dim) + 1 + a, p);
                e += coef * (blk(o, g * (1 + dim), p) + o->tau[i] * dg);
            }
            s += e * x[o->col[p]];
        }
        y[i] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Patch block-Jacobi preconditioner.  Patches: the domain box is cut into
 * cubes of side h = 2 (|box| / n)^(1/dim) (doubled while the grid would have
 * more than 2^26 cells); a point belongs to the cube floor((x - lo) / h)
 * (taken as (x - lo) * (1/h), clamped to the grid), cubes are numbered with
 * the last axis fastest, and the points of one cube in increasing index form
 * patches of at most ORC_PATCH_MAX consecutive points.  For an ordinate m the
 * preconditioner solves L_m[P,P] z_P = v_P on every patch P (dense LU with
 * partial pivoting); the GMRES iterate is unchanged in the limit, only the
 * iteration count depends on it.                                            */
#define ORC_PATCH_MAX 16

typedef struct {
    int64_t np;         /* patches */
    int64_t *start;     /* [np+1] into pts */
    int32_t *pts;       /* [n] points, patch by patch */
} orc_patches;

typedef struct { int64_t cell; int32_t i; } cell_pt;

static int cmp_cell_pt(const void *a, const void *b)
{
    const cell_pt *p = (const cell_pt *)a, *q = (const cell_pt *)b;
    if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
    return p->i < q->i ? -1 : (p->i > q->i);
}

static void make_patches(const op_ctx *o, orc_patches *pt)
{
    int dim = o->dim;
    int64_t n = o->n;
    double vol = 1.0;
    for (int a = 0; a < dim; ++a) vol *= o->dom_hi[a] - o->dom_lo[a];
    double h = 2.0 * pow(vol / (double)n, 1.0 / dim);
    int64_t dims[3];
    for (;;) {
        int64_t tot = 1;
        for (int a = 0; a < dim; ++a) {
            int64_t c = (int64_t)ceil((o->dom_hi[a] - o->dom_lo[a]) / h);
            dims[a] = c < 1 ? 1 : c;
            tot *= dims[a];
        }
        if (tot <= ((int64_t)1 << 26)) break;
        h *= 2.0;
    }
    double ih = 1.0 / h;
    cell_pt *cp = (cell_pt *)malloc(sizeof(cell_pt) * n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = 0;
        for (int a = 0; a < dim; ++a) {
            double t = (o->x[i * dim + a] - o->dom_lo[a]) * ih;
            int64_t b = t < 0.0 ? 0 : (int64_t)floor(t);
            if (b > dims[a] - 1) b = dims[a] - 1;
            id = id * dims[a] + b;
        }
        cp[i].cell = id;
        cp[i].i = (int32_t)i;
    }
    qsort(cp, (size_t)n, sizeof(cell_pt), cmp_cell_pt);
    pt->pts = (int32_t *)malloc(sizeof(int32_t) * n);
    pt->start = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    pt->np = 0;
    int64_t run = 0;
    for (int64_t k = 0; k < n; ++k) {
        pt->pts[k] = cp[k].i;
        int fresh = k == 0 || cp[k].cell != cp[k - 1].cell;
        if (fresh) run = 0;
        if (fresh || run == ORC_PATCH_MAX) {
            pt->start[pt->np++] = k;
            run = 0;
        }
        run++;
    }
    pt->start[pt->np] = n;
    free(cp);
}

/* LU factors (row pivoting) of the patch blocks L_m[P,P] of one ordinate,
 * from its entries Lv; lu[p] holds s*s values, piv[p] s row indices.  A zero
 * pivot leaves the block as its diagonal (or 1 where that is 0).            */
typedef struct {
    double **lu;
    int **piv;
} orc_patch_lu;

static double Lv_at(const op_ctx *o, const double *Lv, int64_t i, int32_t j)
{
    for (int64_t p = o->row_off[i]; p < o->row_off[i + 1]; ++p)
        if (o->col[p] == j) return Lv[p];
    return 0.0;
}

static void patch_factor(const op_ctx *o, const orc_patches *pt, const double *Lv, orc_patch_lu *f)
{
    f->lu = (double **)malloc(sizeof(double *) * pt->np);
    f->piv = (int **)malloc(sizeof(int *) * pt->np);
    for (int64_t p = 0; p < pt->np; ++p) {
        int s = (int)(pt->start[p + 1] - pt->start[p]);
        const int32_t *q = pt->pts + pt->start[p];
        double *A = (double *)malloc(sizeof(double) * s * s);
        int *pv = (int *)malloc(sizeof(int) * s);
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b) A[a * s + b] = Lv_at(o, Lv, q[a], q[b]);
        int ok = 1;
        for (int k = 0; k < s; ++k) {
            int r = k;
            for (int a = k + 1; a < s; ++a)
                if (fabs(A[a * s + k]) > fabs(A[r * s + k])) r = a;
            pv[k] = r;
            if (A[r * s + k] == 0.0) { ok = 0; break; }
            if (r != k)
                for (int b = 0; b < s; ++b) { double t = A[k * s + b]; A[k * s + b] = A[r * s + b]; A[r * s + b] = t; }
            for (int a = k + 1; a < s; ++a) {
                double l = A[a * s + k] / A[k * s + k];
                A[a * s + k] = l;
                for (int b = k + 1; b < s; ++b) A[a * s + b] -= l * A[k * s + b];
            }
        }
        if (!ok) {
            /* diagonal fallback: an identity permutation and a diagonal U */
            for (int a = 0; a < s; ++a) {
                double d = Lv_at(o, Lv, q[a], q[a]);
                for (int b = 0; b < s; ++b) A[a * s + b] = 0.0;
                A[a * s + a] = d != 0.0 ? d : 1.0;
                pv[a] = a;
            }
        }
        f->lu[p] = A;
        f->piv[p] = pv;
    }
}

/* z = M^-1 v: on every patch, the LU solve of L_m[P,P] z_P = v_P. */
static void patch_solve(const orc_patches *pt, const orc_patch_lu *f, const double *v, double *z)
{
    double t[ORC_PATCH_MAX];
    for (int64_t p = 0; p < pt->np; ++p) {
        int s = (int)(pt->start[p + 1] - pt->start[p]);
        const int32_t *q = pt->pts + pt->start[p];
        const double *A = f->lu[p];
        const int *pv = f->piv[p];
        for (int a = 0; a < s; ++a) t[a] = v[q[a]];
        for (int k = 0; k < s; ++k) {
            int r = pv[k];
            if (r != k) { double u = t[k]; t[k] = t[r]; t[r] = u; }
        }
        for (int a = 1; a < s; ++a)
            for (int b = 0; b < a; ++b) t[a] -= A[a * s + b] * t[b];
        for (int a = s - 1; a >= 0; --a) {
            for (int b = a + 1; b < s; ++b) t[a] -= A[a * s + b] * t[b];
            t[a] /= A[a * s + a];
        }
        for (int a = 0; a < s; ++a) z[q[a]] = t[a];
    }
}

static void patch_free(const orc_patches *pt, orc_patch_lu *f)
{
    for (int64_t p = 0; p < pt->np; ++p) { free(f->lu[p]); free(f->piv[p]); }
    free(f->lu);
    free(f->piv);
}

/* Restarted GMRES with right point-Jacobi preconditioning for L_m x = f,
 * x0 = 0, modified Gram-Schmidt Arnoldi and Givens rotations (Saad,
 * Iterative Methods for Sparse Linear Systems, Alg. 6.9 with right
 * preconditioning).  Stops when ||f - L x|| <= tol ||f||.  Returns the
 * number of Arnoldi steps; *res gets the final relative residual.           */
static int64_t gmres_L(const op_ctx *o, int m, const double *f, double *x, double *res)
{
    int64_t n = o->n;
    int k = o->restart_in;
    double *Vb = (double *)malloc(sizeof(double) * n * (k + 1));
    double *z = (double *)malloc(sizeof(double) * n), *w = (double *)malloc(sizeof(double) * n);
    double *r = (double *)malloc(sizeof(double) * n), *dinv = (double *)malloc(sizeof(double) * n);
    double *H = (double *)calloc((size_t)(k + 1) * k, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * k), *sn = (double *)malloc(sizeof(double) * k);
    double *g = (double *)malloc(sizeof(double) * (k + 1)), *yv = (double *)malloc(sizeof(double) * k);
    double *Lv = L_values(o, m);
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t p = o->row_off[i]; p < o->row_off[i + 1]; ++p)
            if (o->col[p] == i) d = Lv[p];
        dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
        x[i] = 0.0;
    }
    orc_patches pt = {0, NULL, NULL};
    orc_patch_lu plu = {NULL, NULL};
    double *u = NULL;
    if (o->precond == 1) {
        make_patches(o, &pt);
        patch_factor(o, &pt, Lv, &plu);
        u = (double *)malloc(sizeof(double) * n);
    }
    double fn = sqrt(dot(n, f, f));
    int64_t its = 0;
    double rel = 0.0;
    if (fn == 0.0) goto done;
    for (;;) {
        apply_Lv(o, Lv, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = f[i] - r[i];
        double beta = sqrt(dot(n, r, r));
        rel = beta / fn;
        if (beta <= o->tol_in * fn || its >= o->max_in) break;
        for (int64_t i = 0; i < n; ++i) Vb[i] = r[i] / beta;
        for (int j = 0; j <= k; ++j) g[j] = 0.0;
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < k; ++j) {
            const double *vj = Vb + (int64_t)j * n;
            if (o->precond == 1) patch_solve(&pt, &plu, vj, z);
            else
                for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * vj[i];
            apply_Lv(o, Lv, z, w);
            for (int q = 0; q <= j; ++q) {
                const double *vq = Vb + (int64_t)q * n;
                double h = dot(n, w, vq);
                H[q * k + j] = h;
                for (int64_t i = 0; i < n; ++i) w[i] -= h * vq[i];
            }
            double hn = sqrt(dot(n, w, w));
            H[(j + 1) * k + j] = hn;
            for (int q = 0; q < j; ++q) {
                double a = H[q * k + j], b = H[(q + 1) * k + j];
                H[q * k + j] = cs[q] * a + sn[q] * b;
                H[(q + 1) * k + j] = -sn[q] * a + cs[q] * b;
            }
            double a = H[j * k + j], b = H[(j + 1) * k + j];
            double den = sqrt(a * a + b * b);
            cs[j] = den == 0.0 ? 1.0 : a / den;
            sn[j] = den == 0.0 ? 0.0 : b / den;
            H[j * k + j] = den;
            H[(j + 1) * k + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            its++;
            jend = j + 1;
            if (fabs(g[j + 1]) <= o->tol_in * fn || hn == 0.0 || its >= o->max_in) break;
            double *vn = Vb + (int64_t)(j + 1) * n;
            for (int64_t i = 0; i < n; ++i) vn[i] = w[i] / hn;
        }
        for (int q = jend - 1; q >= 0; --q) {
            double s = g[q];
            for (int p = q + 1; p < jend; ++p) s -= H[q * k + p] * yv[p];
            yv[q] = s / H[q * k + q];
        }
        if (o->precond == 1) {
            /* x += M^-1 (V y) */
            for (int64_t i = 0; i < n; ++i) u[i] = 0.0;
            for (int q = 0; q < jend; ++q) {
                const double *vq = Vb + (int64_t)q * n;
                for (int64_t i = 0; i < n; ++i) u[i] += yv[q] * vq[i];
            }
            patch_solve(&pt, &plu, u, z);
            for (int64_t i = 0; i < n; ++i) x[i] += z[i];
        } else {
            for (int q = 0; q < jend; ++q) {
                const double *vq = Vb + (int64_t)q * n;
                for (int64_t i = 0; i < n; ++i) x[i] += dinv[i] * yv[q] * vq[i];
            }
        }
    }
done:
    *res = rel;
    if (o->precond == 1) {
        patch_free(&pt, &plu);
        free(pt.start); free(pt.pts); free(u);
    }
    free(Lv); free(Vb); free(z); free(w); free(r); free(dinv); free(H); free(cs); free(sn); free(g); free(yv);
    return its;
}

typedef struct {
    int64_t inner_its;
    double inner_res_max;
    int64_t inner_solves;
} solve_stats;

/* X = L^-1 F for every ordinate (L is block diagonal in angle).  F, X are
 * [n][M], ordinate fastest.                                                 */
static void Linv_all(const op_ctx *o, const double *F, double *X, solve_stats *st)
{
    int M = o->n_ord;
    int64_t n = o->n;
    int64_t its_sum = 0;
    double res_max = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : its_sum) reduction(max : res_max)
    for (int m = 0; m < M; ++m) {
        double *f = (double *)malloc(sizeof(double) * n), *x = (double *)malloc(sizeof(double) * n);
        for (int64_t i = 0; i < n; ++i) f[i] = F[i * M + m];
        double res;
        its_sum += gmres_L(o, m, f, x, &res);
        if (res > res_max) res_max = res;
        for (int64_t i = 0; i < n; ++i) X[i * M + m] = x[i];
        free(f); free(x);
    }
    st->inner_its += its_sum;
    st->inner_solves += 1;
    if (res_max > st->inner_res_max) st->inner_res_max = res_max;
}

/* Y[i][m] = (MS_m phi)_i */
static void MS_all(const op_ctx *o, const double *phi, double *Y)
{
    int M = o->n_ord;
    int64_t n = o->n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int m = 0; m < M; ++m) {
        double *y = (double *)malloc(sizeof(double) * n);
        apply_MD(o, m, 1, phi, y);
        for (int64_t i = 0; i < n; ++i) Y[i * M + m] = y[i];
        free(y);
    }
}

/* (D Psi)_i = sum_m w_m Psi_{m,i} */
static void D_op(const op_ctx *o, const double *Psi, double *phi)
{
    int M = o->n_ord;
    for (int64_t i = 0; i < o->n; ++i) {
        double s = 0.0;
        for (int m = 0; m < M; ++m) s += o->wq[m] * Psi[i * M + m];
        phi[i] = s;
    }
}

/* Outer operator A phi = phi - D L^-1 MS phi (Eq. krylov-operator). */
static void apply_outer(const op_ctx *o, const double *phi, double *out, double *tmp1, double *tmp2,
                        solve_stats *st)
{
    MS_all(o, phi, tmp1);
    Linv_all(o, tmp1, tmp2, st);
    D_op(o, tmp2, out);
    for (int64_t i = 0; i < o->n; ++i) out[i] = phi[i] - out[i];
}

/* Right-hand side of one backward-Euler step (Sec. 4.1-4.2):
 *   F_m = T_m Psi^{n-1} + r_m,
 *   r_m = (N_i, |W.n| psi_b)_{W.n<0} + <N_i, q_m> + tau_i W.<dN_i, q_m>.     */
static void build_rhs(const op_ctx *o, const double *psi_prev, const double *q, const double *psib, double *F)
{
    int M = o->n_ord, dim = o->dim;
    int64_t n = o->n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int m = 0; m < M; ++m) {
        double *a = (double *)malloc(sizeof(double) * n), *b = (double *)malloc(sizeof(double) * n);
        double *c = (double *)malloc(sizeof(double) * n), *d = (double *)malloc(sizeof(double) * n);
        for (int64_t i = 0; i < n; ++i) { a[i] = psi_prev ? psi_prev[i * M + m] : 0.0; c[i] = q[i * M + m]; }
        apply_MD(o, m, 0, a, b);        /* (Mass + tau W.D) Psi^{n-1} */
        apply_MD(o, m, 0, c, d);        /* (Mass + tau W.D) q         */
        for (int64_t i = 0; i < n; ++i) F[i * M + m] = o->a0 * b[i] + d[i];
        free(a); free(b); free(c); free(d);
    }
    if (psib) {
        for (int64_t k = 0; k < o->nbq; ++k) {
            const double *nf = face_normal[o->bq_face[k]];
            for (int m = 0; m < M; ++m) {
                double wn = 0.0;
                for (int a = 0; a < dim; ++a) wn += o->omega[m * dim + a] * nf[a];
                if (wn >= 0.0) continue;
                double val = psib[k * M + m];
                if (val == 0.0) continue;
                for (int t = 0; t < o->bq_nact[k]; ++t) {
                    int32_t i = o->bq_act[k * o->kmax + t];
                    F[(int64_t)i * M + m] += o->bq_w[k] * (-wn) * o->bq_N[k * o->kmax + t] * val;
                }
            }
        }
    }
}

/* One backward-Euler step, or a steady solve when a0 = 0 (Sec. 4.2):
 *   b_psi = L^-1 (T Psi^{n-1} + r),  b_phi = D b_psi,
 *   GMRES on (I - D L^-1 MS) Phi = b_phi from Phi0,
 *   Psi = L^-1 MS Phi + b_psi.
 * out_stats: [outer its, inner its total, inner solves], res: [outer rel res, max inner rel res] */
int orc_step(op_ctx *o, const double *psi_prev, const double *q, const double *psib, const double *phi0,
             double *psi_out, double *phi_out, int64_t *out_stats, double *out_res)
{
    int M = o->n_ord;
    int64_t n = o->n;
    solve_stats st = {0, 0.0, 0};
    double *F = (double *)malloc(sizeof(double) * n * M), *bpsi = (double *)malloc(sizeof(double) * n * M);
    double *tmp1 = (double *)malloc(sizeof(double) * n * M), *tmp2 = (double *)malloc(sizeof(double) * n * M);
    build_rhs(o, psi_prev, q, psib, F);
    Linv_all(o, F, bpsi, &st);
    double *bphi = (double *)malloc(sizeof(double) * n);
    D_op(o, bpsi, bphi);

    /* outer GMRES(k), unpreconditioned */
    int k = o->restart_out;
    double *Vb = (double *)malloc(sizeof(double) * n * (k + 1));
    double *w = (double *)malloc(sizeof(double) * n), *r = (double *)malloc(sizeof(double) * n);
    double *H = (double *)calloc((size_t)(k + 1) * k, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * k), *sn = (double *)malloc(sizeof(double) * k);
    double *g = (double *)malloc(sizeof(double) * (k + 1)), *yv = (double *)malloc(sizeof(double) * k);
    double *phi = phi_out;
    for (int64_t i = 0; i < n; ++i) phi[i] = phi0 ? phi0[i] : 0.0;
    double bn = sqrt(dot(n, bphi, bphi));
    int64_t outer = 0;
    double orel = 0.0;
    if (bn > 0.0) {
        for (;;) {
            apply_outer(o, phi, r, tmp1, tmp2, &st);
            for (int64_t i = 0; i < n; ++i) r[i] = bphi[i] - r[i];
            double beta = sqrt(dot(n, r, r));
            orel = beta / bn;
            if (beta <= o->tol_out * bn || outer >= o->max_out) break;
            for (int64_t i = 0; i < n; ++i) Vb[i] = r[i] / beta;
            for (int j = 0; j <= k; ++j) g[j] = 0.0;
            g[0] = beta;
            int jend = 0;
            for (int j = 0; j < k; ++j) {
                apply_outer(o, Vb + (int64_t)j * n, w, tmp1, tmp2, &st);
                for (int q2 = 0; q2 <= j; ++q2) {
                    const double *vq = Vb + (int64_t)q2 * n;
                    double h = dot(n, w, vq);
                    H[q2 * k + j] = h;
                    for (int64_t i = 0; i < n; ++i) w[i] -= h * vq[i];
                }
                double hn = sqrt(dot(n, w, w));
                H[(j + 1) * k + j] = hn;
                for (int q2 = 0; q2 < j; ++q2) {
                    double a = H[q2 * k + j], b = H[(q2 + 1) * k + j];
                    H[q2 * k + j] = cs[q2] * a + sn[q2] * b;
                    H[(q2 + 1) * k + j] = -sn[q2] * a + cs[q2] * b;
                }
                double a = H[j * k + j], b = H[(j + 1) * k + j];
                double den = sqrt(a * a + b * b);
                cs[j] = den == 0.0 ? 1.0 : a / den;
                sn[j] = den == 0.0 ? 0.0 : b / den;
                H[j * k + j] = den;
                H[(j + 1) * k + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                outer++;
                jend = j + 1;
                if (fabs(g[j + 1]) <= o->tol_out * bn || hn == 0.0 || outer >= o->max_out) break;
                double *vn = Vb + (int64_t)(j + 1) * n;
                for (int64_t i = 0; i < n; ++i) vn[i] = w[i] / hn;
            }
            for (int q2 = jend - 1; q2 >= 0; --q2) {
                double s = g[q2];
                for (int p = q2 + 1; p < jend; ++p) s -= H[q2 * k + p] * yv[p];
                yv[q2] = s / H[q2 * k + q2];
            }
            for (int q2 = 0; q2 < jend; ++q2)
                for (int64_t i = 0; i < n; ++i) phi[i] += yv[q2] * Vb[(int64_t)q2 * n + i];
        }
    } else {
        for (int64_t i = 0; i < n; ++i) phi[i] = 0.0;
    }
    /* recovery: Psi = L^-1 MS Phi + b_psi */
    MS_all(o, phi, tmp1);
    Linv_all(o, tmp1, tmp2, &st);
    for (int64_t t = 0; t < n * M; ++t) psi_out[t] = tmp2[t] + bpsi[t];
    out_stats[0] = outer;
    out_stats[1] = st.inner_its;
    out_stats[2] = st.inner_solves;
    out_res[0] = orel;
    out_res[1] = st.inner_res_max;
    free(F); free(bpsi); free(tmp1); free(tmp2); free(bphi); free(Vb); free(w); free(r); free(H);
    free(cs); free(sn); free(g); free(yv);
    return 0;
}

/* Source iteration Phi <- D L^-1 MS Phi + b_phi, the fixed-point alternative
 * named in Sec. 4.2; used only as an independent cross-check of the GMRES
 * outer solve. */
int orc_step_source_iteration(op_ctx *o, const double *psi_prev, const double *q, const double *psib,
                              int iters, double *psi_out, double *phi_out)
{
    int M = o->n_ord;
    int64_t n = o->n;
    solve_stats st = {0, 0.0, 0};
    double *F = (double *)malloc(sizeof(double) * n * M), *bpsi = (double *)malloc(sizeof(double) * n * M);
    double *tmp1 = (double *)malloc(sizeof(double) * n * M), *tmp2 = (double *)malloc(sizeof(double) * n * M);
    double *bphi = (double *)malloc(sizeof(double) * n), *t = (double *)malloc(sizeof(double) * n);
    build_rhs(o, psi_prev, q, psib, F);
    Linv_all(o, F, bpsi, &st);
    D_op(o, bpsi, bphi);
    for (int64_t i = 0; i < n; ++i) phi_out[i] = bphi[i];
    for (int it = 0; it < iters; ++it) {
        MS_all(o, phi_out, tmp1);
        Linv_all(o, tmp1, tmp2, &st);
        D_op(o, tmp2, t);
        for (int64_t i = 0; i < n; ++i) phi_out[i] = t[i] + bphi[i];
    }
    MS_all(o, phi_out, tmp1);
    Linv_all(o, tmp1, tmp2, &st);
    for (int64_t s = 0; s < n * M; ++s) psi_out[s] = tmp2[s] + bpsi[s];
    free(F); free(bpsi); free(tmp1); free(tmp2); free(bphi); free(t);
    return 0;
}

/* Single operator applications, for parity of one sweep and for assembling
 * dense systems in tests.  which: 0 = L, 1 = T, 2 = MS, 3 = source operator
 * (Mass + tau W.D).  X, Y are [n][M].                                        */
void orc_apply(op_ctx *o, int which, const double *X, double *Y)
{
    int M = o->n_ord;
    int64_t n = o->n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int m = 0; m < M; ++m) {
        double *x = (double *)malloc(sizeof(double) * n), *y = (double *)malloc(sizeof(double) * n);
        for (int64_t i = 0; i < n; ++i) x[i] = X[i * M + m];
        if (which == 0) apply_L(o, m, x, y);
        else if (which == 1) { apply_MD(o, m, 0, x, y); for (int64_t i = 0; i < n; ++i) y[i] *= o->a0; }
        else if (which == 2) apply_MD(o, m, 1, x, y);
        else apply_MD(o, m, 0, x, y);
        for (int64_t i = 0; i < n; ++i) Y[i * M + m] = y[i];
        free(x); free(y);
    }
}

/* L_m^-1 for the ordinates m0 <= m < m1 only (used to time a bounded
 * sample of the inner solves).  Returns the Arnoldi steps summed over them. */
int64_t orc_Linv_range(op_ctx *o, const double *F, double *X, int m0, int m1, double *res_max)
{
    int M = o->n_ord;
    int64_t n = o->n;
    int64_t its_sum = 0;
    double rm = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : its_sum) reduction(max : rm)
    for (int m = m0; m < m1; ++m) {
        double *f = (double *)malloc(sizeof(double) * n), *x = (double *)malloc(sizeof(double) * n);
        for (int64_t i = 0; i < n; ++i) f[i] = F[i * M + m];
        double res;
        its_sum += gmres_L(o, m, f, x, &res);
        if (res > rm) rm = res;
        for (int64_t i = 0; i < n; ++i) X[i * M + m] = x[i];
        free(f); free(x);
    }
    *res_max = rm;
    return its_sum;
}

/* Right-hand side F = T Psi^{n-1} + r alone. */
void orc_rhs(op_ctx *o, const double *psi_prev, const double *q, const double *psib, double *F)
{
    build_rhs(o, psi_prev, q, psib, F);
}

/* Point values phi(x_i) = sum_j N_j(x_i) Phi_j (Eq. flux-expansion). */
void orc_point_values(int64_t n, const int64_t *row_off, const int32_t *col, const double *E,
                      const double *coef, int ncomp, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < ncomp; ++c) {
            double s = 0.0;
            for (int64_t p = row_off[i]; p < row_off[i + 1]; ++p) s += E[p] * coef[(int64_t)col[p] * ncomp + c];
            out[i * ncomp + c] = s;
        }
}

/* The patches of the preconditioner (for tests): returns the count, fills
 * start[np+1] and pts[n] (both sized by the caller: n+1 and n).            */
int64_t orc_patches_of(op_ctx *o, int64_t *start, int32_t *pts)
{
    orc_patches pt;
    make_patches(o, &pt);
    for (int64_t p = 0; p <= pt.np; ++p) start[p] = pt.start[p];
    for (int64_t k = 0; k < o->n; ++k) pts[k] = pt.pts[k];
    int64_t np = pt.np;
    free(pt.start); free(pt.pts);
    return np;
}

/* z = M^-1 v for ordinate m (for tests): v, z [n]. */
void orc_patch_precond(op_ctx *o, int m, const double *v, double *z)
{
    orc_patches pt;
    orc_patch_lu plu;
    double *Lv = L_values(o, m);
    make_patches(o, &pt);
    patch_factor(o, &pt, Lv, &plu);
    patch_solve(&pt, &plu, v, z);
    patch_free(&pt, &plu);
    free(pt.start); free(pt.pts); free(Lv);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
