// Quadrature rules of the library (host side).
//
// Volume rule on the fan triangles of a cell (Sec. 3.2, App. A reference
// triangle {xi >= 0, xi0 + xi1 <= 1}): the conical product of a Gauss-Jacobi
// rule for the weight (1-u) with a Gauss-Legendre rule, n*n points, exact
// for polynomials of degree 2n-1.  Surface rule on boundary edges: n-point
// Gauss-Legendre on [-1, 1].  Angular rules: product rules of Sec. 4.1 (see
// mlpg_angular_quadrature in include/mlpg.h).
//
// Nodes come from the Golub-Welsch eigenvalue problem of the three-term
// recurrence (Jacobi rotations on the symmetric tridiagonal matrix), polished
// by Newton steps on the recurrence.
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.hpp"

namespace mlpg {

namespace {

// Eigen-decomposition of a symmetric n x n matrix by cyclic Jacobi rotations.
// A is overwritten; evals get the eigenvalues, Q the eigenvectors (columns).
void sym_eigen(int n, double *A, double *evals, double *Q)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-300) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = A[p * n + p], aqq = A[q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double qkp = Q[k * n + p], qkq = Q[k * n + q];
                    Q[k * n + p] = c * qkp - s * qkq;
                    Q[k * n + q] = s * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) evals[i] = A[i * n + i];
}

// Value and derivative of the Jacobi polynomial P_n^{(alpha,0)} at x by the
// three-term recurrence (alpha = 0 gives Legendre).
void jacobi_poly(int n, double alpha, double x, double *p, double *dp)
{
    const double b = 0.0;
    double p0 = 1.0, p1 = 0.5 * (alpha - b + (alpha + b + 2.0) * x);
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    double d0 = 0.0, d1 = 0.5 * (alpha + b + 2.0);
    for (int k = 2; k <= n; ++k) {
        double c = 2.0 * k + alpha + b;
        double a1 = 2.0 * k * (k + alpha + b) * (c - 2.0);
        double a2 = (c - 1.0) * (alpha * alpha - b * b);
        double a3 = (c - 2.0) * (c - 1.0) * c;
        double a4 = 2.0 * (k + alpha - 1.0) * (k + b - 1.0) * c;
        double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        double d2 = ((a2 + a3 * x) * d1 + a3 * p1 - a4 * d0) / a1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *p = p1;
    *dp = d1;
}

void golub_welsch(int n, double alpha, double *x, double *w)
{
    const double beta = 0.0;
    std::vector<double> T(n * n, 0.0), Q(n * n), ev(n);
    for (int k = 0; k < n; ++k) {
        double s = 2.0 * k + alpha + beta;
        double a = (k == 0) ? (beta - alpha) / (alpha + beta + 2.0)
                            : (beta * beta - alpha * alpha) / (s * (s + 2.0));
        T[k * n + k] = a;
        if (k >= 1) {
            double num = 4.0 * k * (k + alpha) * (k + beta) * (k + alpha + beta);
            double den = s * s * (s + 1.0) * (s - 1.0);
            double b = std::sqrt(num / den);
            T[k * n + k - 1] = b;
            T[(k - 1) * n + k] = b;
        }
    }
    sym_eigen(n, T.data(), ev.data(), Q.data());
    double mu0 = std::pow(2.0, alpha + beta + 1.0) * std::tgamma(alpha + 1.0) * std::tgamma(beta + 1.0) /
                 std::tgamma(alpha + beta + 2.0);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (ev[order[j]] < ev[order[i]]) std::swap(order[i], order[j]);
    for (int i = 0; i < n; ++i) {
        int c = order[i];
        double xi = ev[c];
        // Newton polish on P_n^{(alpha,0)}
        for (int it = 0; it < 3; ++it) {
            double p, dp;
            jacobi_poly(n, alpha, xi, &p, &dp);
            if (dp == 0.0) break;
            xi -= p / dp;
        }
        x[i] = xi;
        w[i] = mu0 * Q[0 * n + c] * Q[0 * n + c];
    }
}

Rules g_rules;
std::once_flag g_rules_once;

void make_rules()
{
    double u[kTriN], wu[kTriN], v[kTriN], wv[kTriN];
    gauss_jacobi(kTriN, 1.0, u, wu);
    gauss_legendre(kTriN, v, wv);
    int q = 0;
    for (int a = 0; a < kTriN; ++a) {
        double ua = 0.5 * (u[a] + 1.0), wa = wu[a] / 4.0;   // weight (1-u) on [0,1]
        for (int b = 0; b < kTriN; ++b) {
            double vb = 0.5 * (v[b] + 1.0), wb = 0.5 * wv[b];
            g_rules.tri_pts[q][0] = ua;
            g_rules.tri_pts[q][1] = (1.0 - ua) * vb;
            g_rules.tri_w[q] = wa * wb;
            q++;
        }
    }
    gauss_legendre(kSegRule, g_rules.seg_pts, g_rules.seg_w);

    // Tetrahedron {xi >= 0, xi0 + xi1 + xi2 <= 1}: collapsed coordinates
    // (u, v, s) -> (u, (1-u) v, (1-u)(1-v) s) with Jacobian (1-u)^2 (1-v),
    // absorbed by Gauss-Jacobi rules in u (alpha 2) and v (alpha 1).
    double tu[kTetN], twu[kTetN], tv[kTetN], twv[kTetN], ts[kTetN], tws[kTetN];
    gauss_jacobi(kTetN, 2.0, tu, twu);
    gauss_jacobi(kTetN, 1.0, tv, twv);
    gauss_legendre(kTetN, ts, tws);
    q = 0;
    for (int a = 0; a < kTetN; ++a) {
        double ua = 0.5 * (tu[a] + 1.0), wa = twu[a] / 8.0;
        for (int b = 0; b < kTetN; ++b) {
            double vb = 0.5 * (tv[b] + 1.0), wb = twv[b] / 4.0;
            for (int c = 0; c < kTetN; ++c) {
                double sc = 0.5 * (ts[c] + 1.0), wc = 0.5 * tws[c];
                g_rules.tet_pts[q][0] = ua;
                g_rules.tet_pts[q][1] = (1.0 - ua) * vb;
                g_rules.tet_pts[q][2] = (1.0 - ua) * (1.0 - vb) * sc;
                g_rules.tet_w[q] = wa * wb * wc;
                q++;
            }
        }
    }
    // boundary triangles in 3D: the same construction as the cell triangles
    double u3[kTri3N], wu3[kTri3N], v3[kTri3N], wv3[kTri3N];
    gauss_jacobi(kTri3N, 1.0, u3, wu3);
    gauss_legendre(kTri3N, v3, wv3);
    q = 0;
    for (int a = 0; a < kTri3N; ++a) {
        double ua = 0.5 * (u3[a] + 1.0), wa = wu3[a] / 4.0;
        for (int b = 0; b < kTri3N; ++b) {
            double vb = 0.5 * (v3[b] + 1.0), wb = 0.5 * wv3[b];
            g_rules.tri3_pts[q][0] = ua;
            g_rules.tri3_pts[q][1] = (1.0 - ua) * vb;
            g_rules.tri3_w[q] = wa * wb;
            q++;
        }
    }
}

}  // namespace

void gauss_legendre(int n, double *x, double *w) { golub_welsch(n, 0.0, x, w); }
void gauss_jacobi(int n, double alpha, double *x, double *w) { golub_welsch(n, alpha, x, w); }

const Rules &rules()
{
    std::call_once(g_rules_once, make_rules);
    return g_rules;
}

}  // namespace mlpg

extern "C" int mlpg_angular_quadrature(int dim, int n_ord, int kind, double *omega, double *w)
{
    using namespace mlpg;
    MLPG_CHECK(omega && w, MLPG_ERR_ARG, "mlpg_angular_quadrature: null output");
    if (dim == 2 && (kind == MLPG_QUAD_PRODUCT || kind == MLPG_QUAD_BEAM_DENSE)) {
        double xg[4], wg[4];
        gauss_legendre(4, xg, wg);
        double xi[2] = {xg[2], xg[3]}, wp[2] = {wg[2], wg[3]};   // positive roots, increasing
        int na = n_ord / 2;
        MLPG_CHECK(n_ord > 0 && 2 * na == n_ord, MLPG_ERR_ARG, "2D product rule needs an even ordinate count");
        std::vector<double> mids(na), widths(na);
        if (kind == MLPG_QUAD_PRODUCT) {
            for (int k = 0; k < na; ++k) {
                mids[k] = (2.0 * (k + 1) - 1.0) * M_PI / na;
                widths[k] = 2.0 * M_PI / na;
            }
        } else {
            MLPG_CHECK(n_ord == 256, MLPG_ERR_ARG, "beam-dense rule is defined for 256 ordinates");
            const double win = 10.0 * M_PI / 180.0;
            // 41 sectors over [-win, win], 87 over [win, 2 pi - win]
            std::vector<double> edges;
            for (int k = 0; k <= 41; ++k) edges.push_back(-win + 2.0 * win * k / 41.0);
            for (int k = 1; k <= 87; ++k) edges.push_back(win + (2.0 * M_PI - 2.0 * win) * k / 87.0);
            for (int k = 0; k < na; ++k) {
                mids[k] = 0.5 * (edges[k] + edges[k + 1]);
                widths[k] = edges[k + 1] - edges[k];
            }
        }
        int m = 0;
        for (int p = 0; p < 2; ++p) {
            double st = std::sqrt(1.0 - xi[p] * xi[p]);
            for (int k = 0; k < na; ++k, ++m) {
                omega[2 * m] = st * std::cos(mids[k]);
                omega[2 * m + 1] = st * std::sin(mids[k]);
                w[m] = 2.0 * wp[p] * widths[k];
            }
        }
        return MLPG_OK;
    }
    if (dim == 3 && kind == MLPG_QUAD_PRODUCT) {
        double xg[6], wg[6];
        gauss_legendre(6, xg, wg);
        int na = n_ord / 6;
        MLPG_CHECK(n_ord > 0 && 6 * na == n_ord, MLPG_ERR_ARG, "3D product rule needs a multiple of 6 ordinates");
        int m = 0;
        for (int p = 0; p < 6; ++p) {
            double st = std::sqrt(1.0 - xg[p] * xg[p]);
            for (int k = 0; k < na; ++k, ++m) {
                double ph = (2.0 * (k + 1) - 1.0) * M_PI / na;
                omega[3 * m] = st * std::cos(ph);
                omega[3 * m + 1] = st * std::sin(ph);
                omega[3 * m + 2] = xg[p];
                w[m] = wg[p] * 2.0 * M_PI / na;
            }
        }
        return MLPG_OK;
    }
    mlpg::set_error("mlpg_angular_quadrature: unsupported dim/kind");
    return MLPG_ERR_ARG;
}

namespace mlpg {
namespace {

// Does the ray from src along the plane direction (cos phi, sin phi) meet the
// disk (center, radius)?  (A source inside the disk sees it in every direction.)
bool ray_hits_disk(const double *src, const double *center, double radius, double phi)
{
    const double dx = center[0] - src[0], dy = center[1] - src[1];
    const double d2 = dx * dx + dy * dy;
    if (d2 <= radius * radius) return true;
    const double t = dx * std::cos(phi) + dy * std::sin(phi);   // distance to the closest approach
    if (t <= 0.0) return false;
    return d2 - t * t <= radius * radius;
}

// Sectors kept for one polar level, in increasing azimuth: (level, index).
// Top-down: a sector of level >= min_level whose goal subsectors all miss the
// object is kept whole; otherwise its two halves are examined, down to the
// goal level, where a sector is always kept.
void refine_sectors(int level, long k, int min_level, int goal_level, const std::vector<char> &hit,
                    std::vector<std::pair<int, long>> &out)
{
    const long span = 1L << (goal_level - level);
    if (level >= min_level) {
        bool any = false;
        for (long c = k * span; c < (k + 1) * span && !any; ++c) any = hit[c] != 0;
        if (!any || level == goal_level) {
            out.emplace_back(level, k);
            return;
        }
    }
    refine_sectors(level + 1, 2 * k, min_level, goal_level, hit, out);
    refine_sectors(level + 1, 2 * k + 1, min_level, goal_level, hit, out);
}

}  // namespace
}  // namespace mlpg

extern "C" int mlpg_refined_quadrature(int min_level, int goal_level, const double *src, const double *center,
                                       double radius, int cap, double *omega, double *w)
{
    using namespace mlpg;
    MLPG_CHECK(min_level >= 0 && goal_level >= min_level && goal_level <= 12, MLPG_ERR_ARG,
               "mlpg_refined_quadrature: need 0 <= min_level <= goal_level <= 12");
    MLPG_CHECK(src && center && radius >= 0.0, MLPG_ERR_ARG, "mlpg_refined_quadrature: null point or negative radius");
    MLPG_CHECK(cap >= 0, MLPG_ERR_ARG, "mlpg_refined_quadrature: negative capacity");
    const long ng = 4L << goal_level;   // goal sectors per polar level
    std::vector<char> hit(ng);
    for (long c = 0; c < ng; ++c) hit[c] = ray_hits_disk(src, center, radius, 2.0 * M_PI * (c + 0.5) / ng) ? 1 : 0;
    std::vector<std::pair<int, long>> sec;
    for (long k = 0; k < 4; ++k) refine_sectors(0, k, min_level, goal_level, hit, sec);
    const int count = 2 * (int)sec.size();
    if (cap == 0) return count;
    MLPG_CHECK(omega && w, MLPG_ERR_ARG, "mlpg_refined_quadrature: null output");
    if (cap < count) {
        set_error("mlpg_refined_quadrature: " + std::to_string(count) + " ordinates exceed the capacity");
        return MLPG_ERR_CAPACITY;
    }
    double xg[4], wg[4];
    gauss_legendre(4, xg, wg);
    const double xi[2] = {xg[2], xg[3]}, wp[2] = {wg[2], wg[3]};
    int m = 0;
    for (int p = 0; p < 2; ++p) {
        const double st = std::sqrt(1.0 - xi[p] * xi[p]);
        for (const auto &e : sec) {
            const double na = (double)(4L << e.first);
            const double mid = (2.0 * (e.second + 1) - 1.0) * M_PI / na;
            omega[2 * m] = st * std::cos(mid);
            omega[2 * m + 1] = st * std::sin(mid);
            w[m] = 2.0 * wp[p] * (2.0 * M_PI / na);
            ++m;
        }
    }
    return count;
}
