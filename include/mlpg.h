/*
 * mlpg.h - C ABI of libmlpg.so, a gfx950 (MI355X) implementation of the hot
 * path of the meshless-local Petrov-Galerkin (MLPG) discrete-ordinates
 * transport method of Bassett & Owen, "Meshless discretization of the
 * discrete-ordinates transport equation with integration based on Voronoi
 * cells" (arXiv 2008.02205).
 *
 * The four stage calls follow the paper's statement of the problem:
 *   mlpg_geometry   Sec. 3.1 (Voronoi-like cells) and Sec. 3.4 (connectivity)
 *   mlpg_integrate  Sec. 2.2 (RK functions), Sec. 3.2 and Alg. 1 (integration)
 *   mlpg_assemble   Sec. 4.1 (Eq. weak-transport: cross sections, ordinates, dt)
 *   mlpg_solve      Sec. 4.2 (Eq. krylov-operator: source, inflow; one step)
 *
 * Conventions for every call:
 *   - Pointers named "device" are HIP device pointers on the current device;
 *     "host" pointers are ordinary host memory.  Inputs are read during the
 *     call (or, for device inputs, by work enqueued on `stream` before the call
 *     returns) and are not retained.  Outputs are written by work enqueued on
 *     `stream`; synchronise the stream before reading them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Arrays of per-point, per-ordinate values are [n][n_ord] with the
 *     ordinate index fastest.  Points keep the caller's order.
 *   - Device memory: the four stage calls (and mlpg_update_points,
 *     mlpg_apply_patch_precond) take a caller-owned workspace, a device
 *     buffer of at least the bytes its *_workspace_bytes query returns,
 *     256-byte aligned; the stage carves all of its buffers and temporaries
 *     out of it and the handle keeps pointers into it, so every workspace
 *     must stay allocated and untouched until it is replaced by the same
 *     stage or the handle is destroyed.  A smaller workspace fails with
 *     MLPG_ERR_WORKSPACE before anything is enqueued.  A NULL workspace makes
 *     the library allocate one of the queried size itself (released by
 *     mlpg_destroy).  Host-side, a handle holds a few pinned host words and
 *     HIP events for its Krylov loops.  mlpg_neighbors_count allocates a
 *     temporary of n counts.  A handle is not thread-safe; separate handles
 *     may be used concurrently on separate streams.
 *   - Every call returns MLPG_OK (0) or a negative mlpg_status.  Arguments are
 *     validated on the host before anything is enqueued; the message of the
 *     last failure on the calling thread is returned by mlpg_last_error().
 */
#ifndef MLPG_H
#define MLPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlpg_problem *mlpg_handle;

typedef enum {
    MLPG_OK = 0,
    MLPG_ERR_ARG = -1,            /* invalid argument (checked before any launch) */
    MLPG_ERR_HIP = -2,            /* a HIP runtime call failed */
    MLPG_ERR_CAPACITY = -3,       /* a fixed per-cell or per-point capacity was exceeded */
    MLPG_ERR_NOT_CONVERGED = -4,  /* a Krylov solve hit its iteration limit */
    MLPG_ERR_GEOMETRY = -5,       /* a cell came out empty or a moment matrix stayed singular */
    MLPG_ERR_WORKSPACE = -6,      /* a workspace smaller than its *_workspace_bytes query */
    MLPG_ERR_STATE = -7           /* stage called out of order */
} mlpg_status;

enum { MLPG_FP64 = 0, MLPG_MIXED = 1 };
enum { MLPG_QUAD_PRODUCT = 0, MLPG_QUAD_BEAM_DENSE = 1 };
enum { MLPG_OP_L = 0, MLPG_OP_T = 1, MLPG_OP_MS = 2, MLPG_OP_SRC = 3 };

/* Message of the last failing call on this thread ("" if none). */
const char *mlpg_last_error(void);

/* ------------------------------------------------------------------------
 * Angular quadrature (Sec. 4.1: ordinates Omega_m and weights w_m with
 * sum_m w_m = 4 pi).  Host-only.
 *   dim = 2, kind = MLPG_QUAD_PRODUCT: two polar levels (the positive roots
 *     of the 4-point Gauss-Legendre rule, weights doubled for the folded
 *     lower hemisphere) times n_ord/2 azimuths phi_k = (2k-1) pi / (n_ord/2).
 *   dim = 3, kind = MLPG_QUAD_PRODUCT: 6-point Gauss-Legendre in Omega_z
 *     times n_ord/6 azimuths.
 *   dim = 2, kind = MLPG_QUAD_BEAM_DENSE, n_ord = 256: two polar levels times
 *     128 azimuthal sectors, 41 uniform sectors in |phi| <= 10 degrees and 87
 *     over the rest, ordinates at sector midpoints (a fixed stand-in for the
 *     locally refined rule of Sec. 4.3).
 * Order: polar level outer (increasing cosine), azimuth inner (increasing).
 * omega: host [n_ord][dim] out; w: host [n_ord] out.
 * ---------------------------------------------------------------------- */
int mlpg_angular_quadrature(int dim, int n_ord, int kind, double *omega, double *w);

/* ------------------------------------------------------------------------
 * Refined angular quadrature (Sec. 4.3 and Alg. 2): keep every ordinate of a
 * fine goal rule whose ray hits an object and merge the others into the
 * coarsest ordinates of a hierarchy that contain no hitting goal ordinate.
 * Host-only, dim = 2.  The hierarchy is azimuthal bisection of the 2D product
 * rule (mlpg_angular_quadrature, kind MLPG_QUAD_PRODUCT): level L has
 * A_L = 4 * 2^L equal azimuthal sectors per polar level, sector k spanning
 * [2 pi k / A_L, 2 pi (k+1) / A_L] with its ordinate at the midpoint and
 * weight 2 w_p (2 pi / A_L) (w_p the polar weight), so that every sector of
 * level L is the union of two of level L+1.  A goal ordinate (level
 * goal_level) hits when the ray from `src` along its projected direction
 * meets the disk (center, radius) (every ray does when src is inside).  A
 * sector of level >= min_level is kept whole when none of its goal
 * subsectors hits and no coarser kept sector contains it; goal sectors
 * are kept otherwise.  Both polar levels are refined alike (the test depends
 * on the azimuth only).  With no hit the result is the product rule of
 * level min_level; with every goal ordinate hitting it is the goal rule.
 * Order: polar level outer (increasing cosine), azimuth inner (increasing
 * sector start).  The weights sum to 4 pi.
 *   src, center: host [2]; radius >= 0; 0 <= min_level <= goal_level <= 12.
 *   cap = 0: only the count is returned (omega, w may be NULL); otherwise
 *   omega: host [cap][2] out, w: host [cap] out.
 * Returns the number of ordinates, MLPG_ERR_CAPACITY when 0 < cap < count,
 * MLPG_ERR_ARG for invalid levels, radius or pointers.
 * ---------------------------------------------------------------------- */
int mlpg_refined_quadrature(int min_level, int goal_level, const double *src, const double *center, double radius,
                            int cap, double *omega, double *w);

/* ------------------------------------------------------------------------
 * Overlap connectivity (Sec. 3.4, Eq. mlpg-connectivity): j != i is a
 * neighbour of i when |x_i - x_j| <= R_i + R_j.  Lists are in increasing j.
 * Two calls: count fills nbr_off (device [n+1], exclusive prefix sums) and
 * returns the total in *total (host; the call synchronises `stream`); fill
 * then writes nbr_idx (device [*total]).
 *   x: device [n][dim]; R: device [n] support radii (> 0).
 * ---------------------------------------------------------------------- */
int mlpg_neighbors_count(int dim, int64_t n, const double *x, const double *R, int64_t *nbr_off,
                         int64_t *total, void *stream);
int mlpg_neighbors_fill(int dim, int64_t n, const double *x, const double *R, const int64_t *nbr_off,
                        int32_t *nbr_idx, void *stream);

/* ------------------------------------------------------------------------
 * The same overlap lists without any allocation, for callers that cannot
 * allocate device memory while they run (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The search's scratch (the
 * points' bounding box and cells, the cell counts and starts, the points in
 * cell order) lives in a static device array of about 20 MiB that every GPU
 * holds until the process ends; no hipMalloc, hipFree or allocating library
 * call is made.  Counts into nbr_off (device [n+1], exclusive prefix sums),
 * the total into *total (host), then, when it is at most cap, the lists into
 * nbr_idx (device [cap]) -- the lists of mlpg_neighbors_count/_fill exactly.
 *   n: 1 .. 2^20 points (MLPG_ERR_ARG beyond: the array's capacity);
 *   cap: entries nbr_idx holds; cap < *total returns MLPG_ERR_CAPACITY with
 *        *total set and nbr_idx untouched (cap = 0: count only).
 * Synchronises `stream`.  Every call on one GPU uses that GPU's one array,
 * which keeps the previous call's contents (the search clears what must
 * start at zero): calls that overlap on one GPU (other threads or streams)
 * race and must be serialised by the caller.
 * ---------------------------------------------------------------------- */
int mlpg_neighbors_static(int dim, int64_t n, const double *x, const double *R, int64_t *nbr_off,
                          int32_t *nbr_idx, int64_t cap, int64_t *total, void *stream);

/* ------------------------------------------------------------------------
 * Stage 1, geometry (Sec. 3.1, Fig. 1; Sec. 3.4).  Creates a handle.  Each
 * point gets the convex cell obtained by clipping the box
 * [x_i - R_i, x_i + R_i]^dim intersected with the domain box by the
 * half-space on x_i's side of the bisector with every overlap neighbour.
 * The cells tile the domain (a partition of unity in space) as long as every
 * cell lies inside its own support, which is checked and reported.
 *   x: device [n][dim] positions; R: device [n] kernel support radii (the
 *     cubic spline of smoothing length R/2 vanishes beyond R);
 *   nbr_off, nbr_idx: device overlap lists as produced by mlpg_neighbors_*;
 *   dom_lo, dom_hi: host [dim] domain box;
 *   regions: host boxes [n_regions][dim] with material ids; a point of space
 *     takes the material of the last box containing it, 0 if none.
 * dim = 2 (polygons, at most 32 vertices) or 3 (polyhedra of at most 40
 * convex faces with at most 16 vertices each; the faces of a clip are built
 * from the cut points ordered about their centroid).  A cell over capacity
 * fails the call with MLPG_ERR_GEOMETRY.  The overlap lists are validated on
 * the device before any other kernel reads them: nbr_off[0] = 0, offsets
 * non-decreasing and within nbr_off[n], every index in [0, n), never the row
 * itself, strictly increasing along a row; otherwise MLPG_ERR_ARG.  The call
 * synchronises `stream` (it sizes the boundary quadrature).  On success *out
 * owns copies of all inputs.
 * ---------------------------------------------------------------------- */
int mlpg_geometry(mlpg_handle *out, int dim, int64_t n, const double *x, const double *R,
                  const int64_t *nbr_off, const int32_t *nbr_idx, const double *dom_lo,
                  const double *dom_hi, int n_regions, const double *region_lo, const double *region_hi,
                  const int32_t *region_mat, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the geometry workspace for n points with nnz_nbr overlap-list
 * entries in the box [dom_lo, dom_hi] (host [dim]): copies of the inputs,
 * the cells (2D: 32 vertices per cell; 3D: 40 faces of 16 vertices), the
 * pattern, the preconditioner patches and the stage's temporaries.  0 for
 * invalid arguments. */
size_t mlpg_geometry_workspace_bytes(int dim, int64_t n, int64_t nnz_nbr, const double *dom_lo,
                                     const double *dom_hi);

/* ------------------------------------------------------------------------
 * Moving points (Sec. 1: with points that move every time step, as in
 * radiation hydrodynamics, the integration is redone at each step and must
 * need no manual adjustment; Sec. 3.1: the cells depend only on the point
 * positions and kernel extents).  Replaces the positions, radii and overlap
 * lists of an existing handle (same n, dim, domain, regions and material
 * fields) and rebuilds the cells, the boundary quadrature sizing and the
 * pattern.  The handle returns to the state after mlpg_geometry: call
 * mlpg_integrate and mlpg_assemble again before the next mlpg_solve.  The
 * state kept by mlpg_solve (the per-point angular flux coefficients
 * Psi^{n-1} and Phi) stays with the points, so the next backward-Euler step
 * uses the old coefficients with the new functions.
 *   x, R, nbr_off, nbr_idx: device, as for mlpg_geometry (n points).
 * Synchronises `stream`.  Errors: MLPG_ERR_STATE without a geometry,
 * MLPG_ERR_GEOMETRY for a cell over capacity (the handle must then be
 * destroyed), MLPG_ERR_ARG for null pointers.
 * ---------------------------------------------------------------------- */
int mlpg_update_points(mlpg_handle h, const double *x, const double *R, const int64_t *nbr_off,
                       const int32_t *nbr_idx, void *workspace, size_t ws_bytes, void *stream);

typedef struct {
    int64_t n;               /* points */
    int dim;
    int n_mat;               /* 1 + largest material id */
    int64_t nnz;             /* pattern entries: i and its overlap neighbours per row */
    int64_t n_bq;            /* boundary quadrature points (after mlpg_geometry) */
    int64_t oversize_cells;  /* cells reaching beyond their own support radius */
    int64_t failed_cells;    /* cells with no volume or over the face/vertex capacity */
    int64_t fallback_qps;    /* quadrature points whose moment matrix needed a lower order */
    int64_t missing_pairs;   /* co-active pairs absent from the pattern (expected 0) */
    int n_ord;               /* ordinates after mlpg_assemble, else 0 */
    int n_blocks;            /* integrated blocks: n_mat(1+dim) + dim^2 + 2 dim */
} mlpg_info;

/* Sizes and counters; synchronises `stream`-independent state (host only). */
int mlpg_get_info(mlpg_handle h, mlpg_info *info);

/* Cell volumes V_i: device [n] out. */
int mlpg_get_volumes(mlpg_handle h, double *V, void *stream);

/* Cell polygons of a 2D problem (MLPG_ERR_ARG for 3D): nv device [n], verts
 * device [n][cap][2], tags device [n][cap] with tag >= 0 the neighbour index
 * of a bisector edge and tag = -1 - f an edge on domain face f (0:-x 1:+x
 * 2:-y 3:+y).  cap is returned by mlpg_cell_capacity. */
int mlpg_cell_capacity(void);
int mlpg_get_cells(mlpg_handle h, int32_t *nv, double *verts, int32_t *tags, void *stream);

/* Boundary quadrature points of the domain faces (App. A surface map), in
 * the order the inflow data psi_b of mlpg_solve must follow:
 *   y: device [n_bq][dim]; face: device [n_bq] (0:-x 1:+x 2:-y 3:+y ...). */
int mlpg_boundary_points(mlpg_handle h, double *y, int32_t *face, void *stream);

/* ------------------------------------------------------------------------
 * Spatially varying materials (Sec. 5.1: opacities that vary smoothly in
 * space, evaluated at the integration points).  Optional, between
 * mlpg_geometry and mlpg_integrate.  Field r moves the fraction
 *   v_r(y) = a + b prod_alpha cos(k y_alpha + phase)
 * of every volume quadrature point y from material 0 to material mat[r],
 * after the region boxes have set the point's material; so the fractions
 * still sum to one and the integrated blocks become
 *   Mass_g[i,j] = <f_g N_i, N_j>,  D^a_g[i,j] = <f_g d^a N_i, N_j>.
 * With sigma_t, sigma_s given per material at assembly, the cross sections
 * at a point are sum_g f_g sigma_g (a product of sines is a product of
 * cosines with phase -pi/2).
 *   n_fields: 0..8 (0 removes the fields); param: host [n_fields][4]
 *   (a, b, k, phase); mat: host [n_fields], each in [1, 8).  Raises the
 *   handle's material count to cover every mat[r].  Resets the handle to the
 *   state after mlpg_geometry (integrate again before assembling).
 * Errors: MLPG_ERR_ARG for a count or material out of range or a NULL array
 * with n_fields > 0; MLPG_ERR_STATE before mlpg_geometry.
 * ---------------------------------------------------------------------- */
int mlpg_material_fields(mlpg_handle h, int n_fields, const double *param, const int32_t *mat);

/* ------------------------------------------------------------------------
 * Shells of material (the asteroid of Sec. 5.4: an absorbing shell around a
 * centre; annuli in 2D).  Optional, between mlpg_geometry and mlpg_integrate.
 * At every volume quadrature point y the material set by the region boxes is
 * replaced by mat[r] for each shell r with r_in <= |y - centre_r| <= r_out
 * (in order, last match wins); material fields then apply as described
 * above.
 *   n_shells: 0..8 (0 removes the shells); center: host [n_shells][dim];
 *   radii: host [n_shells][2] (r_in, r_out, 0 <= r_in <= r_out); mat: host
 *   [n_shells], each in [0, 8).  Raises the material count to cover every
 *   mat[r]; resets the handle to the state after mlpg_geometry.
 * Errors: MLPG_ERR_ARG for a count, radius or material out of range or a
 * NULL array with n_shells > 0; MLPG_ERR_STATE before mlpg_geometry.
 * ---------------------------------------------------------------------- */
int mlpg_material_shells(mlpg_handle h, int n_shells, const double *center, const double *radii,
                         const int32_t *mat);

/* ------------------------------------------------------------------------
 * Stage 2, integration (Sec. 2.2; Sec. 3.2 and Alg. 1; App. A).  At every
 * quadrature point of every cell (2D: fan triangles from the generator with
 * the 25-point conical-product rule, 5-point Gauss-Legendre on boundary
 * edges; 3D: tetrahedra joining the generator to the fan triangles of every
 * face with the 8-point conical-product rule, 4-point rule on boundary
 * triangles)
 * the RK functions N_j = V_j U_j of order rk_order (0, 1, 2) and their
 * gradients are formed from the moment matrix (batched Cholesky in FP64,
 * falling back one order at a time when a pivot is below 1e-6 of the largest
 * diagonal entry) and accumulated into direction-independent blocks over the
 * overlap pattern:
 *   Mass_g = <N_i,N_j>, D^a_g = <d^a N_i, N_j> per material g,
 *   K^ab = <d^a N_i, d^b N_j>, S_f = (N_i,N_j) on domain face f.
 * Also forms the point-value matrix E_ij = N_j(x_i) (Eq. flux-expansion).
 * MLPG_ERR_CAPACITY when a cell has more candidate functions than the
 * per-cell capacity (64 in 2D, 512 in 3D) or a boundary point more active
 * functions than it stores (32 in 2D, 128 in 3D).  MLPG_ERR_ARG when two
 * functions active at one quadrature point are not overlap neighbours (the
 * caller's lists were incomplete; the blocks would silently lose entries).
 * ---------------------------------------------------------------------- */
int mlpg_integrate(mlpg_handle h, int rk_order, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the integration workspace of handle h (after mlpg_geometry and any
 * mlpg_material_fields / mlpg_material_shells, which set the material
 * count): the blocks, the point-value matrix, the boundary quadrature and the
 * surface-row offsets; in 3D with one material and no fields or shells also
 * a region for the cells' weighted-value panels, whose Gram products are
 * formed on the matrix cores a batch of cells at a time (up to 1024 cells of
 * 2 MiB estimated each; a problem with larger panels takes smaller batches).
 * 0 before mlpg_geometry or for an invalid order. */
size_t mlpg_integrate_workspace_bytes(mlpg_handle h, int rk_order);

/* Pattern and blocks for parity checks.  row_off: device [n+1]; col: device
 * [nnz]; blocks: device [n_blocks][nnz] in the order
 *   for g: Mass_g, D^0_g .. D^{dim-1}_g;  K^ab (a-major);  S_0 .. S_{2dim-1};
 * E: device [nnz]. */
int mlpg_get_pattern(mlpg_handle h, int64_t *row_off, int32_t *col, void *stream);
int mlpg_get_blocks(mlpg_handle h, double *blocks, double *E, void *stream);

/* ------------------------------------------------------------------------
 * Stage 3, assembly (Sec. 4.1, Eq. weak-transport; Sec. 4.2 operators).
 * Combines the blocks with the cross sections, a0 = 1/(c dt) (0 = steady)
 * and the SUPG lengths tau_i into per-ordinate-combinable value streams:
 *   L_m = sum_g (a0 + sigma_t,g) Mass_g
 *       + sum_a W^a [(a0 tau_i - 1) D^a + tau_i sum_g sigma_t,g D^a_g]
 *       + tau_i sum_ab W^a W^b K^ab + sum_f max(0, W.n_f) S_f,   W = Omega_m
 *   T_m = a0 (Mass + tau_i W.D),   MS_m = (1/4pi) sum_g sigma_s,g (Mass_g + tau_i W.D_g)
 * and the point-Jacobi diagonal of every L_m.
 *   n_ord: 1..256 ordinates; omega: host [n_ord][dim]; w: host [n_ord];
 *   sigma_t, sigma_s: host [n_mat];
 *   tau: device [n] SUPG lengths (Sec. 4.1: about the point spacing);
 *   precision: MLPG_FP64 (every inner solve in FP64) or MLPG_MIXED (each
 *     inner solve is FP64 iterative refinement: the residual f - L_m x is
 *     formed with FP64 values, and each correction is an FP32 GMRES solve
 *     with FP32 values, FP32 vectors and FP32 SpMV accumulation, FP64
 *     Gram-Schmidt sums and Hessenberg; the stopping test is the FP64 one).
 * May be called again with new cross sections, dt or ordinates.
 * ---------------------------------------------------------------------- */
int mlpg_assemble(mlpg_handle h, int n_ord, const double *omega, const double *w, int n_mat,
                  const double *sigma_t, const double *sigma_s, double inv_c_dt, const double *tau,
                  int precision, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the assembly workspace (after mlpg_integrate): the state Psi, Phi
 * (kept at the start of the workspace: passing the same workspace again with
 * the same n_ord keeps the state; a different one receives a copy of it, and
 * the previous one must stay valid until the call returns), the value
 * streams, coefficient tables, surface rows, Jacobi scaling, the
 * diffusion-synthetic operators and, for MLPG_MIXED, the FP32 copies. */
size_t mlpg_assemble_workspace_bytes(mlpg_handle h, int n_ord, int precision);

/* One operator application Y = op X for all ordinates (parity accessor):
 * which = MLPG_OP_L, MLPG_OP_T, MLPG_OP_MS or MLPG_OP_SRC (Mass + tau W.D);
 * X, Y: device [n][n_ord]. */
int mlpg_apply(mlpg_handle h, int which, const double *X, double *Y, void *stream);

/* ------------------------------------------------------------------------
 * Stage 4, one backward-Euler step (Sec. 4.1) or a steady solve (a0 = 0),
 * by the Krylov iteration of Sec. 4.2:
 *   b_psi = L^-1 (T Psi^{n-1} + r),  b_phi = D b_psi,
 *   (I - D L^-1 MS) Phi = b_phi by GMRES from the previous Phi,
 *   Psi = L^-1 MS Phi + b_psi,
 * with r = (N_i, |W.n| psi_b)_{W.n<0} + <N_i, q_m> + tau_i W.<dN_i, q_m>,
 * q expanded in the RK basis from its point values.  Every L_m^-1 is a
 * restarted GMRES with right point-Jacobi preconditioning, all ordinates
 * advanced together.  Psi^{n-1} is the handle's state (zero until
 * mlpg_set_state); on return the state holds the new Psi and Phi.
 *   q: device [n][n_ord] source point values (per steradian);
 *   psi_b: device [n_bq][n_ord] inflow values at mlpg_boundary_points, or NULL (vacuum);
 *   phi_coef: device [n] out, Phi; phi_point: device [n] out, phi(x_i) (may be NULL);
 *   psi_out: device [n][n_ord] out, Psi (may be NULL);
 *   opts: host, NULL for defaults; info: host out, may be NULL.
 * The call synchronises `stream` at Krylov convergence checks.  An inner
 * solve that reaches max_inner before tol_inner ends the step at once (the
 * outer iteration needs every L_m^-1 as a fixed linear map): the call returns
 * MLPG_ERR_NOT_CONVERGED with the outputs and the state unwritten and `info`
 * counting the work done.  When only the outer iteration reaches max_outer,
 * it returns MLPG_ERR_NOT_CONVERGED with the outputs of the last iterate
 * written.
 * ---------------------------------------------------------------------- */
typedef struct {
    double tol_inner;     /* ||f - L_m x|| <= tol ||f|| per ordinate (default 1e-13) */
    double tol_outer;     /* outer relative residual (default 1e-12; MLPG_MIXED stops at 1e-10 at the
                             tightest: its inner solves make the outer operator linear only to about
                             tol_inner / (1 - c)) */
    int restart_inner;    /* GMRES restart length, <= 60 (default 30); above 30 each Gram-Schmidt pass
                             runs in two chunks over the basis and the solve workspace holds two more
                             FP64 fields of the inner systems' shape (same sums, bit for bit) */
    int restart_outer;    /* <= 60 (default 30) */
    int max_inner;        /* Arnoldi steps per ordinate per solve (default 3000) */
    int max_outer;        /* (default 500) */
    int check_every;      /* Arnoldi steps queued ahead of the host convergence check (default 3) */
    double tol_inner_lo;  /* MLPG_MIXED: FP32 correction solves stop at this relative residual, or earlier
                             for an ordinate whose remaining gap to tol_inner is smaller (default 3e-5) */
    int max_refine;       /* MLPG_MIXED: FP64 refinement steps per inner solve (default 12) */
    int accel;            /* outer iteration: MLPG_ACCEL_NONE (default) or MLPG_ACCEL_DSA, a
                             diffusion-synthetic right preconditioner (see below) */
    int precond;          /* inner solves: MLPG_PRECOND_JACOBI (default, point Jacobi) or
                             MLPG_PRECOND_PATCH (patch block Jacobi, see below) */
    int graphs;           /* 1: every restart cycle of an inner solve (its Arnoldi steps, the
                             least-squares update, the new residual and the next cycle's start) is
                             captured once per set of launch arguments as a HIP graph and replayed;
                             the host then waits once per cycle instead of every few steps, and
                             steps after the last system converges return at their device gates.
                             0 (default): launched one by one, the host stopping a few steps after
                             the last system converges.  The results are the same bit for bit.
                             Kernel timing (mlpg_profile_begin) launches one by one. */
} mlpg_solve_opts;

/* Right preconditioning of the inner solves L_m x = f (Sec. 4.2 preconditions
 * every L_m; the paper factors each with ILUT, a sequential algorithm).
 * MLPG_PRECOND_JACOBI scales by 1 / L_m[i,i].  MLPG_PRECOND_PATCH groups the
 * points into spatial patches -- the cells of a uniform grid of side
 * 2 (|domain| / n)^(1/dim) over the domain box, each cell's points in
 * increasing index, split into chunks of at most 16 (2^dim points per patch
 * on a lattice) -- and applies, per patch P and ordinate m, the inverse of the
 * dense block L_m[P, P] (surface terms included; Gauss-Jordan elimination
 * with partial pivoting, a singular block falls back to its diagonal).  It
 * cuts the iteration counts several-fold where point Jacobi stalls (wide
 * kernels in 3D, rows whose diagonal entry is small or negative on coarse
 * point sets).  The patches are built on the first solve after
 * mlpg_geometry or mlpg_update_points, the inverses on the first solve after
 * mlpg_assemble (n_patch_entries * n_ord values, FP64, plus an FP32 copy for
 * MLPG_MIXED; about 8 n n_ord values for 3D lattices).  The converged
 * solution does not depend on the choice. */
enum { MLPG_PRECOND_JACOBI = 0, MLPG_PRECOND_PATCH = 1 };

/* Y = M^-1 X for every ordinate with the patch block-Jacobi preconditioner
 * of the assembled operators (parity accessor; builds the inverses when they
 * are not current).  X, Y: device [n][n_ord], distinct; *n_patches (host, may
 * be NULL) gets the patch count; workspace: a solve workspace for options
 * with precond = MLPG_PRECOND_PATCH (or NULL). */
int mlpg_apply_patch_precond(mlpg_handle h, const double *X, double *Y, int64_t *n_patches, void *workspace,
                             size_t ws_bytes, void *stream);

/* Acceleration of the scattering iteration (Sec. 6 names it as needed for
 * scattering-dominated problems; Sec. 4.2 runs the outer GMRES without a
 * preconditioner).  MLPG_ACCEL_DSA preconditions the outer GMRES on
 * (I - D L^-1 MS) Phi = b from the right with
 *   P^-1 v = v + C^-1 (Ms v),
 * where, on the same pattern and with the same test functions,
 *   C[i,j]  = (1 / (3 sigma_t,i)) sum_a K^aa[i,j] + sum_g sigma_a,g Mass_g[i,j] + 1/2 sum_f S_f[i,j]
 *   Ms[i,j] = sum_g sigma_s,g Mass_g[i,j]
 * is the diffusion approximation of the scattering correction (Marshak
 * vacuum terms on the domain faces); sigma_a,g = sigma_t,g - sigma_s,g +
 * 1/(c dt), and sigma_t,i is point i's mass-weighted mean of sigma_t,g +
 * 1/(c dt).  C x = r is solved by GMRES(30) with point Jacobi to a relative
 * residual of 1e-4 (at most 2,000 steps).  The outer iteration is then
 * flexible GMRES: it keeps every P^-1 v_j and updates Phi with them, so its
 * residual is that of the unaccelerated system whatever the accuracy of the
 * diffusion solve; the converged Phi is the same as without acceleration, and
 * the outer iteration count drops where scattering dominates.  The solve
 * workspace holds restart_outer more fields of n values. */
enum { MLPG_ACCEL_NONE = 0, MLPG_ACCEL_DSA = 1 };

typedef struct {
    int outer_iters;
    int inner_solves;            /* batched L^-1 applications */
    int64_t inner_iters;         /* Arnoldi steps summed over ordinates and solves */
    int64_t inner_sweeps;        /* batched Arnoldi steps (one SpMV over all ordinates each) */
    double outer_res;            /* final outer relative residual */
    double inner_res_max;        /* largest final inner relative residual */
    int converged;               /* 1 if every solve met its tolerance */
    int refinements;             /* MLPG_MIXED: FP64 refinement steps summed over inner solves */
    int fp64_completions;        /* MLPG_MIXED: inner solves finished in FP64 after the FP32
                                    corrections stagnated or the refinement budget was spent */
    int64_t accel_iters;         /* MLPG_ACCEL_DSA: Arnoldi steps of the diffusion solves */
} mlpg_solve_info;

void mlpg_default_opts(mlpg_solve_opts *o);
int mlpg_set_state(mlpg_handle h, const double *psi, void *stream);
int mlpg_get_state(mlpg_handle h, double *psi, double *phi, void *stream);
int mlpg_solve(mlpg_handle h, const double *q, const double *psi_b, double *phi_coef, double *phi_point,
               double *psi_out, const mlpg_solve_opts *opts, mlpg_solve_info *info, void *workspace,
               size_t ws_bytes, void *stream);

/* Bytes of the solve workspace for opts (NULL: defaults) after mlpg_assemble:
 * right-hand sides and intermediate fields, the batched inner Krylov space
 * (restart_inner), the outer one (restart_outer), the FP32 space and
 * refinement vectors of MLPG_MIXED, the diffusion solve's space of
 * MLPG_ACCEL_DSA and the patch inverses of MLPG_PRECOND_PATCH (rebuilt when
 * the operators change or the workspace moves).  0 for invalid options. */
size_t mlpg_solve_workspace_bytes(mlpg_handle h, const mlpg_solve_opts *opts);

/* Point values out[i] = sum_j N_j(x_i) coef[j] (Eq. flux-expansion);
 * coef, out: device [n]. */
int mlpg_point_values(mlpg_handle h, const double *coef, double *out, void *stream);

/* ------------------------------------------------------------------------
 * Kernel timing for roofline reports.  Between mlpg_profile_begin and
 * mlpg_profile_end every launch of the kernel classes below is bracketed by
 * HIP events on the stream it runs on, and the algorithmic bytes it must
 * move (each input and output counted once, gathered vectors once) are
 * accumulated.  Process-wide; not thread-safe.
 *   class 0: SpMV of the transport operator L (all ordinates); its bytes are
 *            the sweep's own per unit (row and ordinate): the value streams and
 *            column indices once per row, shared by the ordinates, x read and y
 *            written once (a fused normalisation of the next basis vector is
 *            Gram-Schmidt traffic and not counted here)
 *   class 1: Gram-Schmidt pass A (projections of the new vector and of the
 *            operator output on the basis)
 *   class 2: Gram-Schmidt pass B (reorthogonalised basis vector, projected
 *            operator output, its norm)
 *   class 3: end-of-cycle pass A (projections of the last vector only)
 * Only the first 4096 launches of each class in a session are bracketed.
 * mlpg_profile_end synchronises the device and fills, per class (arrays of
 * MLPG_PROF_CLASSES): total time in ms, launch count and bytes of the
 * bracketed launches.
 * ---------------------------------------------------------------------- */
#define MLPG_PROF_CLASSES 4
int mlpg_profile_begin(void);
int mlpg_profile_end(double *ms, int64_t *launches, double *bytes);

/* ------------------------------------------------------------------------
 * Launch-shape autotuning of the transport sweep.  Before the first solve of
 * a problem shape (rows n, ordinates, value streams, value size) the library
 * times every candidate launch shape of the sweep on the problem's own
 * operator, as the inner solver calls it and with the caches evicted by a
 * read of the solve's Krylov basis before each timed launch (as between two
 * sweeps of the Arnoldi loop), and keeps the fastest in a process-wide table
 * used by every later sweep of that shape:
 *   n_ord >= 48, form 0 (stream values read with scalar loads by each wave):
 *     2, 4 or 8 waves per workgroup, 1 or 2 (row, 64-ordinate) items per
 *     wave, workgroups renumbered so that each of the 8 dies walks one
 *     contiguous row range (xcd_split = 8) or not (1);
 *   48 <= n_ord <= 64 with 6 or 10 streams, form 1 (stream values staged
 *     through LDS by the workgroup, two rounds deep): 4 or 8 waves (4 only
 *     for 10 FP64 streams), 2 or 4 rounds of one row per wave, xcd_split 8;
 *   n_ord > 64 with 6 or 10 streams, form 2 (as form 0 with 2 or 4 adjacent
 *     ordinates per lane, so that an item is a row and 128 or 256 ordinates;
 *     n_ord a multiple of the count, and the count only where it makes fewer
 *     items than half of it: 96 and 128 ordinates take 2, 256 take 2 or 4):
 *     2, 4 or 8 waves, 1 item per wave, xcd_split 8 or 1;
 *   n_ord < 48: 128, 256 or 512 threads per workgroup.
 * mlpg_set_autotune(0) keeps the built-in shape (form 0, 4 waves, 1 item,
 * split 8; 256 threads) for shapes not yet in the table, (1) measures again
 * (the default), (2) empties the table.  Every shape computes each row's sums
 * in the same order, so the results do not depend on the choice.
 * mlpg_get_tuning copies up to cap entries to out (host) and returns the
 * table's size.  mlpg_set_tuning inserts or replaces the entry of
 * entry->(n, n_ord, streams, value_bytes) (host struct; us_best and
 * us_default are stored as given), so that a table saved from one process
 * can be loaded into the next, or a shape pinned; MLPG_ERR_ARG for a shape
 * outside the ranges above (form 1: 4 or 8 waves, 1..64 rounds; forms 0 and
 * 2: 1..8 waves, 1..64 items; form 2: 2 or 4 ordinates per lane; xcd_split 1
 * or 8; threads in [n_ord, 512]).
 * Process-wide; the table is guarded by a lock.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    int n_ord, streams, value_bytes;
    int form;                    /* 0, 1 or 2 as above (0 for n_ord < 48) */
    int waves_per_block, items_per_wave, rounds, xcd_split, threads;
    int ords_per_lane;           /* form 2: 2 or 4; otherwise 1 */
    float us_best, us_default;   /* measured duration of the chosen and of the built-in shape */
} mlpg_tune_entry;
int mlpg_set_autotune(int mode);
int mlpg_get_tuning(int cap, mlpg_tune_entry *out);
int mlpg_set_tuning(const mlpg_tune_entry *entry);

/* ------------------------------------------------------------------------
 * Progress reports for long solves.  When set, the library calls
 * fn(user, level, iters, resid) on the calling host thread after every
 * batched Krylov solve: level 0 = an inner solve over all ordinates, 1 = the
 * outer solve; iters = Arnoldi steps of that solve summed over its systems;
 * resid = its largest final relative residual.  Process-wide; NULL turns it
 * off.  The callback must not call back into the library.
 * ---------------------------------------------------------------------- */
typedef void (*mlpg_progress_fn)(void *user, int level, int64_t iters, double resid);
int mlpg_set_progress(mlpg_progress_fn fn, void *user);

/* Releases the handle and all its device memory (NULL is ignored). */
void mlpg_destroy(mlpg_handle h);

#ifdef __cplusplus
}
#endif
#endif /* MLPG_H */
