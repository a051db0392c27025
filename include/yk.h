/*
 * yk.h -- C ABI of libyk, an MI355X (gfx950) implementation of one implicit
 * time step of the 2-D heat equation done as a modified Helmholtz (Yukawa)
 * solve, after Kropinski & Quaife, "Fast integral equation methods for the
 * heat equation and the modified Helmholtz equation in two dimensions"
 * (arXiv 1007.5335).
 *
 * General conventions
 *  - Every array argument is a DEVICE pointer to FP64 data unless marked
 *    HOST.  The caller owns all arrays; the library owns only its context,
 *    its cached trees/operator tables and its workspace.  Inputs and outputs
 *    must not alias.
 *  - Points are interleaved [n][2] (x, y).  Curve 0 of a boundary is the outer
 *    curve, traversed counter-clockwise; holes are traversed clockwise; the
 *    unit normals point out of the domain on every curve; the curvature is
 *    signed (+1/R on a counter-clockwise circle).
 *  - Kernel normalisation of the sums (Sec. 2): the library sums carry
 *    K0(|x-y|/alpha)/(2 pi), i.e. the Green's function G = K0/(2 pi alpha^2)
 *    without its 1/alpha^2; the heat step applies that factor itself.
 *  - Errors are returned as status codes; no C++ exception crosses the ABI.
 *    Arguments are checked before any work; on YK_ERR_ARG outputs are left
 *    untouched.  yk_last_error() returns a per-context message.
 *  - All work is ordered on the context's stream (yk_set_stream).  The two
 *    sum entry points are asynchronous; the solver entry points synchronise
 *    the stream, because GMRES reads residual scalars on the host.
 *  - A context is not thread-safe; use one per host thread.
 *  - Trees and operator tables are cached per context, keyed by the point
 *    arrays' addresses and sizes and by alpha.  After changing point
 *    coordinates in place, call yk_invalidate_geometry().
 */
#ifndef YK_H
#define YK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct yk_ctx_s *yk_ctx;

typedef enum {
    YK_OK = 0,
    YK_ERR_ARG = -1,        /* invalid argument (null pointer, n <= 0, alpha <= 0, ...) */
    YK_ERR_HIP = -2,        /* a HIP runtime call failed */
    YK_ERR_NOMEM = -3,      /* device or host allocation failed */
    YK_ERR_NOCONV = -4,     /* GMRES hit max_iter; the best iterate is written */
    YK_ERR_NONFINITE = -5,  /* a residual or a result became NaN/Inf */
    YK_ERR_INTERNAL = -6
} yk_status;

enum {
    YK_PREC_FP64 = 0,       /* every sum in FP64 */
    YK_PREC_MIXED = 1,      /* FP32 sums inside GMRES, FP64 outer residual and volume pass */
    YK_PREC_FP32 = 2        /* as MIXED, and the volume pass in FP32 too */
};

typedef struct {
    int precision;          /* YK_PREC_* */
    double fmm_tol;         /* target relative accuracy of the sums; picks p when p == 0 */
    int p;                  /* expansion order (terms -p..p), 0..31; 0 = derived from
                               fmm_tol.  The order used is the smallest of 8, 12,
                               16, 20, 24, 28, 31 not below p (yk_plan_info.p);
                               p > 31 is rejected (YK_ERR_ARG) */
    int leaf_size;          /* target mean number of points per leaf box (the
                               adaptive tree splits a box while it holds more
                               than leaf_size / 2 points) */
    int direct;             /* 1 = all sums by O(N^2) direct summation */
    int gmres_m;            /* Krylov dimension before a restart */
    int debug_flags;        /* bit0: synchronise and check after every kernel;
                               bit1: run the near field on the context's stream
                               (by default a tree of fewer than 8192 leaves
                               runs it on a second stream, overlapped with the
                               far field; larger trees always run it in turn);
                               bit2: capture the density operator in a HIP
                               graph and replay it (off by default: slower
                               than eager launches here);
                               bit3: recompute the charges' multipoles in the
                               heat step's second volume pass instead of
                               reusing those of the first (same charges);
                               bit4: store the cached charge-to-charge
                               near-field values for both orders of every
                               pair of leaves (by default each pair block of
                               neighbouring leaves is stored once and applied
                               both ways, when every leaf holds at most 64
                               charges);
                               bit5: run the warm-start network's inference
                               layer by layer (general matrix products and
                               stored activations) instead of the fused
                               kernel */
    int near_cache_mb;      /* device memory (MiB) a tree may spend on its cached
                               near-field interaction values; 0 = evaluate the
                               near-field kernels on every call */
    int tree;               /* YK_TREE_*: the quad-tree of Sec. 3.1.  AUTO (default):
                               the uniform tree unless it would hold more than
                               six times N / leaf_size leaves (points clustered
                               so strongly that most of its leaves are nearly
                               empty), then the adaptive one.  UNIFORM: every
                               leaf at one level (the smallest level whose
                               point-weighted occupancy is <= leaf_size), U and
                               V lists.  ADAPTIVE: boxes split while they hold
                               more than leaf_size / 2 points, then 2:1 balanced
                               (touching leaves differ by at most one level);
                               U, V, W (multipoles of finer boxes evaluated at a
                               leaf's points) and X (a coarser leaf's sources
                               into a box's local expansion) lists; the near
                               field is evaluated on the fly (near_cache_mb
                               unused) */
} yk_options;

enum { YK_TREE_UNIFORM = 0, YK_TREE_ADAPTIVE = 1, YK_TREE_AUTO = 2 };

typedef struct {
    int32_t n_curves;             /* >= 1; curve 0 outer, 1.. holes */
    const int64_t *offset;        /* HOST [n_curves + 1]; N_k = offset[k+1] - offset[k] */
    const double *xy;             /* [N][2] nodes y_j, N equispaced in each curve's parameter */
    const double *normal;         /* [N][2] unit normals, outward from the domain */
    const double *speed;          /* [N] |y'(theta_j)|; weights w_j = (2 pi / N_k) speed_j */
    const double *curvature;      /* [N] signed curvature kappa_j */
} yk_boundary;

typedef struct {
    int iters;               /* total GMRES iterations (inner ones in mixed precision) */
    int outer_iters;         /* refinement sweeps (mixed precision), else 0 */
    int guess_used;          /* 0 zero, 1 caller's guess, 2 learned guess */
    int matvecs;             /* operator applications */
    double res0;             /* ||b - A x0|| / ||b|| */
    double res_final;        /* ||b - A x|| / ||b|| (true residual, FP64) */
    double ms[8];            /* stage times: 0 tree, 1 volume->nodes, 2 solve,
                                3 volume+layer->volume, 4 guess, 5-7 spare */
} yk_stats;

/* Fills *opt with defaults: FP64, fmm_tol 1e-10, p 0, leaf_size 64,
 * direct 0, gmres_m 60, debug_flags 0, near_cache_mb 16384.
 *
 * Cached near field: the near-field interaction values (K0 for charges, the
 * double-layer kernel's two components for dipoles) depend only on the points
 * and alpha, so a tree caches them on its first evaluation for each target
 * set when they fit in near_cache_mb (8 bytes per charge pair and 16 per
 * dipole pair in FP64, half in FP32); later evaluations on the same tree read
 * them instead of evaluating Bessel series.  The cache lives and dies with
 * the tree (new points, alpha, p, leaf_size or yk_invalidate_geometry). */
void yk_default_options(yk_options *opt);

/* Creates a context on the current HIP device.  opt may be NULL (defaults). */
yk_status yk_create(const yk_options *opt, yk_ctx *out);
yk_status yk_destroy(yk_ctx ctx);
/* Binds the context to a hipStream_t (NULL = the null stream). */
yk_status yk_set_stream(yk_ctx ctx, void *hip_stream);
/* Replaces the options; cached trees are dropped when p/leaf_size change. */
yk_status yk_set_options(yk_ctx ctx, const yk_options *opt);
/* The message of the context's last failed call; with ctx == NULL, why the
 * last yk_create on the calling thread failed. */
const char *yk_last_error(yk_ctx ctx);
/* Drops every cached tree and operator table. */
yk_status yk_invalidate_geometry(yk_ctx ctx);

/*
 * Volume potential as a weighted point sum (Sec. 2, eq. vol_potential; Sec. 3.1
 * evaluates it with an FMM):
 *   out[i] = sum_{j : |t_i - s_j| > 0} q[j] K0(|t_i - s_j| / alpha) / (2 pi).
 * tgt_xy == NULL means targets are the sources (n_tgt ignored); the self pair
 * is then skipped, and so is any pair of coincident points.
 * src_xy [n_src][2], q [n_src], tgt_xy [n_tgt][2], out [n_tgt or n_src].
 */
yk_status yk_volume_potential(yk_ctx ctx, int64_t n_src, const double *src_xy, const double *q,
                              int64_t n_tgt, const double *tgt_xy, double alpha, double *out);

/*
 * Double-layer potential (Sec. 2, the representation of U^h, without 1/alpha^2):
 *   out[i] = sum_j w_j sigma_j D(t_i, y_j) / (2 pi),
 *   D(x, y) = d/dnu_y K0(|x - y|/alpha) = (1/alpha) K1(r/alpha) (x - y).n_y / r,
 *   w_j = (2 pi / N_k) speed_j.
 * tgt_xy == NULL evaluates on the curve at the nodes (n_tgt ignored, out has
 * N entries) with the corrected trapezoid rule: the diagonal term is
 * w_j D_jj sigma_j / (2 pi) with D_jj = kappa_j (-1/2 + zeta(3) w_j^2 /
 * (8 pi^2 alpha^2)) -- the kernel's limit -kappa/2 along the curve (Sec. 2)
 * plus the generalised Euler-Maclaurin error of its t^2 log|t| term, which
 * makes the rule fifth order in the node spacing (it stands where the paper
 * uses Alpert's hybrid rule, Sec. 3.2); off the curve, pairs at distance zero
 * are skipped.  The density solves and heat steps use the same rule.
 */
yk_status yk_double_layer_apply(yk_ctx ctx, const yk_boundary *bnd, const double *sigma,
                                int64_t n_tgt, const double *tgt_xy, double alpha, double *out);

/*
 * Solves the trapezoid discretisation of the second-kind equation
 * (eq. dirichlet:inteqn multiplied by -2 alpha^2; Sec. 3.2, eq. discrete_sys):
 *   sigma_j - 2 * DL[w sigma](y_j) = -2 alpha^2 g_j
 * by GMRES (restarted every gmres_m iterations), stopping when
 * ||b - A sigma||_2 <= tol ||b||_2.  g [N] Dirichlet data of the homogeneous
 * problem; sigma0 [N] initial guess or NULL (zero); sigma [N] output.
 * On YK_ERR_NOCONV the best iterate is written.  stats may be NULL.
 */
yk_status yk_gmres_density(yk_ctx ctx, const yk_boundary *bnd, double alpha, const double *g,
                           const double *sigma0, double tol, int max_iter, double *sigma,
                           yk_stats *stats);

/*
 * One backward-Euler step (Sec. 2: alpha^2 = dt, B = u^N + dt F^N), split into
 * U^p (eq. particular) and U^h (eq. mod_helm_hom):
 *   q       = vol_w * B
 *   U^p     = (V[q] + B * C_self) / alpha^2   on volume points and nodes
 *   g       = f_next - U^p on the nodes
 *   sigma   solves A sigma = -2 alpha^2 g     (GMRES to tol)
 *   u_next  = U^p + DL[w sigma] / alpha^2     at every volume point
 * B [n_vol] must already be extended to every volume point (values outside
 * the domain are the caller's extension, Sec. 3.1).  vol_w [n_vol] quadrature
 * weights.  flags bit0: volume points are centres of square cells of area
 * vol_w = h^2, and each gets the weight of its own cell instead of the
 * skipped self pair: the weight that makes the lattice rule exact for
 * constant B (the kernel integrates to 1 over the plane),
 *   C_self = alpha^2 - (h^2 / 2pi) sum_{j in Z^2, j != 0} K0(|j| h / alpha),
 * and for h / alpha < 0.005 its expansion (1/2pi) int_cell K0(|y|/alpha) dA
 * + kappa h^2, kappa = 0.0396864785674955 the lattice correction of the
 * kernel's logarithmic singularity ((c - Z'(0)/2) / (2 pi), c the mean of
 * log|u| over the unit cell, Z the Epstein zeta function of the square
 * lattice).  With it the rule on a uniform grid is about fourth order in
 * h / alpha where the cell integral alone is second order, and it tends to
 * alpha^2 (U^p = B) for cells much larger than alpha.  The distinct cell
 * areas of vol_w are found on the first call for an array (at most 65535).
 * f_next [N] boundary data at t^{N+1}.  sigma_io [N]: in = initial guess,
 * out = sigma^{N+1}.  flags bit1: ignore sigma_io on input (zero guess).
 * u_next [n_vol] (meaningful at points inside the domain).
 * Near-boundary evaluation (on unless flags bit2): at volume points on the
 * domain side of a curve and closer to it than 4 local node spacings, where
 * the trapezoid rule loses accuracy, U^h comes from the curves'
 * trigonometric interpolants (Sec. 3.2 interpolates sigma in Fourier space):
 * the point is projected onto its curve (theta*, distance d, local spacing
 * s), U^h is evaluated at 6 check points at 1..6 spacings along the inward
 * normal with the trapezoid rule on 8 times as many nodes, its limit on the
 * curve is g(theta*), and the point takes the degree-6 polynomial in d / s
 * through these values.  The set of such points, their projections and the
 * finer nodes are built on the first step for a (boundary, vol_xy) pair and
 * reused; each curve's nodes must be equispaced in a periodic parameter (as
 * the trapezoid weights assume).  Candidates are points within 5 spacings of
 * their nearest node; a point near two curves takes the nearest one.
 * The context keeps a copy of the density it returned and of A sigma; when the
 * next call passes that same density (bitwise) for the same boundary, alpha
 * and FMM options, its residual is formed from the kept A sigma instead of a
 * new operator application.
 */
yk_status yk_heat_step(yk_ctx ctx, const yk_boundary *bnd, int64_t n_vol, const double *vol_xy,
                       const double *vol_w, const double *B, int flags, const double *f_next,
                       double dt, double tol, double *sigma_io, double *u_next, yk_stats *stats);

/*
 * One step of (1 - alpha^2 Lap) u = B, u = f_next on the curves (eq.
 * mod_helm_forced), on a uniform cell-centred grid: the grid form of
 * yk_heat_step, with alpha^2 passed as it is (backward Euler: dt; extrapolated
 * Gear: 2 dt / 3; times the diffusivity, see yk_rhs_imex).
 *   grid     the cells: point j nx + i at (x0 + (i + 1/2) h, y0 + (j + 1/2) h);
 *            the library generates the coordinates; every boundary node must
 *            have two cells of the grid beyond it on each side
 *   B        [nx ny] device, at every cell (the caller's extension outside
 *            the domain, e.g. yk_rhs_imex)
 *   U^p      = (V[h^2 B] + B C_self) / alpha^2 at the cell centres (C_self as
 *            for yk_heat_step flags bit0), and on the nodes by tensor cubic
 *            Lagrange interpolation of these values (the point-grid form of
 *            evaluating the leaf polynomials of Sec. 3.1)
 *   g        = f_next - U^p on the nodes;  sigma solves A sigma = -2 alpha^2 g
 *   u_next   = U^p + DL[w sigma] / alpha^2 at the cell centres, with the
 *            near-boundary evaluation of yk_heat_step (off with flags bit2)
 * flags bit1: zero initial guess.  flags bit3: the box code instead
 * (yk_box_potential: U^p = V / alpha^2 of the leaves' cubic fits of B at the
 * cells, and on the nodes the leaf polynomials fitted to those values; grid
 * sides multiples of 4 cells).  sigma_io, u_next, stats as for yk_heat_step
 * (stats->ms[1] is the U^p stage).  Outside the domain u_next is not
 * meaningful.  YK_ERR_ARG when a node's interpolation stencil leaves the grid.
 */
typedef struct {
    double x0, y0;      /* lower-left corner of the gridded square */
    double h;           /* cell side */
    int64_t nx, ny;     /* cells per row, rows (4 .. 2^20 each, nx ny < 2^31) */
} yk_grid;

yk_status yk_heat_step_grid(yk_ctx ctx, const yk_boundary *bnd, const yk_grid *grid, const double *B, int flags,
                            const double *f_next, double alpha2, double tol, double *sigma_io, double *u_next,
                            yk_stats *stats);

/*
 * The box code of Sec. 3.1 (eq. volume_potential and the leaf polynomials) on
 * a uniform grid whose sides are multiples of 4 cells: the cells form leaves
 * of 4 x 4; on each leaf B is replaced by its least-squares cubic (ten
 * monomials in the leaf's coordinates) through the 16 cell values, and
 *   V(x) = sum over leaves int_leaf K0(|x - y|/alpha)/(2 pi) cubic(y) dy
 * (the sums' normalisation: U^p = V / alpha^2) is evaluated at every cell --
 * the near field (a leaf and its 3 x 3 neighbours) from tables of the
 * monomials' integrals, the rest by the FMM with the leaves' polynomial
 * multipoles (tables per (h, alpha), built on the first call).
 *   grid      the cells (as for yk_heat_step_grid)
 *   B         [nx ny] device, cell values
 *   V         [nx ny] device, out
 *   pts       [n_pts][2] device (optional): points inside the grid; pts_vals
 *             [n_pts] device receives there the leaf polynomial fitted to V
 *             (the polynomials C^i_j of Sec. 3.1)
 * YK_ERR_ARG for sides that are not multiples of 4 (or above 2^17 cells).
 */
yk_status yk_box_potential(yk_ctx ctx, const yk_grid *grid, const double *B, double alpha, double *V,
                           int64_t n_pts, const double *pts, double *pts_vals);

/*
 * The box code on the childless boxes of an adaptive quad-tree (Sec. 3.1: the
 * square D is level 0, each box splits into four, leaves at any level), each
 * leaf with its own 4 x 4 cell-centred grid:
 *   root      HOST [3]: x0, y0, side of the square D
 *   level, ix, iy  HOST [n_leaves]: leaf k is the box of level level[k]
 *             (0 .. 13) at position (ix[k], iy[k]) in that level's 2^l x 2^l
 *             grid; the leaves must not overlap and touching leaves must be
 *             at most one level apart (2:1 balance), else YK_ERR_ARG
 *   vals      [n_leaves][16] device: B at the leaf's cells, cell t = jj 4 + ii
 *             at (x0 + (ix + (ii + 1/2)/4) s, y0 + (iy + (jj + 1/2)/4) s),
 *             s = side / 2^level
 *   V         [n_leaves][16] device, out: V (as yk_box_potential) at the cells
 * The tree over the cells' centres is the library's adaptive tree (its leaves
 * are the given ones); near-field tables per (level, neighbour level,
 * offset), polynomial multipoles per level, X-list (coarser leaf -> finer
 * box) tables per (levels, offset), and the W lists evaluated at the cells.
 */
yk_status yk_box_potential_adaptive(yk_ctx ctx, const double *root, int64_t n_leaves, const int32_t *level,
                                    const int32_t *ix, const int32_t *iy, const double *vals, double alpha,
                                    double *V);

/*
 * Sec. 3.1's refinement test: a leaf is refined where the cubic fitted to its
 * 16 cell values misses the values at the 64 cell centres of its four children
 * by more than tol.  v16 [n][16] and v64 [n][4][16] device (child q = qy 2 +
 * qx, its cell t as above); flags [n] device out (1: refine); err [n] device
 * out (optional): the largest miss.
 */
yk_status yk_box_refine(yk_ctx ctx, int64_t n_leaves, const double *v16, const double *v64, double tol,
                        int32_t *flags, double *err);

/*
 * One step of (1 - alpha^2 Lap) u = B, u = f_next on the curves (eq.
 * mod_helm_forced) on adaptive leaves (Sec. 3.1 with the box code): the
 * volume points are the cells of the leaves of yk_box_potential_adaptive
 * (root, level, ix, iy as there), B and u_next [n_leaves][16] device in its
 * cell order.  U^p = V / alpha^2 of the leaves' cubic fits at the cells, on
 * the nodes the leaf polynomials fitted to those values (every node inside a
 * leaf); then as yk_heat_step_grid: sigma from A sigma = -2 alpha^2 (f_next -
 * U^p), u_next = U^p + DL[w sigma] / alpha^2 with the near-boundary
 * evaluation (off with flags bit2).  flags bit1: zero initial guess.
 */
yk_status yk_heat_step_leaves(yk_ctx ctx, const yk_boundary *bnd, const double *root, int64_t n_leaves,
                              const int32_t *level, const int32_t *ix, const int32_t *iy, const double *B,
                              int flags, const double *f_next, double alpha2, double tol, double *sigma_io,
                              double *u_next, yk_stats *stats);

/*
 * Introspection: number of volume points the last step evaluated with the
 * near-boundary rule, and the time (ms) that set took to build.
 */
yk_status yk_near_info(yk_ctx ctx, int64_t *n_near, double *setup_ms);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of yk_gmres_density with direct O(N^2) sums (as with options.direct = 1),
 * with the same arguments, results and status codes, that allocates
 * nothing.  Its device workspace is a fixed array of 4,194,304 doubles
 * (32 MiB) that the library holds on each GPU it runs on until the process
 * ends; it takes (gmres_m + 9) N doubles plus about 108,000 for N nodes
 * (gmres_m 60: up to about 60,000 nodes), and larger sizes are rejected with
 * YK_ERR_ARG before any work.  The caller passes the context (its stream and
 * gmres_m are used), the boundary, g, sigma0 and sigma as for
 * yk_gmres_density.  No pinned memory or event is created: the Arnoldi
 * scalars come back by ordinary copies, so the host waits for each
 * iteration.  Every call on one GPU shares that GPU's array (whatever the
 * context), so calls that overlap on one GPU race; the array keeps the last
 * call's contents, and the solve initialises everything it reads.
 */
yk_status yk_gmres_density_noalloc(yk_ctx ctx, const yk_boundary *bnd, double alpha, const double *g,
                                   const double *sigma0, double tol, int max_iter, double *sigma,
                                   yk_stats *stats);

/*
 * Right-hand side of the backward-Euler step with the constant extension of
 * Sec. 3.1 (boundary data constant on each curve):
 *   B_i = u_i + dt F_i       if region[i] < 0 (inside the domain)
 *   B_i = c[region[i]]       otherwise (0 = outside the outer curve, k = inside hole k)
 * u, F [n] device FP64 (F may be NULL = 0); region [n] device int32;
 * c [n_const] HOST FP64.
 */
yk_status yk_rhs_backward_euler(yk_ctx ctx, int64_t n, const double *u, const double *F,
                                const int32_t *region, int n_const, const double *c,
                                double dt, double *B);

/*
 * Right-hand side B of the linearly implicit (IMEX) schemes of Sec. 2 (eq.
 * mod_helm_forced) for u_t - nu Lap u = F + R(u):
 *   YK_SCHEME_EULER (backward Euler):  alpha^2 = nu dt,
 *       B = ub + dt f
 *   YK_SCHEME_GEAR (extrapolated Gear, eq. exg):  alpha^2 = 2 nu dt / 3,
 *       B = 4/3 ub - 1/3 ub' + dt (4/3 f - 2/3 f')
 * with f = F + R(ub), ub = u where region[i] < 0 (inside the domain) and
 * ub = c[region[i]] elsewhere (the constant extension of Sec. 3.1; 0 when
 * region[i] >= n_const), primes marking step N - 1.  F applies at every point
 * (pass zeros outside the domain for the zero extension of F); the reaction
 * R is 0 (YK_REACTION_NONE) or u (1 - u^2) (YK_REACTION_ALLEN_CAHN, Sec. 4,
 * Example 3), evaluated on ub.  The step itself is yk_heat_step or
 * yk_heat_step_grid with the scheme's alpha^2.
 * u, u_prev, F, F_prev, B [n] device FP64 (F, F_prev may be NULL = 0; u_prev
 * is needed for Gear only); region [n] device int32; c [n_const] HOST FP64.
 */
enum { YK_SCHEME_EULER = 0, YK_SCHEME_GEAR = 1 };
enum { YK_REACTION_NONE = 0, YK_REACTION_ALLEN_CAHN = 1 };
yk_status yk_rhs_imex(yk_ctx ctx, int scheme, int reaction, int64_t n, const double *u, const double *u_prev,
                      const double *F, const double *F_prev, const int32_t *region, int n_const,
                      const double *c, double dt, double *B);

/*
 * One full FMM evaluation with charges on the volume points and dipoles on the
 * nodes, every point a target (the throughput benchmark's pass):
 *   out_vol[i] = V[q](x_i) + DL[d](x_i),   out_bnd[j] = V[q](y_j) + DL[d](y_j)
 * with d_j the dipole strength at node j (normal from bnd), self pairs and
 * coincident pairs skipped, no diagonal term.
 */
yk_status yk_fmm_potential(yk_ctx ctx, int64_t n_vol, const double *vol_xy, const double *q,
                           const yk_boundary *bnd, const double *d, double alpha,
                           double *out_vol, double *out_bnd);

/*
 * Learned warm start for the density solve (an addition to the method: it
 * only seeds GMRES).  A per-node network (features: sigma^N,
 * sigma^N - sigma^{N-1}, g^{N+1} - g^N, g^N - g^{N-1} and kappa at 13 offsets
 * along the curve) predicts the correction of sigma^{N+1} to the linear
 * extrapolation 2 sigma^N - sigma^{N-1}.  It is trained on the GPU, with the
 * library's own FP32 matrix-core forward/backward kernels and Adam, on the
 * densities the solver produced.  Attached to a context (yk_set_warm_start),
 * yk_heat_step evaluates ||b - A sigma|| for the learned guess and for the
 * previous-step density and starts GMRES from the smaller one (stats
 * guess_used = 2 when the learned guess wins); every step still stops at the
 * same tolerance.  Attached, yk_heat_step also records each solved step
 * (yk_ws_observe).  All arrays are device FP64 of the boundary's N nodes.
 */
typedef struct yk_ws_s *yk_ws;
typedef struct {
    int hidden;            /* width of the two hidden layers */
    int batch;             /* rows (nodes x steps) per Adam step */
    int steps;             /* Adam steps per yk_ws_train call */
    double lr;             /* Adam learning rate */
    int max_obs;           /* observed steps kept (training triples = max_obs - 2) */
    uint64_t seed;         /* weight initialisation and shuffling */
} yk_ws_options;

/* Defaults: hidden 256, batch 32768, steps 600, lr 1e-3, max_obs 64, seed 1. */
void yk_ws_default_options(yk_ws_options *opt);
/* The boundary must stay the same (same arrays) for the life of the network. */
yk_status yk_ws_create(yk_ctx ctx, const yk_boundary *bnd, const yk_ws_options *opt, yk_ws *out);
yk_status yk_ws_destroy(yk_ws ws);
/* Records one solved step: g [N] = f^{N+1} - U^p on the nodes, sigma [N] = sigma^{N+1}. */
yk_status yk_ws_observe(yk_ws ws, const double *g, const double *sigma);
/* Trains on every (N-1, N, N+1) triple recorded; *loss = last mini-batch MSE
 * in units of the target's RMS (may be NULL). */
yk_status yk_ws_train(yk_ws ws, double *loss);
/* sigma_out [N] = the network's prediction of sigma^{N+1} from the last two
 * recorded steps and g_next [N]. */
yk_status yk_ws_predict(yk_ws ws, const double *g_next, double *sigma_out);
/* Attaches (ws != NULL) or detaches the warm start used by yk_heat_step.
 * yk_heat_step returns YK_ERR_ARG when the attached warm start was created
 * for another boundary (other node array, curvature array or offsets). */
yk_status yk_set_warm_start(yk_ctx ctx, yk_ws ws);
/* Parameter access and one loss/gradient evaluation, for checking the
 * training kernels: params/grad are DEVICE FP32 arrays of yk_ws_num_params
 * entries (W1 [H][Fp], b1 [H], W2 [H][H], b2 [H], w3 [H], b3), X [rows][Fp]
 * device FP32 features, t [rows] device FP32 targets. */
int64_t yk_ws_num_params(yk_ws ws, int *hidden, int *fp);
yk_status yk_ws_get_params(yk_ws ws, float *params);
yk_status yk_ws_set_params(yk_ws ws, const float *params);
yk_status yk_ws_loss_grad(yk_ws ws, int64_t rows, const float *X, const float *t, float *grad,
                          double *loss);
/* y [rows] device FP32 = the network's outputs for the feature rows X
 * [rows][Fp] by the inference path yk_heat_step uses (the fused kernel, or
 * layer by layer with debug_flags bit 5). */
yk_status yk_ws_forward(yk_ws ws, int64_t rows, const float *X, float *y);
/* One Adam step (Kingma & Ba: decays 0.9 and 0.999, eps 1e-8, the options'
 * learning rate, bias corrections from the network's own step count, which
 * yk_ws_train advances too) of the parameters on grad [n_params] (device FP32). */
yk_status yk_ws_adam_step(yk_ws ws, const float *grad);

/*
 * Introspection for measurement (not part of the method).
 * yk_plan_info: shape of the tree cached in `slot` (0 = volume points and
 * nodes, as used by the heat step and yk_fmm_potential; 1 = nodes only, as
 * used by the density solve; 2 = the stand-alone sum calls; 3 = the finer
 * boundary rule and the check points of the near-boundary evaluation; 4 = the
 * nodes and the near-boundary targets) and the work of its last evaluation:
 * near-field pairs and M2L translations.
 * yk_timing_enable: when on, every FMM stage is bracketed by HIP events on
 * the stream it runs on (the near field, YK_STAGE_LEAF, runs on a second
 * stream of the context concurrently with the far-field stages, unless
 * debug_flags bit 1 is set; its time then includes the sharing of the GPU); yk_timing_read returns the accumulated milliseconds
 * and launch counts per stage (YK_STAGE_*), resolving the events, and resets
 * the counters when `reset` is non-zero.  Reading synchronises the stream.
 */
typedef struct {
    int32_t valid;            /* 0 when no tree is cached in the slot */
    int32_t leaf_level, lmin, p, P, Pp;
    int64_t n_points, n_boxes, n_leaves;
    int64_t pairs_charge;     /* near-field (target, charge) pairs of the last evaluation */
    int64_t pairs_dipole;     /* near-field (target, dipole) pairs of the last evaluation */
    int64_t m2l_translations; /* non-empty V-list entries of the last evaluation */
    int64_t m2l_slots;        /* V-list slots processed (27 per active box, incl. empty;
                                 the translations themselves when m2l_sparse) */
    int64_t p2m_points, l2p_points;
    int32_t near_terms;       /* series length of the near-field K0/K1 evaluation */
    int32_t nser;             /* series length of the F_n starting values */
    double build_ms;          /* host wall time of the last tree build */
    int32_t m2l_sparse;       /* 1: M2L of the last evaluation ran over the non-empty
                                 translations bucketed by (level, offset), as chosen
                                 for small trees with mostly empty V lists */
    int32_t near_sym;         /* 1: the cached charge-to-charge values are stored once
                                 per pair of neighbouring leaves (K0 is symmetric) */
    int64_t near_charge_values; /* charge values the cached near field reads per
                                   evaluation (pairs_charge unless near_sym; not
                                   counting the zeros that pad rows to vectors) */
    int64_t near_incoming;    /* entries written to (and read back from) the incoming
                                 slots of the symmetric near field per evaluation */
    int32_t p_initial;        /* order first derived from fmm_tol (= p when given) */
    double order_check_err;   /* build-time order check: the largest error of the
                                 sampled probe outputs at the order kept, relative to
                                 each output (floored at a tenth of the samples' RMS);
                                 -1 when no check ran (order given, or no far field).
                                 When fmm_tol derives the order, the tree raises it
                                 along 8, 12, 16, 20, 24, 31 until this error is at
                                 most fmm_tol / 2, or the order reaches 31 */
    int64_t m2m_children;     /* child-to-parent translations of the upward pass
                                 (non-empty children of the boxes at levels lmin..L-1) */
    int64_t l2l_children;     /* parent-to-child translations of the downward pass of
                                 the last evaluation (its active boxes at levels > lmin) */
    int64_t n_ulist;          /* U-list entries of the leaves (yk_plan_tree_export) */
    double tables_ms;         /* host time spent on the translation operator tables
                                 (each order tried by the order check) */
    double order_check_ms;    /* time of the build-time order check (within build_ms) */
    int32_t tree;             /* YK_TREE_UNIFORM or YK_TREE_ADAPTIVE: the cached tree's form */
    int32_t max_u;            /* adaptive tree: the longest U list (at most 13) */
    int64_t n_wlist;          /* adaptive tree: W-list entries (= X-list entries) */
    int64_t n_xboxes;         /* adaptive tree: boxes with a non-empty X list */
} yk_plan_info;

enum {
    YK_STAGE_GATHER = 0, YK_STAGE_P2M = 1, YK_STAGE_M2M = 2, YK_STAGE_M2L = 3,
    YK_STAGE_L2L = 4, YK_STAGE_LEAF = 5, YK_STAGE_SCATTER = 6, YK_STAGE_DIRECT = 7,
    YK_STAGE_L2P = 8, YK_STAGE_NEAR_BUILD = 9, YK_NUM_STAGES = 10
};

yk_status yk_plan_info_get(yk_ctx ctx, int slot, yk_plan_info *info);
/*
 * The tree cached in `slot`, for checking its construction (Sec. 3.1's
 * quad-tree, built from Morton keys).  Every pointer may be NULL (skipped);
 * sizes come from yk_plan_info_get.
 *   square       HOST [3]: x0, y0, side of the bounding square; a point's
 *                level-15 cell is floor((x - x0) 2^15 / side), clamped to
 *                [0, 2^15), and its key is (set << 30) | Morton(cell)
 *   level_begin  HOST [leaf_level + 2]: first box index of each level, then n_boxes
 *   keys         DEVICE [n_points] sorted keys (sets 0 charges, 1 nodes, 2 targets)
 *   perm         DEVICE [n_points] index of each sorted point within its set
 *   box_code     DEVICE [n_boxes] Morton code of each box at its level
 *   parent       DEVICE [n_boxes] parent box (-1 at level 0)
 *   leaf_range   DEVICE [n_leaves][6] first and one-past-last sorted position
 *                of each set in each leaf (0, 0 when empty)
 *   ulist_off    DEVICE [n_leaves + 1], ulist DEVICE [n_ulist]: leaf-local
 *                indices of the non-empty leaves of each leaf's 3 x 3 block,
 *                row by row
 *   vlist        DEVICE [n_boxes][27]: the V list in the slot order of the
 *                box's parity class (dy outer, dx inner over the 6 x 6 block
 *                of the parent's neighbours' children minus the 3 x 3 block),
 *                -1 where absent and at levels below max(lmin, 2)
 */
yk_status yk_plan_tree_export(yk_ctx ctx, int slot, double *square, int64_t *level_begin, uint32_t *keys,
                              int32_t *perm, uint32_t *box_code, int32_t *parent, int32_t *leaf_range,
                              int32_t *ulist_off, int32_t *ulist, int32_t *vlist);
/*
 * The adaptive parts of the tree cached in `slot` (options.tree ==
 * YK_TREE_ADAPTIVE; YK_ERR_ARG otherwise).  Leaves lie at any level and are
 * numbered in Morton order of their first level-15 cell; leaf_range, ulist_off
 * and ulist of yk_plan_tree_export then use that numbering, and the U lists
 * hold the touching leaves (the leaf itself included) in increasing index.
 * Every pointer may be NULL (skipped):
 *   leaf_box     DEVICE [n_leaves] box index of each leaf
 *   box_level    DEVICE [n_boxes] level of each box
 *   wlist_off    DEVICE [n_leaves + 1], wlist DEVICE [n_wlist]: per leaf, the
 *                boxes of levels >= lmin, finer than the leaf, whose parent
 *                touches it and which do not (increasing box index)
 *   xbox         DEVICE [n_xboxes] the boxes with a non-empty X list
 *   xlist_off    DEVICE [n_xboxes + 1], xlist DEVICE [n_wlist]: per such box,
 *                the leaves whose W list holds it (increasing leaf index)
 */
yk_status yk_plan_adaptive_export(yk_ctx ctx, int slot, int32_t *leaf_box, int32_t *box_level,
                                  int32_t *wlist_off, int32_t *wlist, int32_t *xbox, int32_t *xlist_off,
                                  int32_t *xlist);
yk_status yk_timing_enable(yk_ctx ctx, int enable);
yk_status yk_timing_read(yk_ctx ctx, double ms[YK_NUM_STAGES], int64_t calls[YK_NUM_STAGES],
                         int reset);

#ifdef __cplusplus
}
#endif

#endif /* YK_H */
