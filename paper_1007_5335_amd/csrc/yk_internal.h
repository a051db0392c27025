// yk_internal.h -- shared declarations of libyk's host layer and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "yk.h"

namespace yk {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv2Pi = 1.0 / (2.0 * kPi);
constexpr double kZeta3 = 1.2020569031595942854;   // Apery's constant

// The diagonal entry w_j D(y_j, y_j) / (2 pi) of the on-curve double layer.
// The kernel's limit along the curve is -kappa / 2 (Sec. 2); its only
// non-smooth part is -(kappa |y'|^2 / (4 alpha^2)) t^2 log|t| (t the parameter
// offset, from the (z^2/2) log z term of z K1(z)), whose trapezoid-rule error
// -2 zeta'(-2) h^3 g(0) (generalised Euler-Maclaurin expansion, with
// zeta'(-2) = -zeta(3) / (4 pi^2)) is added back at the node: the rule becomes
// fifth order.  w = |y'| h is the node's weight, inv_a2 = 1 / alpha^2.
__host__ __device__ inline double dl_diag_weight(double w, double kappa, double inv_a2) {
    return w * kappa * (-0.5 + (kZeta3 / (8.0 * kPi * kPi)) * w * w * inv_a2) * kInv2Pi;
}

// Internal error: thrown inside the library, converted to a status at the ABI.
struct Error {
    yk_status code;
    std::string msg;
};

#define YK_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::yk::Error{YK_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define YK_REQUIRE(cond, msg)                                      \
    do {                                                           \
        if (!(cond)) throw ::yk::Error{YK_ERR_ARG, std::string(msg)}; \
    } while (0)

// Device buffer owned by the library (grow-only), or a borrowed window of
// fixed size into memory the library does not allocate here (the
// allocation-free entry point's array): a borrowed buffer never allocates or
// frees, and asking it for more than its window is an internal error.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    bool borrowed = false;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void borrow(T *ptr, size_t count) {
        release();
        p = ptr;
        n = count;
        borrowed = true;
    }
    void release() {
        if (p && !borrowed) (void)hipFree(p);
        p = nullptr;
        n = 0;
        borrowed = false;
    }
    T *ensure(size_t count) {
        if (count <= n && p) return p;
        if (borrowed)
            throw Error{YK_ERR_INTERNAL, "a fixed workspace window of " + std::to_string(n) +
                                             " entries was asked for " + std::to_string(count)};
        release();
        size_t c = count ? count : 1;
        if (hipMalloc(&p, c * sizeof(T)) != hipSuccess) {
            p = nullptr;
            throw Error{YK_ERR_NOMEM, "device allocation of " + std::to_string(c * sizeof(T)) + " bytes failed"};
        }
        n = c;
        return p;
    }
};

struct Context;
struct WarmStart;

// Launch-time check (and optional synchronous check in debug mode).
void check_launch(Context &ctx, const char *what);

// Boundary geometry prepared once per boundary (weights, curve ids).
struct BoundaryData {
    uint64_t gen = 0;                 // distinct for every preparation
    const double *xy = nullptr;
    int64_t n = 0;
    int n_curves = 0;
    std::vector<int64_t> offset;      // host copy
    DevBuf<double> w;                 // (2 pi / N_k) speed_j
    DevBuf<int32_t> curve;            // curve id per node
    DevBuf<int32_t> idx;              // node index within its curve
    const double *normal = nullptr;
    const double *curvature = nullptr;
    const double *speed = nullptr;
};

// Near-boundary evaluation of the double layer (near.hip): the targets
// closer to a curve than a few node spacings, their projections, check
// points and the finer trapezoid rule used there.
struct NearPlan;
struct NearPlanDeleter {
    void operator()(NearPlan *p) const;
};
using NearPtr = std::unique_ptr<NearPlan, NearPlanDeleter>;

// (node, cell) pairs of the cell-integral correction of U^p at the nodes (cells.hip)
struct CellNodePlan;
struct CellNodePlanDeleter {
    void operator()(CellNodePlan *p) const;
};
using CellNodePtr = std::unique_ptr<CellNodePlan, CellNodePlanDeleter>;

// Box code on a uniform grid (box.hip): leaves of 4 x 4 cells, their cubic
// fits, the near-field and expansion tables, and the tree over the leaves
struct BoxPlan;
struct BoxPlanDeleter {
    void operator()(BoxPlan *p) const;
};
using BoxPtr = std::unique_ptr<BoxPlan, BoxPlanDeleter>;

struct FmmPlan;   // tree + lists + operator tables (fmm.hip)
void destroy_plan(FmmPlan *p);
struct PlanDeleter {
    void operator()(FmmPlan *p) const { destroy_plan(p); }
};
using PlanPtr = std::unique_ptr<FmmPlan, PlanDeleter>;

// A captured application of the density operator for one boundary tree
// (plan generation), alpha and precision, with its own input, output and
// work buffers (the graph holds their addresses).
struct BieGraph {
    uint64_t plan_gen = 0;
    double alpha = 0;
    int prec = 0;
    int runs = 0;            // eager applications so far (capture after the first)
    bool failed = false;     // capture or instantiation failed: stay eager
    hipGraphExec_t exec = nullptr;
    DevBuf<double> x, y, dn, dl;
    ~BieGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

struct Context {
    yk_options opt{};
    hipStream_t stream = nullptr;
    std::string last_error;
    int device = 0;

    std::unique_ptr<BoundaryData> bnd;     // cached boundary preparation
    PlanPtr plan_vol;                      // tree over volume points and nodes
    PlanPtr plan_bnd;                      // tree over the nodes only (solver)
    PlanPtr plan_misc;                     // tree for the stand-alone sum calls
    PlanPtr plan_near;                     // fine nodes -> near-boundary check points
    PlanPtr plan_nearc;                    // nodes -> near targets (coarse rule, subtracted)
    NearPtr near;                          // near-boundary targets of the last volume set
    CellNodePtr cell_nodes;                // cells next to the nodes (heat step, flags bit0)
    BoxPtr box;                            // box code of the last grid and alpha

    // own-cell weights of yk_heat_step's cell centres (flags bit0): the
    // distinct cell areas of vol_w, an index per point, the weights for alpha
    const double *self_w = nullptr;
    int64_t self_n = 0;
    std::vector<double> self_h2;
    DevBuf<uint16_t> self_idx;
    DevBuf<double> self_dh2, self_w0;
    double self_alpha = 0.0;

    // cell-centred grid of yk_heat_step_grid (coordinates generated here)
    DevBuf<double> grid_xy, grid_up, grid_w0;
    double grid_w0_key[2] = {0, 0};         // (h^2, alpha) of grid_w0
    double grid_key[3] = {0, 0, 0};
    int64_t grid_nx = 0, grid_ny = 0;
    uint64_t grid_bnd_gen = 0;             // boundary whose nodes were checked against the grid

    // workspaces
    DevBuf<double> ws_a, ws_b, ws_c, ws_d, ws_e, ws_f;
    DevBuf<double> krylov;                 // (m+1) x N
    DevBuf<double> gm_w, gm_r;             // GMRES-private vectors
    DevBuf<double> partial;                // reduction partials
    DevBuf<double> scal;                   // small device scalars
    DevBuf<double> arn_partial;            // Arnoldi passes: block partials
    double *gm_host = nullptr;             // pinned host copy of an Arnoldi column (hipHostMalloc)
    // allocation-free mode: every device buffer is borrowed, no event or
    // pinned memory is created, and host copies go through host_scal
    bool noalloc = false;
    DevBuf<double> dn;                     // dipole vectors [N][2]
    DevBuf<double> direct_part;            // direct sums split over source chunks: [chunk][target]
    std::vector<double> host_scal;

    struct WarmStart *warm = nullptr;       // attached learned warm start (not owned)

    // last solution of the FP64 density operator and its image A sigma, so the
    // next heat step gets the residual of the previous-step density for free
    DevBuf<double> memo_sig, memo_Asig, memo_r1, memo_r2;
    DevBuf<int> memo_flag;
    bool memo_valid = false;
    const double *memo_xy = nullptr;
    int64_t memo_n = 0;
    double memo_alpha = 0, memo_tol = 0;
    int memo_p = 0, memo_leaf = 0, memo_direct = 0;
    DevBuf<double> ws_g, ws_ml, ws_t;       // heat-step buffers of the guess selection
    DevBuf<double> ws_q;                    // heat step: volume charges W B (no solver touches it)

    // second stream for the near field (overlaps the far-field chain) and the
    // fork/join events that order it against the context's stream
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_col = nullptr;            // GMRES: an Arnoldi column is on the host

    // graph replays of the density operator (see BieGraph in capi.cpp)
    bool capturing = false;                 // a stream capture is in progress
    hipStream_t cap_stream = nullptr;
    std::vector<std::unique_ptr<BieGraph>> bie_graphs;

    // optional per-stage event timing
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> event_pool;
    double stage_ms[YK_NUM_STAGES] = {0};
    int64_t stage_calls[YK_NUM_STAGES] = {0};
    ~Context();
};

// Brackets a stage with events when timing is on (RAII).
struct StageTimer {
    Context &ctx;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(Context &c, int s, hipStream_t on = nullptr);
    ~StageTimer();
};
void resolve_timings(Context &ctx);
// creates the side stream and its events on first use
void ensure_side_stream(Context &ctx);

// ---------------------------------------------------------------- kernels ---
// Direct sums (FP64): out[i] (+)= sum_j q_j K0/(2pi) + sum_j (x_i - y_j).dn_j K1(z)/(alpha^2 z)/(2pi)
void launch_direct(Context &ctx, int64_t nt, const double *txy, int64_t ns, const double *sxy,
                   const double *q, int64_t nb, const double *bxy, const double *dn, double alpha,
                   double *out, bool accumulate);
// dn_j = scale * w_j * sigma_j * n_j  (w == nullptr: unit weights)
void launch_dipole_vectors(Context &ctx, int64_t n, const double *w, const double *sigma,
                           const double *normal, double scale, double *dn);
// out_j += dl_diag_weight(w_j, kappa_j, 1 / alpha^2) sigma_j
void launch_dl_diagonal(Context &ctx, int64_t n, const double *w, const double *kappa, double alpha,
                        const double *sigma, double *out);
// y = x - 2 * dl  (dl already includes 1/(2pi) and the diagonal)
void launch_bie_combine(Context &ctx, int64_t n, const double *x, const double *dl, double *y);
void launch_mul(Context &ctx, int64_t n, const double *a, const double *b, double *out);
// y = x - 2 (dl + dl_diag_weight(w, kappa, 1 / alpha^2) x)  (diagonal + combination)
void launch_bie_finish(Context &ctx, int64_t n, const double *w, const double *kappa, double alpha,
                       const double *x, const double *dl, double *y);
// out = ca * a + cb * b  (b may be null -> out = ca * a)
void launch_axpby(Context &ctx, int64_t n, double ca, const double *a, double cb, const double *b,
                  double *out);
// own-cell weights w0[d] of grid points with squared cell side h2[d] (the
// weight that makes the lattice rule exact for constant B), and
// out = scale * (out + B * w0[idx[i]])  (idx NULL: w0[0] for every point)
void launch_self_weights(Context &ctx, int nd, const double *h2, double alpha, double *w0);
void launch_self_cell(Context &ctx, int64_t n, const uint16_t *idx, const double *w0, const double *B, double scale,
                      double *out_accum);
void launch_rhs_be(Context &ctx, int64_t n, const double *u, const double *F, const int32_t *region,
                   int n_const, const double *c_dev, double dt, double *B);
// B of the Euler (gear false) or extrapolated Gear scheme, optional Allen-Cahn
// reaction; up/Fp are step N - 1 (Gear only); c_dev [n_const] on the device
void launch_rhs_imex(Context &ctx, int64_t n, bool gear, bool allen_cahn, const double *u, const double *up,
                     const double *F, const double *Fp, const int32_t *region, int n_const, const double *c_dev,
                     double dt, double *B);
void launch_boundary_prep(Context &ctx, int64_t n, int n_curves, const int64_t *off_dev,
                          const double *speed, double *w, int32_t *curve, int32_t *idx);

// BLAS for GMRES (deterministic reductions)
// h[k] = sum_i V[k*ld + i] * x[i], k < nv  (result on device at h)
void launch_multi_dot(Context &ctx, int64_t n, int nv, const double *V, int64_t ld,
                      const double *x, double *h);
// h[v] = |x_v|^2 for v = 0, 1, 2 (a null vector gives 0), in one reduction
void launch_sumsq3(Context &ctx, int64_t n, const double *x0, const double *x1, const double *x2, double *h);
// x -= sum_k h[k] V[k*ld + i]
// Arnoldi step in passes (see kernels_blas.hip): w -= sum_{v<nsub} h_v V_v with
// h summed from the partials psub of the previous pass (stored to hsub_out),
// then partials of V_r . w (r < nd) and, with self, of w . w into pout
void launch_arnoldi_pass(Context &ctx, int64_t n, const double *V, int64_t ld, double *w, int nsub,
                         const double *psub, double *hsub_out, int nd, bool self, double *pout);
// CGS2's second subtraction and normalisation from the previous pass's
// partials p (h2 = V^T w in rows 0..nsub-1, |w|^2 in row nsub): y = (w - V h2)
// / sqrt(|w|^2 - |h2|^2); stores h2 and the squared norm; host_dst (pinned, may
// be null) receives h1[0..128), h2 at 128.. and the squared norm at 256
void launch_arnoldi_finish(Context &ctx, int64_t n, const double *V, int64_t ld, const double *w, int nsub,
                           const double *p, double *h2_out, double *nrm2_out, double *y, const double *h1,
                           double *host_dst);
// partial buffer 0, 1 or 2 of the Arnoldi passes
double *arnoldi_partials(Context &ctx, int which);
void launch_multi_axpy(Context &ctx, int64_t n, int nv, const double *V, int64_t ld,
                       const double *h, double *x);
// y = x / *s  (s on device)
void launch_scale_div(Context &ctx, int64_t n, const double *x, const double *s, double *y);
// x += sum_k y[k] V[k*ld+i] with y on device
void launch_add_combination(Context &ctx, int64_t n, int nv, const double *V, int64_t ld,
                            const double *y, double *x);
// flag = any non-finite in x  (writes 0/1 to *flag as double)
void launch_nonfinite(Context &ctx, int64_t n, const double *x, double *flag);

// ------------------------------------------------------------------ GMRES ---
using Apply = std::function<void(const double *x, double *y)>;
struct GmresResult {
    int iters = 0;
    int matvecs = 0;
    double res0 = 0, res_final = 0;   // relative to ||b||
    bool converged = false;
};
// Solves A x = b; x holds the initial guess on entry (zero if zero_guess).
// r0, when given (and zero_guess is false), is b - A x for that guess, which
// saves the first operator application.  r0_norm2 / b_norm2, when >= 0, are
// |r0|^2 and |b|^2 already known to the caller (each saves a synchronising
// reduction).  On return ctx.gm_r holds the true residual b - A x of the
// returned x, unless b was zero.
GmresResult gmres(Context &ctx, const Apply &A, int64_t n, const double *b, double *x,
                  bool zero_guess, double tol, int max_iter, int m, const double *r0 = nullptr,
                  double r0_norm2 = -1.0, double b_norm2 = -1.0);
// pinned host memory of the context (512 doubles: [0, 257) the Arnoldi
// column, [400, 416) the heat step's scalars)
double *pinned_scalars(Context &ctx);
// out[i] = v for i < n
void launch_fill(Context &ctx, int64_t n, double v, double *out);
// flag = 1 if a and b differ anywhere (bitwise), on the context's stream
void launch_differs(Context &ctx, int64_t n, const double *a, const double *b, int *flag);

// takes the device address of the allocation-free entry point's array on this
// device (once per device; noalloc.hip)
void noalloc_init_device(int device);

// -------------------------------------------------------------------- FMM ---
// Evaluate V[q] + DL[dn] at targets with the cached plan.
struct FmmRequest;
BoundaryData &prepare_boundary(Context &ctx, const yk_boundary *b);

// cell centres of a grid, point j nx + i at (x0 + (i + 1/2) h, y0 + (j + 1/2) h)
void launch_grid_points(Context &ctx, int64_t n, double x0, double y0, double h, int64_t nx, double *xy);
// out_j = tensor cubic Lagrange interpolation of the cell-centre values V at xy_j
void launch_bicubic(Context &ctx, int64_t n, const double *xy, double x0, double y0, double h, int64_t nx,
                    int64_t ny, const double *V, double *out);
// box.hip: the box-code volume potential V (K0/(2 pi) normalisation, U^p =
// V / alpha^2) at the cells of a grid whose sides are multiples of 4 cells, and
// the leaf polynomials of cell values evaluated at points inside the grid
void box_potential(Context &ctx, const yk_grid &g, const double *B, double alpha, double *V);
void box_leaf_eval(Context &ctx, const yk_grid &g, const double *vals, int64_t n, const double *xy, double *out);
// the box code on adaptive leaves (level, ix, iy host arrays; vals, V [n][16] device)
void box_potential_adaptive(Context &ctx, const double root[3], int64_t n, const int32_t *lev, const int32_t *ix,
                            const int32_t *iy, const double *vals, double alpha, double *V);
// the adaptive box plan's cell centres [n_leaves * 16][2] (device)
const double *box_cells(Context &ctx);
// the leaf polynomials fitted to vals [n_leaves][16] at n points xy (device),
// the points' leaves cached for (xy, n, gen)
void box_leaves_eval(Context &ctx, const double *vals, int64_t n, const double *xy, uint64_t gen, double *out);
// Sec. 3.1's refinement test of n leaves (device arrays)
void box_refine(Context &ctx, int64_t n, const double *v16, const double *v64, double tol, int32_t *flags,
                double *err);

// near-boundary evaluation (near.hip): the near targets of tgt_xy for the
// boundary (built once per boundary and target array), and one step's
// correction: out[i] = (base ? base[i] : out[i] - coarse DL_i / alpha^2) + U^h_i
NearPlan &near_prepare(Context &ctx, BoundaryData &bd, int64_t n_tgt, const double *tgt_xy);
void near_apply(Context &ctx, NearPlan &np, BoundaryData &bd, double alpha, const double *sigma, const double *g,
                const double *base, double *out);
int64_t near_count(const NearPlan &np);
double near_setup_ms(const NearPlan &np);

// cell-centre volume points (cells.hip): the cells within two sides of each
// node (built once per points, weights and boundary), and
// vb[i] += sum_j B_j (cell integral - point value) for those cells
CellNodePlan &cells_prepare(Context &ctx, BoundaryData &bd, int64_t n, const double *vol_xy, const double *vol_w);
void cells_correct_nodes(Context &ctx, CellNodePlan &cp, BoundaryData &bd, const double *vol_xy, const double *vol_w,
                         const double *B, double alpha, double *vb);
int64_t cells_pair_count(const CellNodePlan &cp);

}  // namespace yk

struct yk_ctx_s {
    yk::Context c;
};
