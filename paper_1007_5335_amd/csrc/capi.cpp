// capi.cpp -- the C ABI of libyk: argument checks, status codes, and the
// drivers of the solve and of the heat step (Kropinski & Quaife, Sec. 2-3).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <new>
#include <unordered_map>

#include "fmm.h"
#include "mlp.h"
#include "sums.h"
#include "yk_internal.h"

namespace yk {

void check_launch(Context &ctx, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{YK_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)};
    if (ctx.opt.debug_flags & 1) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) throw Error{YK_ERR_HIP, std::string(what) + " (sync): " + hipGetErrorString(e)};
    }
}

Context::~Context() {
    for (auto &pe : pending) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    bie_graphs.clear();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_col) (void)hipEventDestroy(ev_col);
    if (side) (void)hipStreamDestroy(side);
    if (gm_host) (void)hipHostFree(gm_host);
}

void ensure_side_stream(Context &ctx) {
    if (ctx.side) return;
    YK_HIP(hipStreamCreateWithFlags(&ctx.side, hipStreamNonBlocking));
    YK_HIP(hipEventCreateWithFlags(&ctx.ev_fork, hipEventDisableTiming));
    YK_HIP(hipEventCreateWithFlags(&ctx.ev_join, hipEventDisableTiming));
}

static hipEvent_t take_event(Context &ctx) {
    if (!ctx.event_pool.empty()) {
        hipEvent_t e = ctx.event_pool.back();
        ctx.event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    YK_HIP(hipEventCreate(&e));
    return e;
}

StageTimer::StageTimer(Context &c, int s, hipStream_t on) : ctx(c), stage(s), st(on ? on : c.stream) {
    if (!ctx.timing || ctx.capturing) return;
    a = take_event(ctx);
    b = take_event(ctx);
    YK_HIP(hipEventRecord(a, st));
}

StageTimer::~StageTimer() {
    if (!a) return;
    if (hipEventRecord(b, st) == hipSuccess)
        ctx.pending.push_back({stage, {a, b}});
}

void resolve_timings(Context &ctx) {
    if (ctx.pending.empty()) return;
    YK_HIP(hipStreamSynchronize(ctx.stream));
    if (ctx.side) YK_HIP(hipStreamSynchronize(ctx.side));
    for (auto &pe : ctx.pending) {
        float ms = 0.f;
        YK_HIP(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
        ctx.stage_ms[pe.first] += ms;
        ctx.stage_calls[pe.first] += 1;
        ctx.event_pool.push_back(pe.second.first);
        ctx.event_pool.push_back(pe.second.second);
    }
    ctx.pending.clear();
}

BoundaryData &prepare_boundary(Context &ctx, const yk_boundary *b) {
    YK_REQUIRE(b != nullptr, "boundary is NULL");
    YK_REQUIRE(b->n_curves >= 1, "boundary needs at least one curve");
    YK_REQUIRE(b->offset != nullptr, "boundary offsets are NULL");
    YK_REQUIRE(b->xy && b->normal && b->speed && b->curvature, "a boundary array is NULL");
    YK_REQUIRE(b->offset[0] == 0, "boundary offset[0] must be 0");
    for (int k = 0; k < b->n_curves; ++k)
        YK_REQUIRE(b->offset[k + 1] > b->offset[k], "boundary offsets must increase strictly");
    const int64_t n = b->offset[b->n_curves];
    YK_REQUIRE(n < (int64_t)1 << 31, "too many boundary nodes");
    BoundaryData *cur = ctx.bnd.get();
    bool same = cur && cur->xy == b->xy && cur->n == n && cur->n_curves == b->n_curves &&
                cur->speed == b->speed && cur->normal == b->normal && cur->curvature == b->curvature;
    if (same)
        for (int k = 0; k <= b->n_curves; ++k) same = same && cur->offset[k] == b->offset[k];
    if (same) return *cur;
    static std::atomic<uint64_t> bnd_gen{0};
    auto nb = std::make_unique<BoundaryData>();
    nb->gen = ++bnd_gen;
    nb->xy = b->xy;
    nb->n = n;
    nb->n_curves = b->n_curves;
    nb->offset.assign(b->offset, b->offset + b->n_curves + 1);
    nb->normal = b->normal;
    nb->curvature = b->curvature;
    nb->speed = b->speed;
    DevBuf<int64_t> off;
    int64_t *doff = off.ensure(b->n_curves + 1);
    YK_HIP(hipMemcpyAsync(doff, nb->offset.data(), (b->n_curves + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, ctx.stream));
    launch_boundary_prep(ctx, n, b->n_curves, doff, b->speed, nb->w.ensure(n), nb->curve.ensure(n),
                         nb->idx.ensure(n));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    ctx.bnd = std::move(nb);
    // trees that contain the nodes are stale, and so is the near-boundary set
    ctx.plan_vol.reset();
    ctx.plan_bnd.reset();
    ctx.plan_near.reset();
    ctx.plan_nearc.reset();
    ctx.near.reset();
    return *ctx.bnd;
}

void evaluate_sums(Context &ctx, PlanSlot slot, const SumProblem &pb, const double *q,
                   const double *dn, double *const out[3], SumPrec prec) {
    if (!ctx.opt.direct) {
        fmm_evaluate(ctx, slot, pb, q, dn, out, prec);
        return;
    }
    if (pb.bie) {   // direct backend: the fused steps as separate kernels
        double *dnb = ctx.dn.ensure(2 * pb.n[1]);
        launch_dipole_vectors(ctx, pb.n[1], pb.bie->w, pb.bie->sigma, pb.bie->normal, 1.0, dnb);
        SumProblem plain = pb;
        plain.bie = nullptr;
        evaluate_sums(ctx, slot, plain, q, dnb, out, prec);
        if (out[1] && pb.bie->kappa)
            launch_bie_finish(ctx, pb.n[1], pb.bie->w, pb.bie->kappa, pb.alpha, pb.bie->sigma, out[1], out[1]);
        return;
    }
    StageTimer st(ctx, YK_STAGE_DIRECT);
    for (int s = 0; s < 3; ++s) {
        if (!out[s] || pb.n[s] == 0) continue;
        launch_direct(ctx, pb.n[s], pb.xy[s], q ? pb.n[0] : 0, pb.xy[0], q, dn ? pb.n[1] : 0,
                      pb.xy[1], dn, pb.alpha, out[s], false);
    }
}

namespace {

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void check_alpha(double a) { YK_REQUIRE(std::isfinite(a) && a > 0.0, "alpha must be finite and > 0"); }

// Operator of eq. discrete_sys (trapezoid rule): y = x - 2 (DL[w x] + diagonal).
struct BieOperator {
    Context &ctx;
    BoundaryData &bd;
    double alpha;
    SumPrec prec;
    // (dn, dl: workspaces of the unfused form, unused now that the dipole
    // vectors and the final combination are formed inside the sum)
    void apply_eager(const double *x, double *y, double *dn, double *dl) const {
        (void)dn;
        (void)dl;
        SumProblem pb;
        pb.n[1] = bd.n;
        pb.xy[1] = bd.xy;
        pb.normal = bd.normal;
        pb.alpha = alpha;
        BieFuse f;
        f.w = bd.w.p;
        f.sigma = x;
        f.normal = bd.normal;
        f.kappa = bd.curvature;
        pb.bie = &f;
        double *const outs[3] = {nullptr, y, nullptr};
        evaluate_sums(ctx, SLOT_BND, pb, nullptr, nullptr, outs, prec);
    }
    // With debug_flags bit 2 the operator, applied many times per solve with
    // the same tree, is captured once (after one eager application) into a
    // HIP graph, kernels and the near-field stream fork included, and
    // replayed: one launch instead of ~20.  Input and output go through the
    // graph's own buffers.  Measured on MI355X with ROCm 7 the replay was
    // slower than eager launches for the 28,672-node boundary tree, so it is
    // off by default.  Debug synchronisation, direct sums or a failed capture
    // keep it eager.
    BieGraph *graph_for_plan() const {
        if (ctx.opt.direct || (ctx.opt.debug_flags & 1) || !(ctx.opt.debug_flags & 4)) return nullptr;
        SumProblem pb;
        pb.n[1] = bd.n;
        pb.xy[1] = bd.xy;
        pb.normal = bd.normal;
        pb.alpha = alpha;
        FmmPlan &pl = get_plan(ctx, SLOT_BND, pb);
        for (auto &g : ctx.bie_graphs)
            if (g->plan_gen == pl.gen && g->alpha == alpha && g->prec == (int)prec) return g.get();
        // entries of other trees are stale
        ctx.bie_graphs.erase(std::remove_if(ctx.bie_graphs.begin(), ctx.bie_graphs.end(),
                                            [&](const std::unique_ptr<BieGraph> &g) { return g->plan_gen != pl.gen; }),
                             ctx.bie_graphs.end());
        auto g = std::make_unique<BieGraph>();
        g->plan_gen = pl.gen;
        g->alpha = alpha;
        g->prec = (int)prec;
        ctx.bie_graphs.push_back(std::move(g));
        return ctx.bie_graphs.back().get();
    }
    void capture(BieGraph &g) const {
        const int64_t n = bd.n;
        g.x.ensure(n);
        g.y.ensure(n);
        g.dn.ensure(2 * n);
        g.dl.ensure(n);
        YK_HIP(hipMemsetAsync(g.x.p, 0, n * sizeof(double), ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
        if (!ctx.cap_stream) YK_HIP(hipStreamCreateWithFlags(&ctx.cap_stream, hipStreamNonBlocking));
        hipStream_t saved = ctx.stream;
        ctx.stream = ctx.cap_stream;
        ctx.capturing = true;
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(ctx.stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            try {
                apply_eager(g.x.p, g.y.p, g.dn.p, g.dl.p);
            } catch (...) {
                ok = false;
            }
            const hipError_t e = hipStreamEndCapture(ctx.stream, &graph);
            ok = ok && e == hipSuccess && graph != nullptr;
        }
        ctx.stream = saved;
        ctx.capturing = false;
        if (ok) ok = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        if (!ok) {
            g.failed = true;
            g.exec = nullptr;
            (void)hipGetLastError();
        }
    }
    void operator()(const double *x, double *y) const {
        const int64_t n = bd.n;
        BieGraph *g = graph_for_plan();
        if (g && !g->failed && !g->exec && g->runs >= 1) capture(*g);
        if (g && g->exec) {
            YK_HIP(hipMemcpyAsync(g->x.p, x, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
            YK_HIP(hipGraphLaunch(g->exec, ctx.stream));
            YK_HIP(hipMemcpyAsync(y, g->y.p, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
            return;
        }
        if (g) g->runs++;
        apply_eager(x, y, ctx.dn.ensure(2 * n), ctx.ws_a.ensure(n));
    }
};

// Solves A sigma = b in FP64, or (mixed) by refinement: FP64 residuals with an
// FP32-operator GMRES for each correction.
// r0: b - A sigma for the incoming sigma (optional); Asig_out (optional): set
// to A sigma of the returned density when the solve converged (FP64 operator);
// r0_norm2, b_norm2: |r0|^2 and |b|^2 when already known (else negative)
GmresResult solve_density(Context &ctx, BoundaryData &bd, double alpha, const double *b,
                          double *sigma, bool zero_guess, double tol, int max_iter, int *outer,
                          const double *r0 = nullptr, double *Asig_out = nullptr,
                          bool *asig_ok = nullptr, double r0_norm2 = -1.0, double b_norm2 = -1.0) {
    if (asig_ok) *asig_ok = false;
    const int64_t n = bd.n;
    BieOperator A64{ctx, bd, alpha, SUM_FP64};
    *outer = 0;
    if (ctx.opt.precision == YK_PREC_FP64 || ctx.opt.direct) {
        GmresResult g = gmres(ctx, A64, n, b, sigma, zero_guess, tol, max_iter, ctx.opt.gmres_m, r0, r0_norm2,
                              b_norm2);
        if (Asig_out && g.converged && g.res_final > 0) {   // A sigma = b - r
            launch_axpby(ctx, n, 1.0, b, -1.0, ctx.gm_r.p, Asig_out);
            if (asig_ok) *asig_ok = true;
        }
        return g;
    }
    BieOperator A32{ctx, bd, alpha, SUM_FP32};
    double *r = ctx.ws_b.ensure(n);
    double *delta = ctx.ws_c.ensure(n);
    double *tmp = ctx.ws_d.ensure(n);
    double *dscal = ctx.scal.ensure(512);
    auto norm = [&](const double *v) {
        launch_multi_dot(ctx, n, 1, v, n, v, dscal + 400);
        double h = 0;
        YK_HIP(hipMemcpyAsync(&h, dscal + 400, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
        return std::sqrt(h);
    };
    GmresResult tot;
    const double bnorm = b_norm2 >= 0.0 ? std::sqrt(b_norm2) : norm(b);
    if (zero_guess) YK_HIP(hipMemsetAsync(sigma, 0, n * sizeof(double), ctx.stream));
    for (int sweep = 0; sweep < 30; ++sweep) {
        if (sweep == 0 && r0 && !zero_guess) {
            YK_HIP(hipMemcpyAsync(r, r0, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
            launch_axpby(ctx, n, 1.0, b, -1.0, r0, tmp);   // A sigma, kept for the memo
        } else {
            A64(sigma, tmp);
            tot.matvecs++;
            launch_axpby(ctx, n, 1.0, b, -1.0, tmp, r);
        }
        const double rn = (sweep == 0 && r0 && !zero_guess && r0_norm2 >= 0.0) ? std::sqrt(r0_norm2) : norm(r);
        if (!std::isfinite(rn)) throw Error{YK_ERR_NONFINITE, "refinement residual is not finite"};
        if (sweep == 0) tot.res0 = bnorm > 0 ? rn / bnorm : 0.0;
        tot.res_final = bnorm > 0 ? rn / bnorm : 0.0;
        if (rn <= tol * bnorm || bnorm == 0.0) {
            tot.converged = true;
            if (Asig_out && bnorm > 0.0) {
                YK_HIP(hipMemcpyAsync(Asig_out, tmp, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
                if (asig_ok) *asig_ok = true;
            }
            break;
        }
        if (tot.iters >= max_iter) break;
        // inner FP32-operator solve: to the reduction that would finish the
        // solve in this sweep (with a factor 2 to spare), but not below what
        // an FP32 operator resolves (about 1e-6 relative, so a residual far
        // above tol takes further sweeps)
        const double inner_tol = std::min(0.5, std::max(1e-6, 0.5 * tol * bnorm / rn));
        // (|r|^2 is known on the host: no second reduction and wait)
        GmresResult in = gmres(ctx, A32, n, r, delta, true, inner_tol, max_iter - tot.iters, ctx.opt.gmres_m,
                               nullptr, -1.0, rn * rn);
        tot.iters += in.iters;
        tot.matvecs += in.matvecs;
        launch_axpby(ctx, n, 1.0, sigma, 1.0, delta, sigma);
        (*outer)++;
    }
    return tot;
}

// The memo of the last FP64 density solve was made for this operator?
bool memo_key_matches(Context &ctx, BoundaryData &bd, double alpha) {
    const yk_options &o = ctx.opt;
    return ctx.memo_valid && ctx.memo_xy == bd.xy && ctx.memo_n == bd.n && ctx.memo_alpha == alpha &&
           ctx.memo_tol == o.fmm_tol && ctx.memo_p == o.p && ctx.memo_leaf == o.leaf_size &&
           ctx.memo_direct == o.direct;
}

// Enqueues the check that sigma is bitwise the memo's density; the returned
// device flag is 0 when it is (read it after a synchronisation)
int *memo_check(Context &ctx, BoundaryData &bd, const double *sigma) {
    int *flag = ctx.memo_flag.ensure(1);
    const int zero = 0;
    YK_HIP(hipMemcpyAsync(flag, &zero, sizeof(int), hipMemcpyHostToDevice, ctx.stream));
    launch_differs(ctx, bd.n, sigma, ctx.memo_sig.p, flag);
    return flag;
}

void memo_store(Context &ctx, BoundaryData &bd, double alpha, const double *sigma) {
    const yk_options &o = ctx.opt;
    YK_HIP(hipMemcpyAsync(ctx.memo_sig.ensure(bd.n), sigma, bd.n * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx.stream));
    ctx.memo_valid = true;
    ctx.memo_xy = bd.xy;
    ctx.memo_n = bd.n;
    ctx.memo_alpha = alpha;
    ctx.memo_tol = o.fmm_tol;
    ctx.memo_p = o.p;
    ctx.memo_leaf = o.leaf_size;
    ctx.memo_direct = o.direct;
}

}  // namespace

GmresResult solve_density_direct(Context &ctx, BoundaryData &bd, double alpha, const double *b, double *sigma,
                                 bool zero_guess, double tol, int max_iter) {
    int outer = 0;
    return solve_density(ctx, bd, alpha, b, sigma, zero_guess, tol, max_iter, &outer);
}

}  // namespace yk

using namespace yk;

template <typename F>
static yk_status guarded(yk_ctx ctx, F &&f) {
    if (!ctx) return YK_ERR_ARG;
    try {
        yk_status s = f(ctx->c);
        if (s == YK_OK) ctx->c.last_error.clear();
        return s;
    } catch (const Error &e) {
        ctx->c.last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->c.last_error = "host allocation failed";
        return YK_ERR_NOMEM;
    } catch (const std::exception &e) {
        ctx->c.last_error = e.what();
        return YK_ERR_INTERNAL;
    } catch (...) {
        ctx->c.last_error = "unknown internal error";
        return YK_ERR_INTERNAL;
    }
}

extern "C" {

void yk_default_options(yk_options *opt) {
    if (!opt) return;
    opt->precision = YK_PREC_FP64;
    opt->fmm_tol = 1e-10;
    opt->p = 0;
    opt->leaf_size = 64;
    opt->direct = 0;
    opt->gmres_m = 60;
    opt->debug_flags = 0;
    opt->near_cache_mb = 16384;
    opt->tree = YK_TREE_AUTO;
}

static bool valid_options(const yk_options *o) {
    return o->precision >= 0 && o->precision <= 2 && o->p >= 0 && o->p <= 31 &&
           o->leaf_size >= 1 && o->leaf_size <= 4096 && o->gmres_m >= 1 && o->gmres_m <= 120 &&
           o->near_cache_mb >= 0 && o->tree >= YK_TREE_UNIFORM && o->tree <= YK_TREE_AUTO &&
           (o->p > 0 || (o->fmm_tol > 0 && o->fmm_tol < 1));
}

// why the last yk_create on this thread failed (no context holds it)
static thread_local std::string g_create_error;

yk_status yk_create(const yk_options *opt, yk_ctx *out) {
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return YK_ERR_ARG;
    }
    *out = nullptr;
    yk_options o;
    yk_default_options(&o);
    if (opt) o = *opt;
    if (!valid_options(&o)) {
        g_create_error = "invalid options";
        return YK_ERR_ARG;
    }
    yk_ctx c = new (std::nothrow) yk_ctx_s();
    if (!c) {
        g_create_error = "host allocation failed";
        return YK_ERR_NOMEM;
    }
    c->c.opt = o;
    const hipError_t e = hipGetDevice(&c->c.device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
        delete c;
        return YK_ERR_HIP;
    }
    try {   // the allocation-free entry point's array on this device
        noalloc_init_device(c->c.device);
    } catch (const Error &err) {
        g_create_error = err.msg;
        delete c;
        return err.code;
    } catch (...) {
        g_create_error = "unknown error taking the workspace array's address";
        delete c;
        return YK_ERR_INTERNAL;
    }
    *out = c;
    return YK_OK;
}

yk_status yk_destroy(yk_ctx ctx) {
    if (!ctx) return YK_ERR_ARG;
    (void)hipStreamSynchronize(ctx->c.stream);
    delete ctx;
    return YK_OK;
}

yk_status yk_set_stream(yk_ctx ctx, void *stream) {
    if (!ctx) return YK_ERR_ARG;
    ctx->c.stream = (hipStream_t)stream;
    return YK_OK;
}

yk_status yk_set_options(yk_ctx ctx, const yk_options *opt) {
    if (!ctx || !opt || !valid_options(opt)) return YK_ERR_ARG;
    const yk_options old = ctx->c.opt;
    ctx->c.opt = *opt;
    ctx->c.memo_valid = false;
    if (old.p != opt->p || old.leaf_size != opt->leaf_size || old.fmm_tol != opt->fmm_tol ||
        old.tree != opt->tree) {
        ctx->c.plan_vol.reset();
        ctx->c.plan_bnd.reset();
        ctx->c.plan_misc.reset();
        ctx->c.plan_near.reset();
        ctx->c.plan_nearc.reset();
    }
    return YK_OK;
}

const char *yk_last_error(yk_ctx ctx) {
    if (!ctx) return g_create_error.empty() ? "null context" : g_create_error.c_str();
    return ctx->c.last_error.c_str();
}

yk_status yk_invalidate_geometry(yk_ctx ctx) {
    return guarded(ctx, [&](Context &c) {
        YK_HIP(hipStreamSynchronize(c.stream));
        c.plan_vol.reset();
        c.plan_bnd.reset();
        c.plan_misc.reset();
        c.plan_near.reset();
        c.plan_nearc.reset();
        c.near.reset();
        c.cell_nodes.reset();
        c.box.reset();
        c.grid_nx = c.grid_ny = 0;
        c.grid_bnd_gen = 0;
        c.self_w = nullptr;
        c.self_n = 0;
        c.bnd.reset();
        c.memo_valid = false;
        return YK_OK;
    });
}

yk_status yk_volume_potential(yk_ctx ctx, int64_t n_src, const double *src_xy, const double *q,
                              int64_t n_tgt, const double *tgt_xy, double alpha, double *out) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(n_src > 0 && src_xy && q && out, "invalid source arguments");
        YK_REQUIRE(!tgt_xy || n_tgt > 0, "n_tgt must be > 0 when targets are given");
        check_alpha(alpha);
        SumProblem pb;
        pb.n[0] = n_src;
        pb.xy[0] = src_xy;
        pb.alpha = alpha;
        double *outs[3] = {nullptr, nullptr, nullptr};
        if (tgt_xy) {
            pb.n[2] = n_tgt;
            pb.xy[2] = tgt_xy;
            outs[2] = out;
        } else {
            outs[0] = out;
        }
        evaluate_sums(c, SLOT_MISC, pb, q, nullptr, outs, SUM_FP64);
        return YK_OK;
    });
}

yk_status yk_double_layer_apply(yk_ctx ctx, const yk_boundary *bnd, const double *sigma,
                                int64_t n_tgt, const double *tgt_xy, double alpha, double *out) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(sigma && out, "sigma/out are NULL");
        YK_REQUIRE(!tgt_xy || n_tgt > 0, "n_tgt must be > 0 when targets are given");
        check_alpha(alpha);
        BoundaryData &bd = prepare_boundary(c, bnd);
        double *dn = c.dn.ensure(2 * bd.n);
        launch_dipole_vectors(c, bd.n, bd.w.p, sigma, bd.normal, 1.0, dn);
        SumProblem pb;
        pb.n[1] = bd.n;
        pb.xy[1] = bd.xy;
        pb.normal = bd.normal;
        pb.alpha = alpha;
        double *outs[3] = {nullptr, nullptr, nullptr};
        if (tgt_xy) {
            pb.n[2] = n_tgt;
            pb.xy[2] = tgt_xy;
            outs[2] = out;
            evaluate_sums(c, SLOT_MISC, pb, nullptr, dn, outs, SUM_FP64);
        } else {
            outs[1] = out;
            evaluate_sums(c, SLOT_BND, pb, nullptr, dn, outs, SUM_FP64);
            launch_dl_diagonal(c, bd.n, bd.w.p, bd.curvature, alpha, sigma, out);
        }
        return YK_OK;
    });
}

static void fill_stats(yk_stats *st, const GmresResult &r, int outer, int guess) {
    if (!st) return;
    st->iters = r.iters;
    st->outer_iters = outer;
    st->guess_used = guess;
    st->matvecs = r.matvecs;
    st->res0 = r.res0;
    st->res_final = r.res_final;
}

yk_status yk_gmres_density(yk_ctx ctx, const yk_boundary *bnd, double alpha, const double *g,
                           const double *sigma0, double tol, int max_iter, double *sigma,
                           yk_stats *stats) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(g && sigma, "g/sigma are NULL");
        YK_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
        YK_REQUIRE(max_iter >= 1, "max_iter must be >= 1");
        check_alpha(alpha);
        if (stats) std::memset(stats, 0, sizeof(*stats));
        BoundaryData &bd = prepare_boundary(c, bnd);
        const int64_t n = bd.n;
        double *b = c.ws_f.ensure(n);
        launch_axpby(c, n, -2.0 * alpha * alpha, g, 0.0, nullptr, b);
        if (sigma0 && sigma0 != sigma)
            YK_HIP(hipMemcpyAsync(sigma, sigma0, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
        auto t0 = std::chrono::steady_clock::now();
        int outer = 0;
        GmresResult r = solve_density(c, bd, alpha, b, sigma, sigma0 == nullptr, tol, max_iter, &outer);
        YK_HIP(hipStreamSynchronize(c.stream));
        fill_stats(stats, r, outer, sigma0 ? 1 : 0);
        if (stats) stats->ms[2] = ms_since(t0);
        if (!r.converged) {
            c.last_error = "GMRES did not reach the tolerance within max_iter";
            return YK_ERR_NOCONV;
        }
        return YK_OK;
    });
}

// Own-cell weights of cell centres whose areas are vol_w (yk_heat_step flags
// bit0): the distinct areas are found once per array (key: pointer and
// size), an index per point is kept on the device, and the weights are
// recomputed when alpha changes.
static const double *self_weights(Context &c, int64_t n, const double *vol_w, double alpha,
                                  const uint16_t **idx_out) {
    if (c.self_w != vol_w || c.self_n != n) {
        std::vector<double> hw((size_t)n);
        YK_HIP(hipMemcpyAsync(hw.data(), vol_w, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        YK_HIP(hipStreamSynchronize(c.stream));
        std::unordered_map<uint64_t, int> seen;
        std::vector<double> distinct;
        for (int64_t i = 0; i < n; ++i) {
            uint64_t bits;
            std::memcpy(&bits, &hw[i], sizeof(bits));
            if (seen.emplace(bits, (int)distinct.size()).second) {
                YK_REQUIRE(std::isfinite(hw[i]) && hw[i] > 0.0, "vol_w must be finite and > 0");
                YK_REQUIRE(distinct.size() < 65535, "cell centres (flags bit0) need at most 65535 distinct cell areas");
                distinct.push_back(hw[i]);
            }
        }
        std::sort(distinct.begin(), distinct.end());
        std::unordered_map<uint64_t, uint16_t> rank;
        for (size_t k = 0; k < distinct.size(); ++k) {
            uint64_t bits;
            std::memcpy(&bits, &distinct[k], sizeof(bits));
            rank[bits] = (uint16_t)k;
        }
        std::vector<uint16_t> hidx((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            uint64_t bits;
            std::memcpy(&bits, &hw[i], sizeof(bits));
            hidx[i] = rank[bits];
        }
        YK_HIP(hipMemcpyAsync(c.self_idx.ensure(n), hidx.data(), n * sizeof(uint16_t), hipMemcpyHostToDevice,
                              c.stream));
        YK_HIP(hipMemcpyAsync(c.self_dh2.ensure(distinct.size()), distinct.data(), distinct.size() * sizeof(double),
                              hipMemcpyHostToDevice, c.stream));
        YK_HIP(hipStreamSynchronize(c.stream));
        c.self_h2 = distinct;
        c.self_w = vol_w;
        c.self_n = n;
        c.self_alpha = 0.0;
    }
    if (c.self_alpha != alpha) {
        launch_self_weights(c, (int)c.self_h2.size(), c.self_dh2.p, alpha, c.self_w0.ensure(c.self_h2.size()));
        c.self_alpha = alpha;
    }
    *idx_out = c.self_idx.p;
    return c.self_w0.p;
}

// The attached warm start must have been made for this boundary: its
// feature kernels read and write N-node arrays with its own offsets.
static void check_warm(Context &c, const BoundaryData &bd) {
    if (!c.warm) return;
    const WarmStart &ws = *c.warm;
    YK_REQUIRE(ws.n == bd.n && ws.offsets == bd.offset && ws.kappa == bd.curvature && ws.xy == bd.xy,
               "the attached warm start was created for another boundary");
}

// The density of one step: the initial guess (the caller's density, whose
// residual may come from the kept image A sigma, or the learned prediction
// when its residual is smaller), GMRES to tol, and the bookkeeping of the kept
// image and the warm start.  b = -2 alpha^2 g and gN = g on the nodes.
static GmresResult step_density(Context &c, BoundaryData &bd, double alpha, const double *b, const double *gN,
                                int flags, double tol, double *sigma_io, yk_stats *stats, int &outer, int &guess) {
    const int64_t nb = bd.n;
    // initial guess: the caller's (previous-step) density, or the learned
    // prediction when its residual is smaller.  When the caller's density
    // is the last solution of this same operator, its image A sigma is
    // still held and its residual costs no operator application.
    guess = (flags & 2) ? 0 : 1;
    const double *r0 = nullptr;
    double r0_norm2 = -1.0;
    double *rprev = c.memo_r1.ensure(nb), *rml = c.memo_r2.ensure(nb);
    BieOperator A64{c, bd, alpha, SUM_FP64};
    // Everything the choice needs is enqueued first and read back with one
    // synchronisation: ds = {|r_ml|^2, |r_prev|^2, |b|^2} and the memo flag.
    const bool memo_key = guess == 1 && memo_key_matches(c, bd, alpha);
    const bool learned = guess == 1 && c.warm && c.warm->trained && c.warm->obs.size() >= 2;
    double *ds = c.scal.ensure(512) + 450;
    double *sml = learned ? c.ws_ml.ensure(nb) : nullptr;
    auto tg = std::chrono::steady_clock::now();
    int *dflag = memo_key ? memo_check(c, bd, sigma_io) : nullptr;
    auto resid_enqueue = [&](const double *x, double *rv, bool from_memo, double *d) {
        if (from_memo) {
            launch_axpby(c, nb, 1.0, b, -1.0, c.memo_Asig.p, rv);
        } else {
            A64(x, rv);
            launch_axpby(c, nb, 1.0, b, -1.0, rv, rv);
        }
        if (d) launch_multi_dot(c, nb, 1, rv, nb, rv, d);
    };
    if (learned) {
        c.warm->predict(gN, sml);
        resid_enqueue(sml, rml, false, nullptr);
    }
    // the previous density's residual: from the memo when it applies (a
    // changed density is caught below), else by an operator application
    // when the learned guess needs it for comparison
    if (memo_key) resid_enqueue(sigma_io, rprev, true, nullptr);
    else if (learned) resid_enqueue(sigma_io, rprev, false, nullptr);
    // the three squared norms in one reduction
    launch_sumsq3(c, nb, learned ? rml : nullptr, (memo_key || learned) ? rprev : nullptr, b, ds);
    double *hsc = pinned_scalars(c) + 400;
    YK_HIP(hipMemcpyAsync(hsc, ds, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    if (dflag) YK_HIP(hipMemcpyAsync(hsc + 3, dflag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    YK_HIP(hipStreamSynchronize(c.stream));
    double r_ml = hsc[0], r_prev = hsc[1];
    const double b_norm2 = hsc[2];
    int hflag = 0;
    if (dflag) std::memcpy(&hflag, hsc + 3, sizeof(int));
    const bool memo = memo_key && hflag == 0;
    if (memo_key && !memo && learned) {   // the caller changed sigma since the memo
        resid_enqueue(sigma_io, rprev, false, ds + 1);
        YK_HIP(hipMemcpyAsync(hsc + 1, ds + 1, sizeof(double), hipMemcpyDeviceToHost, c.stream));
        YK_HIP(hipStreamSynchronize(c.stream));
        r_prev = hsc[1];
    }
    if (learned) {
        if (std::isfinite(r_ml) && r_ml < r_prev) {
            YK_HIP(hipMemcpyAsync(sigma_io, sml, nb * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
            guess = 2;
            r0 = rml;
            r0_norm2 = r_ml;
        } else {
            r0 = rprev;
            r0_norm2 = r_prev;
        }
        if (stats) stats->ms[4] = ms_since(tg);
    } else if (memo) {
        r0 = rprev;
        r0_norm2 = r_prev;
    }
    // sigma
    auto t1 = std::chrono::steady_clock::now();
    outer = 0;
    bool asig_ok = false;
    GmresResult r = solve_density(c, bd, alpha, b, sigma_io, guess == 0, tol, 1000, &outer, r0,
                                  c.memo_Asig.ensure(nb), &asig_ok, r0_norm2, b_norm2);
    if (asig_ok) memo_store(c, bd, alpha, sigma_io);
    else c.memo_valid = false;
    if (c.warm) c.warm->observe(gN, sigma_io);
    if (stats) stats->ms[2] = ms_since(t1);
    return r;
}

yk_status yk_heat_step(yk_ctx ctx, const yk_boundary *bnd, int64_t n_vol, const double *vol_xy,
                       const double *vol_w, const double *B, int flags, const double *f_next,
                       double dt, double tol, double *sigma_io, double *u_next, yk_stats *stats) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(n_vol > 0 && vol_xy && vol_w && B && f_next && sigma_io && u_next,
                   "invalid heat-step arguments");
        YK_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be finite and > 0");
        YK_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
        if (stats) std::memset(stats, 0, sizeof(*stats));
        BoundaryData &bd = prepare_boundary(c, bnd);
        const int64_t nb = bd.n;
        const double alpha = std::sqrt(dt), a2 = dt;
        const SumPrec vprec = c.opt.precision == YK_PREC_FP32 ? SUM_FP32 : SUM_FP64;
        check_warm(c, bd);
        // q = W B, in a buffer of its own (the density solve below takes the
        // shared workspaces and may reallocate them)
        double *q = c.ws_q.ensure(n_vol);
        auto t0 = std::chrono::steady_clock::now();
        launch_mul(c, n_vol, vol_w, B, q);
        SumProblem pb;
        pb.n[0] = n_vol;
        pb.xy[0] = vol_xy;
        pb.n[1] = nb;
        pb.xy[1] = bd.xy;
        pb.normal = bd.normal;
        pb.alpha = alpha;
        // U^p on the nodes: b = -2 alpha^2 (f - V[q]/alpha^2) = -2 alpha^2 f + 2 V[q]
        double *vb = c.ws_e.ensure(nb);
        {
            double *outs[3] = {nullptr, vb, nullptr};
            SumProblem pk = pb;
            pk.keep_charge_m = (c.opt.debug_flags & 8) ? 0 : 1;   // the assembly below has the same charges
            evaluate_sums(c, SLOT_VOL, pk, q, nullptr, outs, vprec);
        }
        // cell centres: the cells next to a node enter with their integral
        if (flags & 1) {
            CellNodePlan &cp = cells_prepare(c, bd, n_vol, vol_xy, vol_w);
            cells_correct_nodes(c, cp, bd, vol_xy, vol_w, B, alpha, vb);
        }
        double *b = c.ws_f.ensure(nb);
        launch_axpby(c, nb, -2.0 * a2, f_next, 2.0, vb, b);
        if (stats) {   // (phase times need a synchronisation)
            YK_HIP(hipStreamSynchronize(c.stream));
            stats->ms[0] = fmm_last_build_ms(c);
            stats->ms[1] = ms_since(t0);
        }
        // g = f - U^p on the nodes (recorded for the learned warm start)
        double *gN = c.ws_g.ensure(nb);
        launch_axpby(c, nb, 1.0, f_next, -1.0 / a2, vb, gN);
        int outer = 0, guess = 0;
        GmresResult r = step_density(c, bd, alpha, b, gN, flags, tol, sigma_io, stats, outer, guess);
        // u = (V[q] + DL[w sigma] + B C_self) / alpha^2 at the volume points
        auto t2 = std::chrono::steady_clock::now();
        {
            double *outs[3] = {u_next, nullptr, nullptr};
            SumProblem pr = pb;
            pr.keep_charge_m = (c.opt.debug_flags & 8) ? 0 : 2;   // the same charges q as the first pass
            BieFuse f;   // dipole vectors w sigma n, formed in the gather
            f.w = bd.w.p;
            f.sigma = sigma_io;
            f.normal = bd.normal;
            pr.bie = &f;
            evaluate_sums(c, SLOT_VOL, pr, q, nullptr, outs, vprec);
        }
        if (flags & 1) {
            const uint16_t *sidx = nullptr;
            const double *w0 = self_weights(c, n_vol, vol_w, alpha, &sidx);
            launch_self_cell(c, n_vol, sidx, w0, B, 1.0 / a2, u_next);
        }
        else launch_axpby(c, n_vol, 1.0 / a2, u_next, 0.0, nullptr, u_next);
        // targets closer to a curve than a few node spacings: U^h from the
        // curves' interpolants instead of the node sums
        if (!(flags & 4)) {
            NearPlan &np = near_prepare(c, bd, n_vol, vol_xy);
            near_apply(c, np, bd, alpha, sigma_io, gN, nullptr, u_next);
        }
        YK_HIP(hipStreamSynchronize(c.stream));
        if (stats) stats->ms[3] = ms_since(t2);
        fill_stats(stats, r, outer, guess);
        if (!r.converged) {
            c.last_error = "GMRES did not reach the tolerance";
            return YK_ERR_NOCONV;
        }
        return YK_OK;
    });
}

namespace {

// Cell centres of the grid in the context's buffer (regenerated, with the
// trees and near-boundary sets that contain them, when the grid changes)
const double *grid_points(Context &c, const yk_grid &g) {
    const int64_t n = g.nx * g.ny;
    if (c.grid_nx == g.nx && c.grid_ny == g.ny && c.grid_key[0] == g.x0 && c.grid_key[1] == g.y0 &&
        c.grid_key[2] == g.h && c.grid_xy.p)
        return c.grid_xy.p;
    c.plan_vol.reset();
    c.plan_near.reset();
    c.plan_nearc.reset();
    c.near.reset();
    c.grid_bnd_gen = 0;
    double *xy = c.grid_xy.ensure(2 * n);
    launch_grid_points(c, n, g.x0, g.y0, g.h, g.nx, xy);
    c.grid_key[0] = g.x0;
    c.grid_key[1] = g.y0;
    c.grid_key[2] = g.h;
    c.grid_nx = g.nx;
    c.grid_ny = g.ny;
    return xy;
}

// every node's 4 x 4 interpolation stencil lies inside the grid
void grid_check_nodes(Context &c, const BoundaryData &bd, const yk_grid &g) {
    if (c.grid_bnd_gen == bd.gen) return;
    std::vector<double> hxy(2 * bd.n);
    YK_HIP(hipMemcpyAsync(hxy.data(), bd.xy, 2 * bd.n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    YK_HIP(hipStreamSynchronize(c.stream));
    for (int64_t j = 0; j < bd.n; ++j) {
        const double sx = (hxy[2 * j] - g.x0) / g.h - 0.5, sy = (hxy[2 * j + 1] - g.y0) / g.h - 0.5;
        YK_REQUIRE(std::isfinite(sx) && std::isfinite(sy) && std::floor(sx) >= 1.0 &&
                       std::floor(sx) + 2.0 <= (double)(g.nx - 1) && std::floor(sy) >= 1.0 &&
                       std::floor(sy) + 2.0 <= (double)(g.ny - 1),
                   "a boundary node's interpolation stencil leaves the grid (keep two cells between the "
                   "curves and the grid's edge)");
    }
    c.grid_bnd_gen = bd.gen;
}

}  // namespace

yk_status yk_heat_step_grid(yk_ctx ctx, const yk_boundary *bnd, const yk_grid *grid, const double *B, int flags,
                            const double *f_next, double alpha2, double tol, double *sigma_io, double *u_next,
                            yk_stats *stats) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(grid && B && f_next && sigma_io && u_next, "invalid grid-step arguments");
        YK_REQUIRE(std::isfinite(grid->x0) && std::isfinite(grid->y0) && std::isfinite(grid->h) && grid->h > 0.0,
                   "invalid grid origin or cell size");
        YK_REQUIRE(grid->nx >= 4 && grid->ny >= 4 && grid->nx <= ((int64_t)1 << 20) &&
                       grid->ny <= ((int64_t)1 << 20) && grid->nx * grid->ny < ((int64_t)1 << 31),
                   "grid sides must be 4 .. 2^20 cells and the grid below 2^31 cells");
        YK_REQUIRE(std::isfinite(alpha2) && alpha2 > 0.0, "alpha2 must be finite and > 0");
        YK_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
        if (stats) std::memset(stats, 0, sizeof(*stats));
        BoundaryData &bd = prepare_boundary(c, bnd);
        check_warm(c, bd);
        const int64_t n = grid->nx * grid->ny, nb = bd.n;
        const double h = grid->h, a2 = alpha2, alpha = std::sqrt(alpha2);
        const SumPrec vprec = c.opt.precision == YK_PREC_FP32 ? SUM_FP32 : SUM_FP64;
        const double *gxy = grid_points(c, *grid);
        grid_check_nodes(c, bd, *grid);
        auto t0 = std::chrono::steady_clock::now();
        SumProblem pb;
        pb.n[0] = n;
        pb.xy[0] = gxy;
        pb.n[1] = nb;
        pb.xy[1] = bd.xy;
        pb.normal = bd.normal;
        pb.alpha = alpha;
        double *up = c.grid_up.ensure(n);
        double *vb = c.ws_e.ensure(nb);
        if (flags & 8) {
            // box code: U^p = V[cubic leaf fits of B] / alpha^2 at the cells,
            // and on the nodes the leaf polynomials fitted to those values
            box_potential(c, *grid, B, alpha, up);
            launch_axpby(c, n, 1.0 / a2, up, 0.0, nullptr, up);
            box_leaf_eval(c, *grid, up, nb, bd.xy, vb);
        } else {
            // U^p = (V[h^2 B] + B (C_cell + kappa h^2)) / alpha^2 at the cell centres
            double *q = c.ws_q.ensure(n);
            launch_axpby(c, n, h * h, B, 0.0, nullptr, q);
            {
                double *outs[3] = {up, nullptr, nullptr};
                evaluate_sums(c, SLOT_VOL, pb, q, nullptr, outs, vprec);
            }
            if (c.grid_w0_key[0] != h * h || c.grid_w0_key[1] != alpha || !c.grid_w0.p) {
                double *dh2 = c.grid_w0.ensure(2);
                const double hh = h * h;
                YK_HIP(hipMemcpyAsync(dh2 + 1, &hh, sizeof(double), hipMemcpyHostToDevice, c.stream));
                launch_self_weights(c, 1, dh2 + 1, alpha, dh2);
                YK_HIP(hipStreamSynchronize(c.stream));
                c.grid_w0_key[0] = hh;
                c.grid_w0_key[1] = alpha;
            }
            launch_self_cell(c, n, nullptr, c.grid_w0.p, B, 1.0 / a2, up);
            // U^p on the nodes by bicubic interpolation
            launch_bicubic(c, nb, bd.xy, grid->x0, grid->y0, h, grid->nx, grid->ny, up, vb);
        }
        // b = -2 alpha^2 (f - U^p), g = f - U^p
        double *b = c.ws_f.ensure(nb);
        launch_axpby(c, nb, -2.0 * a2, f_next, 2.0 * a2, vb, b);
        double *gN = c.ws_g.ensure(nb);
        launch_axpby(c, nb, 1.0, f_next, -1.0, vb, gN);
        if (stats) {
            YK_HIP(hipStreamSynchronize(c.stream));
            stats->ms[0] = fmm_last_build_ms(c);
            stats->ms[1] = ms_since(t0);
        }
        int outer = 0, guess = 0;
        GmresResult r = step_density(c, bd, alpha, b, gN, flags, tol, sigma_io, stats, outer, guess);
        // u = U^p + DL[w sigma] / alpha^2 at the cell centres
        auto t2 = std::chrono::steady_clock::now();
        {
            double *outs[3] = {u_next, nullptr, nullptr};
            SumProblem pr = pb;
            BieFuse f;
            f.w = bd.w.p;
            f.sigma = sigma_io;
            f.normal = bd.normal;
            pr.bie = &f;
            evaluate_sums(c, SLOT_VOL, pr, nullptr, nullptr, outs, vprec);
        }
        launch_axpby(c, n, 1.0, up, 1.0 / a2, u_next, u_next);
        if (!(flags & 4)) {
            NearPlan &np = near_prepare(c, bd, n, gxy);
            near_apply(c, np, bd, alpha, sigma_io, gN, up, u_next);
        }
        YK_HIP(hipStreamSynchronize(c.stream));
        if (stats) stats->ms[3] = ms_since(t2);
        fill_stats(stats, r, outer, guess);
        if (!r.converged) {
            c.last_error = "GMRES did not reach the tolerance";
            return YK_ERR_NOCONV;
        }
        return YK_OK;
    });
}

yk_status yk_box_potential(yk_ctx ctx, const yk_grid *grid, const double *B, double alpha, double *V,
                           int64_t n_pts, const double *pts, double *pts_vals) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(grid && B && V, "invalid box-code arguments");
        YK_REQUIRE(std::isfinite(grid->x0) && std::isfinite(grid->y0) && std::isfinite(grid->h) && grid->h > 0.0,
                   "invalid grid origin or cell size");
        YK_REQUIRE(grid->nx >= 4 && grid->ny >= 4 && grid->nx % 4 == 0 && grid->ny % 4 == 0 &&
                       grid->nx <= ((int64_t)1 << 17) && grid->ny <= ((int64_t)1 << 17) &&
                       grid->nx * grid->ny < ((int64_t)1 << 31),
                   "grid sides must be multiples of 4 cells, 4 .. 2^17");
        YK_REQUIRE(std::isfinite(alpha) && alpha > 0.0, "alpha must be finite and > 0");
        YK_REQUIRE(n_pts >= 0 && (n_pts == 0 || (pts && pts_vals)), "invalid evaluation points");
        box_potential(c, *grid, B, alpha, V);
        if (n_pts > 0) box_leaf_eval(c, *grid, V, n_pts, pts, pts_vals);
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_heat_step_leaves(yk_ctx ctx, const yk_boundary *bnd, const double *root, int64_t n_leaves,
                              const int32_t *level, const int32_t *ix, const int32_t *iy, const double *B,
                              int flags, const double *f_next, double alpha2, double tol, double *sigma_io,
                              double *u_next, yk_stats *stats) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(root && level && ix && iy && B && f_next && sigma_io && u_next, "invalid leaf-step arguments");
        YK_REQUIRE(std::isfinite(root[0]) && std::isfinite(root[1]) && std::isfinite(root[2]) && root[2] > 0.0,
                   "invalid root square");
        YK_REQUIRE(n_leaves >= 1 && n_leaves < ((int64_t)1 << 26), "n_leaves must be 1 .. 2^26");
        YK_REQUIRE(std::isfinite(alpha2) && alpha2 > 0.0, "alpha2 must be finite and > 0");
        YK_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
        if (stats) std::memset(stats, 0, sizeof(*stats));
        BoundaryData &bd = prepare_boundary(c, bnd);
        check_warm(c, bd);
        const int64_t n = 16 * n_leaves, nb = bd.n;
        const double a2 = alpha2, alpha = std::sqrt(alpha2);
        const SumPrec vprec = c.opt.precision == YK_PREC_FP32 ? SUM_FP32 : SUM_FP64;
        auto t0 = std::chrono::steady_clock::now();
        // U^p = V / alpha^2 at the cells (box code on the leaves), and on the
        // nodes the leaf polynomials fitted to those values
        double *up = c.grid_up.ensure(n);
        box_potential_adaptive(c, root, n_leaves, level, ix, iy, B, alpha, up);
        launch_axpby(c, n, 1.0 / a2, up, 0.0, nullptr, up);
        const double *cells = box_cells(c);
        double *vb = c.ws_e.ensure(nb);
        box_leaves_eval(c, up, nb, bd.xy, bd.gen, vb);
        double *b = c.ws_f.ensure(nb);
        launch_axpby(c, nb, -2.0 * a2, f_next, 2.0 * a2, vb, b);
        double *gN = c.ws_g.ensure(nb);
        launch_axpby(c, nb, 1.0, f_next, -1.0, vb, gN);
        if (stats) {
            YK_HIP(hipStreamSynchronize(c.stream));
            stats->ms[0] = fmm_last_build_ms(c);
            stats->ms[1] = ms_since(t0);
        }
        int outer = 0, guess = 0;
        GmresResult r = step_density(c, bd, alpha, b, gN, flags, tol, sigma_io, stats, outer, guess);
        // u = U^p + DL[w sigma] / alpha^2 at the cells
        auto t2 = std::chrono::steady_clock::now();
        {
            SumProblem pr;
            pr.n[0] = n;
            pr.xy[0] = cells;
            pr.n[1] = nb;
            pr.xy[1] = bd.xy;
            pr.normal = bd.normal;
            pr.alpha = alpha;
            double *outs[3] = {u_next, nullptr, nullptr};
            BieFuse f;
            f.w = bd.w.p;
            f.sigma = sigma_io;
            f.normal = bd.normal;
            pr.bie = &f;
            evaluate_sums(c, SLOT_VOL, pr, nullptr, nullptr, outs, vprec);
        }
        launch_axpby(c, n, 1.0, up, 1.0 / a2, u_next, u_next);
        if (!(flags & 4)) {
            NearPlan &np = near_prepare(c, bd, n, cells);
            near_apply(c, np, bd, alpha, sigma_io, gN, up, u_next);
        }
        YK_HIP(hipStreamSynchronize(c.stream));
        if (stats) stats->ms[3] = ms_since(t2);
        fill_stats(stats, r, outer, guess);
        if (!r.converged) {
            c.last_error = "GMRES did not reach the tolerance";
            return YK_ERR_NOCONV;
        }
        return YK_OK;
    });
}

yk_status yk_box_potential_adaptive(yk_ctx ctx, const double *root, int64_t n_leaves, const int32_t *level,
                                    const int32_t *ix, const int32_t *iy, const double *vals, double alpha,
                                    double *V) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(root && level && ix && iy && vals && V, "invalid box-code arguments");
        YK_REQUIRE(std::isfinite(root[0]) && std::isfinite(root[1]) && std::isfinite(root[2]) && root[2] > 0.0,
                   "invalid root square");
        YK_REQUIRE(n_leaves >= 1 && n_leaves < ((int64_t)1 << 26), "n_leaves must be 1 .. 2^26");
        YK_REQUIRE(std::isfinite(alpha) && alpha > 0.0, "alpha must be finite and > 0");
        box_potential_adaptive(c, root, n_leaves, level, ix, iy, vals, alpha, V);
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_box_refine(yk_ctx ctx, int64_t n_leaves, const double *v16, const double *v64, double tol,
                        int32_t *flags, double *err) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(n_leaves >= 0 && (n_leaves == 0 || (v16 && v64 && flags)), "invalid refinement arguments");
        YK_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
        box_refine(c, n_leaves, v16, v64, tol, flags, err);
        return YK_OK;
    });
}

yk_status yk_near_info(yk_ctx ctx, int64_t *n_near, double *setup_ms) {
    if (!ctx) return YK_ERR_ARG;
    Context &c = ctx->c;
    if (n_near) *n_near = c.near ? near_count(*c.near) : 0;
    if (setup_ms) *setup_ms = c.near ? near_setup_ms(*c.near) : 0.0;
    return YK_OK;
}

yk_status yk_rhs_backward_euler(yk_ctx ctx, int64_t n, const double *u, const double *F,
                                const int32_t *region, int n_const, const double *cvals,
                                double dt, double *B) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(n > 0 && u && region && B, "invalid arguments");
        YK_REQUIRE(n_const >= 0 && n_const <= 4096 && (n_const == 0 || cvals), "invalid constants");
        YK_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be finite and > 0");
        double *cdev = c.ws_c.ensure(n_const > 0 ? n_const : 1);
        if (n_const > 0)
            YK_HIP(hipMemcpyAsync(cdev, cvals, n_const * sizeof(double), hipMemcpyHostToDevice, c.stream));
        launch_rhs_be(c, n, u, F, region, n_const, cdev, dt, B);
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_rhs_imex(yk_ctx ctx, int scheme, int reaction, int64_t n, const double *u, const double *u_prev,
                      const double *F, const double *F_prev, const int32_t *region, int n_const,
                      const double *cvals, double dt, double *B) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(scheme == YK_SCHEME_EULER || scheme == YK_SCHEME_GEAR, "unknown scheme");
        YK_REQUIRE(reaction == YK_REACTION_NONE || reaction == YK_REACTION_ALLEN_CAHN, "unknown reaction");
        YK_REQUIRE(n > 0 && u && region && B, "invalid arguments");
        YK_REQUIRE(scheme == YK_SCHEME_EULER || u_prev, "the Gear scheme needs u_prev");
        YK_REQUIRE(n_const >= 0 && n_const <= 4096 && (n_const == 0 || cvals), "invalid constants");
        YK_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be finite and > 0");
        double *cdev = c.ws_c.ensure(n_const > 0 ? n_const : 1);
        if (n_const > 0)
            YK_HIP(hipMemcpyAsync(cdev, cvals, n_const * sizeof(double), hipMemcpyHostToDevice, c.stream));
        launch_rhs_imex(c, n, scheme == YK_SCHEME_GEAR, reaction == YK_REACTION_ALLEN_CAHN, u, u_prev, F,
                        F_prev, region, n_const, cdev, dt, B);
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_fmm_potential(yk_ctx ctx, int64_t n_vol, const double *vol_xy, const double *q,
                           const yk_boundary *bnd, const double *d, double alpha,
                           double *out_vol, double *out_bnd) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(n_vol > 0 && vol_xy && q && d && out_vol && out_bnd, "invalid arguments");
        check_alpha(alpha);
        BoundaryData &bd = prepare_boundary(c, bnd);
        SumProblem pb;
        pb.n[0] = n_vol;
        pb.xy[0] = vol_xy;
        pb.n[1] = bd.n;
        pb.xy[1] = bd.xy;
        pb.normal = bd.normal;
        pb.alpha = alpha;
        // dn_j = d_j n_j, formed as the sum gathers its sources (no quadrature
        // weight: d is the full dipole strength)
        BieFuse f;
        f.sigma = d;
        f.normal = bd.normal;
        pb.bie = &f;
        double *outs[3] = {out_vol, out_bnd, nullptr};
        evaluate_sums(c, SLOT_VOL, pb, q, nullptr, outs,
                      c.opt.precision == YK_PREC_FP32 ? SUM_FP32 : SUM_FP64);
        return YK_OK;
    });
}

void yk_ws_default_options(yk_ws_options *o) {
    if (!o) return;
    o->hidden = 256;
    o->batch = 32768;
    o->steps = 600;
    o->lr = 1e-3;
    o->max_obs = 64;
    o->seed = 1;
}

yk_status yk_ws_create(yk_ctx ctx, const yk_boundary *bnd, const yk_ws_options *opt, yk_ws *out) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        yk_ws_options o;
        yk_ws_default_options(&o);
        if (opt) o = *opt;
        YK_REQUIRE(o.hidden >= 16 && o.hidden <= 1024 && o.hidden % 16 == 0, "hidden must be a multiple of 16 in [16, 1024]");
        YK_REQUIRE(o.batch >= 64 && o.steps >= 0 && o.lr > 0 && o.max_obs >= 3, "invalid warm-start options");
        BoundaryData &bd = prepare_boundary(c, bnd);
        auto w = std::make_unique<WarmStart>(c, bd, o);
        yk_ws h = new yk_ws_s{ctx, std::move(w)};
        *out = h;
        return YK_OK;
    });
}

yk_status yk_ws_destroy(yk_ws ws) {
    if (!ws) return YK_ERR_ARG;
    if (ws->owner) {
        (void)hipStreamSynchronize(ws->owner->c.stream);
        if (ws->owner->c.warm == ws->w.get()) ws->owner->c.warm = nullptr;
    }
    delete ws;
    return YK_OK;
}

yk_status yk_ws_observe(yk_ws ws, const double *g, const double *sigma) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &) {
        YK_REQUIRE(g && sigma, "g/sigma are NULL");
        ws->w->observe(g, sigma);
        return YK_OK;
    });
}

yk_status yk_ws_train(yk_ws ws, double *loss) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &c) {
        const double l = ws->w->train();
        YK_HIP(hipStreamSynchronize(c.stream));
        if (loss) *loss = l;
        return YK_OK;
    });
}

yk_status yk_ws_predict(yk_ws ws, const double *g_next, double *sigma_out) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &) {
        YK_REQUIRE(g_next && sigma_out, "g_next/sigma_out are NULL");
        ws->w->predict(g_next, sigma_out);
        return YK_OK;
    });
}

yk_status yk_set_warm_start(yk_ctx ctx, yk_ws ws) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(!ws || ws->owner == ctx, "the warm start belongs to another context");
        c.warm = ws ? ws->w.get() : nullptr;
        return YK_OK;
    });
}

int64_t yk_ws_num_params(yk_ws ws, int *hidden, int *fp) {
    if (!ws) return -1;
    if (hidden) *hidden = ws->w->H;
    if (fp) *fp = ws->w->Fp;
    return ws->w->n_params;
}

yk_status yk_ws_get_params(yk_ws ws, float *params) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &c) {
        YK_REQUIRE(params != nullptr, "params is NULL");
        YK_HIP(hipMemcpyAsync(params, ws->w->params.p, ws->w->n_params * sizeof(float), hipMemcpyDeviceToDevice,
                              c.stream));
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_ws_set_params(yk_ws ws, const float *params) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &c) {
        YK_REQUIRE(params != nullptr, "params is NULL");
        YK_HIP(hipMemcpyAsync(ws->w->params.p, params, ws->w->n_params * sizeof(float), hipMemcpyDeviceToDevice,
                              c.stream));
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_ws_loss_grad(yk_ws ws, int64_t rows, const float *X, const float *t, float *grad, double *loss) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &c) {
        YK_REQUIRE(rows > 0 && rows < ((int64_t)1 << 31) && X && t && grad, "invalid arguments");
        const double l = ws->w->loss_grad(rows, X, t, grad);
        YK_HIP(hipStreamSynchronize(c.stream));
        if (loss) *loss = l;
        return YK_OK;
    });
}

yk_status yk_ws_forward(yk_ws ws, int64_t rows, const float *X, float *y) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &c) {
        YK_REQUIRE(rows > 0 && rows < ((int64_t)1 << 31) && X && y, "invalid arguments");
        if (c.opt.debug_flags & 32) ws->w->forward(rows, X, y);
        else ws->w->forward_fused(rows, X, y);
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_ws_adam_step(yk_ws ws, const float *grad) {
    if (!ws) return YK_ERR_ARG;
    return guarded(ws->owner, [&](Context &c) {
        YK_REQUIRE(grad != nullptr, "grad is NULL");
        ws->w->adam_step(grad);
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_plan_info_get(yk_ctx ctx, int slot, yk_plan_info *info) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(info != nullptr, "info is NULL");
        YK_REQUIRE(slot >= 0 && slot <= 4, "slot must be 0 .. 4");
        std::memset(info, 0, sizeof(*info));
        const FmmPlan *pl = plan_in_slot(c, slot);
        if (!pl) return YK_OK;
        info->valid = 1;
        info->leaf_level = pl->L;
        info->lmin = pl->lmin;
        info->p = pl->p;
        info->P = pl->P;
        info->Pp = pl->Pp;
        info->n_points = pl->N;
        info->n_boxes = pl->nbox;
        info->n_leaves = pl->nleaf;
        info->build_ms = pl->build_ms;
        info->n_ulist = pl->n_ulist;
        info->tables_ms = pl->tables_ms;
        info->order_check_ms = pl->check_ms;
        info->p_initial = pl->calib_p0;
        info->order_check_err = pl->calib_err;
        info->tree = pl->adaptive ? YK_TREE_ADAPTIVE : YK_TREE_UNIFORM;
        info->max_u = pl->max_u;
        info->n_wlist = pl->n_wl;
        info->n_xboxes = pl->n_xbox;
        if (pl->lmin <= pl->L) {
            for (int l = pl->lmin + 1; l <= pl->L; ++l) info->m2m_children += pl->lev[l].end - pl->lev[l].begin;
        }
        info->near_terms = pl->near_terms;
        info->nser = pl->nser;
        auto it = pl->active.find(pl->last_mask);
        if (it != pl->active.end()) {
            const ActiveSet &as = *it->second;
            info->pairs_charge = pl->last_has_q ? as.pairs_q : 0;
            info->pairs_dipole = pl->last_has_d ? as.pairs_d : 0;
            const bool far = pl->lmin <= pl->L;
            info->m2l_translations = far ? as.m2l_trans : 0;
            info->m2l_slots = far ? (as.m2l_sparse ? as.m2l_trans : as.n_m2l_boxes * kNumV) : 0;
            info->m2l_sparse = far && as.m2l_sparse ? 1 : 0;
            info->near_sym = as.near_sym ? 1 : 0;
            info->near_charge_values = pl->last_has_q ? (as.near_sym ? as.near_q_vals : as.pairs_q) : 0;
            info->near_incoming = pl->last_has_q && as.near_sym ? as.inc_len : 0;
            info->l2p_points = far ? as.l2p_points : 0;
            if (far)
                for (int l = pl->lmin + 1; l <= pl->L; ++l) info->l2l_children += as.l2l_count[l];
            info->p2m_points = far ? (pl->last_has_q ? pl->toff[1] - pl->toff[0] : 0) +
                                         (pl->last_has_d ? pl->toff[2] - pl->toff[1] : 0)
                                   : 0;
        }
        return YK_OK;
    });
}

yk_status yk_plan_tree_export(yk_ctx ctx, int slot, double *square, int64_t *level_begin, uint32_t *keys,
                              int32_t *perm, uint32_t *box_code, int32_t *parent, int32_t *leaf_range,
                              int32_t *ulist_off, int32_t *ulist, int32_t *vlist) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(slot >= 0 && slot <= 4, "slot must be 0 .. 4");
        const FmmPlan *pl = plan_in_slot(c, slot);
        YK_REQUIRE(pl != nullptr, "no tree is cached in this slot");
        auto copy = [&](void *dst, const void *src, size_t bytes) {
            if (dst && bytes) YK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.stream));
        };
        if (square) {
            square[0] = pl->x0;
            square[1] = pl->y0;
            square[2] = pl->size;
        }
        if (level_begin)
            for (int l = 0; l <= pl->L + 1; ++l) level_begin[l] = l <= pl->L ? pl->lev[l].begin : pl->nbox;
        copy(keys, pl->skeys.p, (size_t)pl->N * sizeof(uint32_t));
        copy(perm, pl->perm.p, (size_t)pl->N * sizeof(int32_t));
        copy(box_code, pl->bcode.p, (size_t)pl->nbox * sizeof(uint32_t));
        copy(parent, pl->bparent.p, (size_t)pl->nbox * sizeof(int32_t));
        copy(leaf_range, pl->lrange.p, (size_t)pl->nleaf * 6 * sizeof(int32_t));
        copy(ulist_off, pl->ulist_off.p, (size_t)(pl->nleaf + 1) * sizeof(int32_t));
        copy(ulist, pl->ulist.p, (size_t)pl->n_ulist * sizeof(int32_t));
        copy(vlist, pl->vlist.p, (size_t)pl->nbox * kNumV * sizeof(int32_t));
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_plan_adaptive_export(yk_ctx ctx, int slot, int32_t *leaf_box, int32_t *box_level,
                                  int32_t *wlist_off, int32_t *wlist, int32_t *xbox, int32_t *xlist_off,
                                  int32_t *xlist) {
    return guarded(ctx, [&](Context &c) {
        YK_REQUIRE(slot >= 0 && slot <= 4, "slot must be 0 .. 4");
        const FmmPlan *pl = plan_in_slot(c, slot);
        YK_REQUIRE(pl != nullptr, "no tree is cached in this slot");
        YK_REQUIRE(pl->adaptive, "the tree in this slot is not adaptive");
        auto copy = [&](void *dst, const void *src, size_t bytes) {
            if (dst && bytes) YK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.stream));
        };
        copy(leaf_box, pl->leaf_box.p, (size_t)pl->nleaf * sizeof(int32_t));
        copy(box_level, pl->blevel.p, (size_t)pl->nbox * sizeof(int32_t));
        copy(wlist_off, pl->woff.p, (size_t)(pl->nleaf + 1) * sizeof(int32_t));
        copy(wlist, pl->wl.p, (size_t)pl->n_wl * sizeof(int32_t));
        copy(xbox, pl->xbox.p, (size_t)pl->n_xbox * sizeof(int32_t));
        copy(xlist_off, pl->xoff.p, (size_t)(pl->n_xbox + 1) * sizeof(int32_t));
        copy(xlist, pl->xl.p, (size_t)pl->n_xl * sizeof(int32_t));
        YK_HIP(hipStreamSynchronize(c.stream));
        return YK_OK;
    });
}

yk_status yk_timing_enable(yk_ctx ctx, int enable) {
    return guarded(ctx, [&](Context &c) {
        resolve_timings(c);
        c.timing = enable != 0;
        return YK_OK;
    });
}

yk_status yk_timing_read(yk_ctx ctx, double ms[YK_NUM_STAGES], int64_t calls[YK_NUM_STAGES],
                         int reset) {
    return guarded(ctx, [&](Context &c) {
        resolve_timings(c);
        for (int k = 0; k < YK_NUM_STAGES; ++k) {
            if (ms) ms[k] = c.stage_ms[k];
            if (calls) calls[k] = c.stage_calls[k];
            if (reset) {
                c.stage_ms[k] = 0;
                c.stage_calls[k] = 0;
            }
        }
        return YK_OK;
    });
}

}  // extern "C"
