// fmm.hip -- FMM backend of the kernel sums: plan cache and evaluation.
#include <chrono>

#include <atomic>

#include "fmm.h"

namespace yk {

void destroy_plan(FmmPlan *p) { delete p; }

namespace {

PlanPtr &slot_ref(Context &ctx, PlanSlot slot) {
    switch (slot) {
        case SLOT_VOL: return ctx.plan_vol;
        case SLOT_BND: return ctx.plan_bnd;
        case SLOT_NEAR: return ctx.plan_near;
        case SLOT_NEARC: return ctx.plan_nearc;
        default: return ctx.plan_misc;
    }
}

bool plan_matches(const FmmPlan &pl, const Context &ctx, const SumProblem &pb) {
    for (int s = 0; s < 3; ++s)
        if (pl.key_n[s] != pb.n[s] || pl.key_xy[s] != (pb.n[s] ? pb.xy[s] : nullptr)) return false;
    return pl.alpha == pb.alpha && pl.opt_p == ctx.opt.p && pl.opt_leaf == ctx.opt.leaf_size &&
           pl.opt_tol == ctx.opt.fmm_tol && pl.opt_tree == ctx.opt.tree;
}

}  // namespace

FmmPlan &get_plan(Context &ctx, PlanSlot slot, const SumProblem &pb) {
    PlanPtr &ref = slot_ref(ctx, slot);
    if (ref && plan_matches(*ref, ctx, pb)) {
        ref->fresh = false;
        return *ref;
    }
    ref.reset();
    PlanPtr pl(new FmmPlan());
    for (int s = 0; s < 3; ++s) {
        pl->key_n[s] = pb.n[s];
        pl->key_xy[s] = pb.n[s] ? pb.xy[s] : nullptr;
    }
    static std::atomic<uint64_t> plan_gen{0};
    pl->gen = ++plan_gen;
    pl->alpha = pb.alpha;
    pl->opt_p = ctx.opt.p;
    pl->opt_leaf = ctx.opt.leaf_size;
    pl->opt_tol = ctx.opt.fmm_tol;
    pl->opt_tree = ctx.opt.tree;
    const auto t0 = std::chrono::steady_clock::now();
    build_tree(ctx, *pl, pb);
    calibrate_order(ctx, *pl, pb);
    pl->last_mask = 0;
    pl->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    pl->fresh = true;
    ref = std::move(pl);
    return *ref;
}

void fmm_evaluate(Context &ctx, PlanSlot slot, const SumProblem &pb, const double *q,
                  const double *dn, double *const out[3], SumPrec prec) {
    FmmPlan &pl = get_plan(ctx, slot, pb);
    fmm_run(ctx, pl, q, dn, out, prec, pb.bie, pb.keep_charge_m);
}

double fmm_last_build_ms(Context &ctx) {
    double ms = 0;
    for (PlanPtr *p : {&ctx.plan_vol, &ctx.plan_bnd, &ctx.plan_misc, &ctx.plan_near, &ctx.plan_nearc})
        if (*p && (*p)->fresh) ms += (*p)->build_ms;
    return ms;
}

}  // namespace yk
