// sums.h -- one interface for the kernel sums, with a direct and an FMM backend.
#pragma once

#include "yk_internal.h"

namespace yk {

// Up to three point sets, each a target set:
//   0: charge sources (volume points),  strengths q
//   1: dipole sources (boundary nodes), dipole vectors dn = strength * normal
//   2: target-only points
// out[s] (if non-null) receives, at every point of set s,
//   sum_q q_j K0(r/alpha)/(2pi) + sum_d (x - y_j).dn_j K1(r/alpha)/(alpha r)/(2pi)
// with pairs at distance zero skipped.
// Dipole vectors formed inside a sum over boundary nodes (set 1):
// dn_j = w_j sigma_j n_j (w null: w_j = 1) instead of being passed; with kappa
// also the double-layer operator: set 1's output v becomes
// y = sigma - 2 (v + dl_diag_weight(w, kappa, 1 / alpha^2) sigma).
struct BieFuse {
    const double *w = nullptr, *sigma = nullptr, *normal = nullptr, *kappa = nullptr;
};

struct SumProblem {
    int64_t n[3] = {0, 0, 0};
    const double *xy[3] = {nullptr, nullptr, nullptr};
    double alpha = 0.0;
    const BieFuse *bie = nullptr;   // (FMM backend only; see evaluate_sums)
    const double *normal = nullptr; // unit normals of set 1 [n1][2] when known (FMM
                                    // backend: the build-time order check probes
                                    // dipoles along them)
    // FMM backend: 1 = leave the leaf multipoles of this (charges-only) pass
    // in place for a later pass; 2 = the charges equal those of that pass on
    // the same tree, with no other pass on it in between: start from its
    // multipoles and add only the dipoles' (both are hints: a pass that
    // cannot use them computes everything)
    int keep_charge_m = 0;
    // FMM backend: a fixed bounding square {x0, y0, side} for the tree (null:
    // the points' bounding square); every point must lie inside it
    const double *square = nullptr;
};

enum PlanSlot { SLOT_VOL = 0, SLOT_BND = 1, SLOT_MISC = 2, SLOT_NEAR = 3, SLOT_NEARC = 4 };

enum SumPrec { SUM_FP64 = 0, SUM_FP32 = 1 };

void evaluate_sums(Context &ctx, PlanSlot slot, const SumProblem &pb, const double *q,
                   const double *dn, double *const out[3], SumPrec prec);

// FMM backend (fmm.hip)
void fmm_evaluate(Context &ctx, PlanSlot slot, const SumProblem &pb, const double *q,
                  const double *dn, double *const out[3], SumPrec prec);
// Time spent building the last tree, in ms (0 when reused).
double fmm_last_build_ms(Context &ctx);

}  // namespace yk
