// fmm.hip -- placeholder until the tree and expansion kernels land.
#include "sums.h"

namespace yk {
struct FmmPlan {};
void destroy_plan(FmmPlan *p) { delete p; }
void fmm_evaluate(Context &, PlanSlot, const SumProblem &, const double *, const double *,
                  double *const[3], SumPrec) {
    throw Error{YK_ERR_ARG, "FMM backend not available; set options.direct = 1"};
}
double fmm_last_build_ms(Context &) { return 0.0; }
}  // namespace yk
