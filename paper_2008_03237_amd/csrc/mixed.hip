// Mixed-precision refinement driver (placeholder until the split kernels land).
#include "plan_internal.h"

using namespace dlpno;

extern "C" dlpno_status dlpno_solve_mixed(dlpno_plan* P, int32_t n_outer, int32_t n_inner, double* T, double* R,
                                          double* e_pair, double* e_total, double* max_abs_R, void* stream) {
  (void)n_outer; (void)n_inner; (void)T; (void)R; (void)e_pair; (void)e_total; (void)max_abs_R; (void)stream;
  if (!P) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan");
  return fail(DLPNO_ERR_UNSUPPORTED, "mixed-precision solve not available in this build");
}
