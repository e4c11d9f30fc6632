// Mixed-precision solve with FP64 iterative refinement.
//
// The residual is affine in T: R(T) = K + (D + A) T.  Each outer step takes
// the exact FP64 residual r = R(T) (FP64 grouped kernel), then solves the
// correction equation (D + A~) delta = -r with the plan's low-precision
// operator A~ (BF16x2 / FP16x2 / FP32 contractions) by Jacobi iterations
// with DIIS on delta - the same finishing kernel with the driver replaced by
// r, FP64 denominators, updates and extrapolation - and sets T <- T + delta.
// The error of T contracts by about |(D + A~)^-1 (A~ - A)| per outer step, so
// a few FP64 residuals bring the low-precision solution to FP64 accuracy.
// After the last step one FP64 residual and Jacobi update give the reported
// amplitudes, residual norm and energies.
#include "plan_internal.h"

using namespace dlpno;

#define MIXCK(expr)                                                                                  \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return fail(DLPNO_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// FP64 residual r = R(T); energies and max |r| of the Jacobi-updated T are
// recorded in the history (the updated amplitudes go to `scratch`).  T's
// same-spin blocks are antisymmetric here (projected after every correction)
// unless the plan takes general amplitudes.
static hipError_t fp64_residual(dlpno_plan* P, const double* T, double* r, double* scratch, double* e_pair,
                                double* e_total, double* rmax, bool in_place, hipStream_t s, bool zero_T = false) {
  hipError_t e;
  if (!zero_T && (e = run_grouped(P, T, s, DLPNO_FP64)) != hipSuccess) return e;
  FinishArgs f = finish_args(P, T);
  f.no_partials = zero_T ? 1 : 0;   // T = 0: the residual is the driver alone
  f.R = r;
  f.T_new = in_place ? const_cast<double*>(T) : scratch;
  if ((e = launch_finish(f, s)) != hipSuccess) return e;
  ReduceArgs ra{};
  ra.partial = P->d_red_partial;
  ra.pairs = P->d_pairs;
  ra.blocks = P->d_blocks;
  ra.n_blocks = P->n_blocks;
  ra.n_pairs = P->n_pairs;
  ra.e_block = P->d_e_block;
  ra.rmax_block = P->d_rmax_block;
  ra.e_pair = e_pair;
  ra.e_total = e_total ? e_total : P->d_scalars;
  ra.rmax = rmax ? rmax : P->d_scalars + 1;
  ra.hist = P->d_hist;
  ra.iter = P->d_hist_iter;
  ra.hist_cap = kHistCap;
  return launch_reduce(ra, s);
}

extern "C" dlpno_status dlpno_solve_mixed(dlpno_plan* P, int32_t n_outer, int32_t n_inner, double* T, double* R,
                                          double* e_pair, double* e_total, double* max_abs_R, void* stream) {
  if (!P || n_outer < 0 || n_inner < 0 || ((!T || !R) && P->n_T > 0))
    return fail(DLPNO_ERR_INVALID_ARG, "bad arguments");
  if (P->opt.precision == DLPNO_FP64)
    return fail(DLPNO_ERR_UNSUPPORTED, "mixed solve needs a plan of precision FP32, BF16X2 or FP16X2");
  hipStream_t s = (hipStream_t)stream;
  const size_t nT = (size_t)std::max<int64_t>(P->n_T, 1);
  if (!P->d_mix_r) {
    if (hipMalloc(&P->d_mix_r, nT * sizeof(double)) != hipSuccess) {
      P->d_mix_r = nullptr;
      return fail(DLPNO_ERR_OOM, "mixed solve workspace");
    }
    if (hipMalloc(&P->d_mix_delta, nT * sizeof(double)) != hipSuccess) {
      P->d_mix_delta = nullptr;
      return fail(DLPNO_ERR_OOM, "mixed solve workspace");
    }
  }
  // The low-precision corrections carry rounding that is not antisymmetric in
  // the same-spin blocks; T is projected back onto the amplitude space (where
  // the FP64 residual mirrors those blocks) at the start and after each step.
  const bool project = (P->opt.flags & DLPNO_FLAG_GENERAL_T) == 0;
  if (project) MIXCK(launch_antisymmetrize(P->d_blocks, P->n_blocks, T, s));
  bool zero = false;
  if (n_outer > 0 && P->n_T > 0) MIXCK(amplitudes_zero(P, T, s, &zero));
  for (int o = 0; o < n_outer; ++o) {
    MIXCK(fp64_residual(P, T, P->d_mix_r, P->d_mix_delta, nullptr, nullptr, nullptr, false, s, o == 0 && zero));
    MIXCK(launch_fill(P->d_mix_delta, 0.0, P->n_T, s));
    MIXCK(launch_diis_reset(P->d_diis, std::max(1, P->opt.diis_max), std::max(1, P->opt.diis_start), s));
    // delta starts at zero: the first inner residual is -r alone (no grouped launches)
    for (int k = 0; k < n_inner; ++k)
      MIXCK(enqueue_iteration(P, P->d_mix_delta, R, nullptr, nullptr, nullptr, s, P->d_mix_r, -1, false, k == 0));
    MIXCK(launch_axpy(T, P->d_mix_delta, 1.0, P->n_T, s));
    if (project) MIXCK(launch_antisymmetrize(P->d_blocks, P->n_blocks, T, s));
  }
  MIXCK(fp64_residual(P, T, R, nullptr, e_pair, e_total, max_abs_R, true, s));
  P->host_iter += n_outer + 1;
  return read_status(P, s);
}
