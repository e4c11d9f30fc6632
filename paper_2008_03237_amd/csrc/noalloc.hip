// Residual evaluation that allocates nothing: dlpno_residual_noalloc.
//
// dlpno_residual writes the partial sums of the grouped kernel (one slot per
// spin block and auxiliary or coupling range) into a workspace the plan
// allocates.  Callers that cannot allocate device memory at all - code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation -
// get this variant, whose kernels (the same ones) use a static device array
// of the library instead.  The array exists once per GPU the library runs on
// and is held until the process ends; its device address is taken once per
// device, with that device current, when a plan is created there.
//
// No slot needs clearing: every work item overwrites all elements of the
// slots it owns, and the finishing kernel reads only slots written by the
// same call.  Calls that overlap in time on one GPU (other streams, other
// threads) share the array and race.
#include "plan_internal.h"

#include <mutex>
#include <string>

using namespace dlpno;

namespace {
// 256 MiB of FP64 partial sums per GPU
constexpr int64_t kScratchDoubles = (int64_t)1 << 25;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device
}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

dlpno_status dlpno::scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return DLPNO_OK;   // dlpno_residual_noalloc refuses such devices
  if (g_scratch[device]) return DLPNO_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(DLPNO_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch[device] = static_cast<double*>(p);
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_residual_noalloc(dlpno_plan* P, const double* T, double* R, void* stream) {
  if (!P || ((!T || !R) && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  if (P->ws_elems > kScratchDoubles)
    return fail(DLPNO_ERR_DIM_RANGE, "the plan's partial sums need " + std::to_string(P->ws_elems) +
                                         " doubles; the static scratch holds " + std::to_string(kScratchDoubles) +
                                         " (create the plan with fewer workers or items per wave)");
  double* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (P->device >= 0 && P->device < kMaxDevices) ws = g_scratch[P->device];
  }
  if (!ws) return fail(DLPNO_ERR_UNSUPPORTED, "no static scratch for device " + std::to_string(P->device));
  hipStream_t s = (hipStream_t)stream;
  // phase timing would create events: off for this call
  const bool prof = P->profiling;
  P->profiling = false;
  hipError_t e = run_grouped(P, T, s, -1, false, ws);
  if (e == hipSuccess) {
    FinishArgs f = finish_args(P, T, ws);
    f.R = R;
    e = launch_finish(f, s);
  }
  P->profiling = prof;
  if (e != hipSuccess) return fail(DLPNO_ERR_HIP, std::string("dlpno_residual_noalloc: ") + hipGetErrorString(e));
  return DLPNO_OK;
}
