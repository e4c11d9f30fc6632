// Iteration to convergence with divergence detection, and checkpoints of the
// iteration state (amplitudes, DIIS history, energy history).
#include "plan_internal.h"

#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

using namespace dlpno;

#define SOLVECK(expr)                                                                                       \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) return fail(DLPNO_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

namespace {
// iterations launched between two convergence checks (one graph replay each)
constexpr int kCheckEvery = 2;
// max |R| this many times above its smallest value since the call started:
// the iteration diverges
constexpr double kGrowth = 1e3;

struct CheckpointHeader {
  char magic[8];
  int64_t n_T, n_blocks, diis_max, hist_entries, host_iter;
};
constexpr char kMagic[8] = {'D', 'L', 'P', 'N', 'O', 'C', 'K', '1'};
}  // namespace

extern "C" dlpno_status dlpno_solve(dlpno_plan* P, int32_t max_iter, double tol_r, double tol_e, double* T,
                                    double* R, double* e_pair, double* e_total, double* max_abs_R, int32_t* n_done,
                                    void* stream) {
  if (n_done) *n_done = 0;
  if (!P || max_iter < 0 || !(tol_r >= 0.0) || !(tol_e >= 0.0) || ((!T || !R) && P->n_T > 0))
    return fail(DLPNO_ERR_INVALID_ARG, "bad arguments");
  if (P->host_iter + max_iter > kHistCap)
    return fail(DLPNO_ERR_DIM_RANGE, "the iteration history holds " + std::to_string(kHistCap) +
                                         " iterations; dlpno_reset the plan first");
  hipStream_t s = (hipStream_t)stream;
  const int64_t h0 = P->host_iter;
  int done = 0;
  double e_prev = std::numeric_limits<double>::quiet_NaN();
  double rmin = std::numeric_limits<double>::infinity();
  std::vector<double> h(2 * kCheckEvery);
  while (done < max_iter) {
    const int k = std::min(kCheckEvery, max_iter - done);
    const dlpno_status st = dlpno_iterate(P, k, T, R, e_pair, e_total, max_abs_R, stream);
    if (st != DLPNO_OK) {
      if (n_done) *n_done = done;
      return st;
    }
    SOLVECK(hipMemcpyAsync(h.data(), P->d_hist + 2 * (h0 + done), 2 * sizeof(double) * k, hipMemcpyDeviceToHost, s));
    SOLVECK(hipStreamSynchronize(s));
    for (int x = 0; x < k; ++x) {
      const double E = h[2 * x], r = h[2 * x + 1];
      rmin = std::min(rmin, r);
      if (n_done) *n_done = done + x + 1;
      if (r > kGrowth * rmin)
        return fail(DLPNO_ERR_NOT_CONVERGED, "the iteration diverges: max|R| " + std::to_string(r) + " at iteration " +
                                                 std::to_string(done + x + 1) + ", " + std::to_string(kGrowth) +
                                                 " times its smallest value " + std::to_string(rmin));
      if (r < tol_r && std::fabs(E - e_prev) < tol_e) {
        if (n_done) *n_done = done + k;   // the iterations of the last check all ran
        return DLPNO_OK;
      }
      e_prev = E;
    }
    done += k;
  }
  return fail(DLPNO_ERR_NOT_CONVERGED, "no convergence in " + std::to_string(max_iter) + " iterations");
}

extern "C" dlpno_status dlpno_checkpoint_size(const dlpno_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or output");
  const size_t nT = (size_t)P->n_T, dm = (size_t)P->opt.diis_max;
  *bytes = sizeof(CheckpointHeader) + sizeof(DiisState) + sizeof(double) * (nT + 2 * dm * nT + 2 * (size_t)kHistCap);
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_checkpoint_save(const dlpno_plan* P, const double* T, void* dst, void* stream) {
  if (!P || !dst || (!T && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)stream;
  const size_t nT = (size_t)P->n_T, dm = (size_t)P->opt.diis_max;
  CheckpointHeader hd{};
  memcpy(hd.magic, kMagic, sizeof kMagic);
  hd.n_T = P->n_T;
  hd.n_blocks = P->n_blocks;
  hd.diis_max = P->opt.diis_max;
  hd.hist_entries = kHistCap;
  hd.host_iter = P->host_iter;
  char* o = static_cast<char*>(dst);
  memcpy(o, &hd, sizeof hd);
  o += sizeof hd;
  SOLVECK(hipMemcpyAsync(o, P->d_diis, sizeof(DiisState), hipMemcpyDeviceToHost, s));
  o += sizeof(DiisState);
  if (nT > 0) SOLVECK(hipMemcpyAsync(o, T, nT * sizeof(double), hipMemcpyDeviceToHost, s));
  o += nT * sizeof(double);
  if (dm > 0 && nT > 0) {
    SOLVECK(hipMemcpyAsync(o, P->d_ring_vecs, dm * nT * sizeof(double), hipMemcpyDeviceToHost, s));
    o += dm * nT * sizeof(double);
    SOLVECK(hipMemcpyAsync(o, P->d_ring_errs, dm * nT * sizeof(double), hipMemcpyDeviceToHost, s));
    o += dm * nT * sizeof(double);
  }
  SOLVECK(hipMemcpyAsync(o, P->d_hist, 2 * kHistCap * sizeof(double), hipMemcpyDeviceToHost, s));
  SOLVECK(hipStreamSynchronize(s));
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_checkpoint_load(dlpno_plan* P, double* T, const void* src, void* stream) {
  if (!P || !src || (!T && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)stream;
  const size_t nT = (size_t)P->n_T, dm = (size_t)P->opt.diis_max;
  CheckpointHeader hd;
  const char* o = static_cast<const char*>(src);
  memcpy(&hd, o, sizeof hd);
  if (memcmp(hd.magic, kMagic, sizeof kMagic) != 0) return fail(DLPNO_ERR_INVALID_ARG, "not a checkpoint");
  if (hd.n_T != P->n_T || hd.n_blocks != P->n_blocks || hd.diis_max != P->opt.diis_max || hd.hist_entries != kHistCap)
    return fail(DLPNO_ERR_INVALID_ARG, "the checkpoint belongs to a plan of other sizes or DIIS options");
  o += sizeof hd;
  SOLVECK(hipMemcpyAsync(P->d_diis, o, sizeof(DiisState), hipMemcpyHostToDevice, s));
  o += sizeof(DiisState);
  if (nT > 0) SOLVECK(hipMemcpyAsync(T, o, nT * sizeof(double), hipMemcpyHostToDevice, s));
  o += nT * sizeof(double);
  if (dm > 0 && nT > 0) {
    SOLVECK(hipMemcpyAsync(P->d_ring_vecs, o, dm * nT * sizeof(double), hipMemcpyHostToDevice, s));
    o += dm * nT * sizeof(double);
    SOLVECK(hipMemcpyAsync(P->d_ring_errs, o, dm * nT * sizeof(double), hipMemcpyHostToDevice, s));
    o += dm * nT * sizeof(double);
  }
  SOLVECK(hipMemcpyAsync(P->d_hist, o, 2 * kHistCap * sizeof(double), hipMemcpyHostToDevice, s));
  // the device counter of recorded iterations follows the restored history
  const int32_t it = (int32_t)std::min<int64_t>(hd.host_iter, kHistCap);
  SOLVECK(hipMemcpyAsync(P->d_hist_iter, &it, sizeof it, hipMemcpyHostToDevice, s));
  SOLVECK(hipStreamSynchronize(s));
  P->host_iter = hd.host_iter;
  return DLPNO_OK;
}
