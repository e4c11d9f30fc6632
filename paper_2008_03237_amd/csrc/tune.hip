// Autotuner of the grouped kernel's schedule.
//
// For every PNO tile class (1..4 tiles of 16) it times each compiled ladder
// and projection variant of that class on the plan's own workload (the other
// classes keep their current choice), then the queue granularity, and keeps
// the fastest.  Timings are HIP events around the grouped kernel on the
// caller's stream, best of three launches; a candidate replaces the current
// choice only when it is faster by more than kMinGain, so that run-to-run
// timing noise does not flip the schedule between otherwise equal runs.
#include "plan_internal.h"

#include <algorithm>
#include <cstdio>
#include <string>

using namespace dlpno;

static constexpr float kMinGain = 0.005f;

static float time_grouped(dlpno_plan* P, const double* T, hipStream_t s, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.f;
  float best = 1e30f;
  for (int k = 0; k < reps; ++k) {
    (void)hipEventRecord(a, s);
    if (run_grouped(P, T, s) != hipSuccess) {
      best = -1.f;
      break;
    }
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    best = std::min(best, ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

static dlpno_status apply(dlpno_plan* P, hipStream_t s) {
  dlpno_status st = build_schedule(P);
  if (st != DLPNO_OK) return st;
  return upload_schedule(P, s);
}

extern "C" dlpno_status dlpno_autotune(dlpno_plan* P, const double* T, double* R, void* stream) {
  if (!P || (!T && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  (void)R;
  hipStream_t s = (hipStream_t)stream;
  const bool prof = P->profiling;
  P->profiling = false;
  std::string log;
  char buf[256];
  // which tile classes occur
  bool present[4] = {false, false, false, false};
  for (auto& pr : P->pairs_h)
    if (pr.nblk > 0) present[(pr.n + 15) / 16 - 1] = true;
  dlpno_status st = apply(P, s);
  if (st != DLPNO_OK) return st;
  float best = time_grouped(P, T, s, 3);
  if (best < 0) return fail(DLPNO_ERR_HIP, "autotune: launch failed");
  snprintf(buf, sizeof buf, "autotune start %.3f ms\n", best);
  log += buf;
  for (int nt = 1; nt <= 4; ++nt) {
    if (!present[nt - 1]) continue;
    for (int v = 0; v < kNumLadderVariants; ++v) {
      if (kLadderVariants[v].nt != nt || v == P->tune.ladder_variant[nt - 1]) continue;
      // cooperative items: FP64 only; the one-block form serves remainders
      if (kLadderCoop[v] && (P->opt.precision != DLPNO_FP64 || v == kLadderCoopOne)) continue;
      const int keep = P->tune.ladder_variant[nt - 1];
      P->tune.ladder_variant[nt - 1] = v;
      if ((st = apply(P, s)) != DLPNO_OK) return st;
      const float t = time_grouped(P, T, s, 3);
      snprintf(buf, sizeof buf, "  ladder nt=%d variant %d: %.3f ms\n", nt, v, t);
      log += buf;
      if (t > 0 && t < best * (1.f - kMinGain)) best = t;
      else P->tune.ladder_variant[nt - 1] = keep;
    }
    for (int v = 0; v < kNumProjVariants; ++v) {
      if (kProjVariants[v].nt != nt || v == P->tune.proj_variant[nt - 1]) continue;
      const int keep = P->tune.proj_variant[nt - 1];
      P->tune.proj_variant[nt - 1] = v;
      if ((st = apply(P, s)) != DLPNO_OK) return st;
      const float t = time_grouped(P, T, s, 3);
      snprintf(buf, sizeof buf, "  projection nt=%d variant %d: %.3f ms\n", nt, v, t);
      log += buf;
      if (t > 0 && t < best * (1.f - kMinGain)) best = t;
      else P->tune.proj_variant[nt - 1] = keep;
    }
  }
  if (P->opt.precision == DLPNO_FP64) {
    P->tune.two_wave = !P->tune.two_wave;
    if ((st = apply(P, s)) != DLPNO_OK) return st;
    const float t = time_grouped(P, T, s, 3);
    snprintf(buf, sizeof buf, "  two-wave ladder launch %s: %.3f ms\n", P->tune.two_wave ? "on" : "off", t);
    log += buf;
    if (t > 0 && t < best * (1.f - kMinGain)) best = t;
    else P->tune.two_wave = !P->tune.two_wave;
  }
  const double ipw[] = {2.0, 4.0, 6.0, 10.0, 16.0};
  for (double x : ipw) {
    if (x == P->tune.items_per_wave) continue;
    const double keep = P->tune.items_per_wave;
    P->tune.items_per_wave = x;
    if ((st = apply(P, s)) != DLPNO_OK) return st;
    const float t = time_grouped(P, T, s, 3);
    snprintf(buf, sizeof buf, "  items/wave %.0f: %.3f ms\n", x, t);
    log += buf;
    if (t > 0 && t < best * (1.f - kMinGain)) best = t;
    else P->tune.items_per_wave = keep;
  }
  if ((st = apply(P, s)) != DLPNO_OK) return st;
  if (hipStreamSynchronize(s) != hipSuccess) return fail(DLPNO_ERR_HIP, "autotune: sync failed");
  snprintf(buf, sizeof buf, "autotune best %.3f ms\n", best);
  log += buf;
  P->profiling = prof;
  P->info = describe(P) + log;
  return DLPNO_OK;
}
