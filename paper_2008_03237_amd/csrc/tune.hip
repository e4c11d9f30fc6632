// Autotuner of the grouped kernel's schedule.
//
// For every PNO tile class (1..4 tiles of 16) it times each compiled ladder
// and projection variant of that class on the plan's own workload (the other
// classes keep their current choice), then the queue granularity and the
// persistent workgroup count, and keeps the fastest.  dlpno_autotune_cached
// persists the choices per (device architecture, precision) in a JSON file.  Timings are HIP events around the grouped kernel on the
// caller's stream, best of three launches; a candidate replaces the current
// choice only when it is faster by more than kMinGain, so that run-to-run
// timing noise does not flip the schedule between otherwise equal runs.
#include "plan_internal.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

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
      if (kLadderSplitOnly[v] && !is_split(P->opt.precision)) continue;
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
  // persistent workgroups per launch (multiples of the 8 XCDs): fewer leave
  // compute units idle but change the item sizes; more make smaller items
  {
    const double frac[] = {0.5, 0.75, 1.25, 1.5};
    for (double fr : frac) {
      const int w = std::max(8, (int)(fr * P->num_cu) / 8 * 8);
      if (w == P->workers) continue;
      const int keep = P->workers;
      P->workers = w;
      if ((st = apply(P, s)) != DLPNO_OK) return st;
      const float t = time_grouped(P, T, s, 3);
      snprintf(buf, sizeof buf, "  workgroups %d: %.3f ms\n", w, t);
      log += buf;
      if (t > 0 && t < best * (1.f - kMinGain)) best = t;
      else P->workers = keep;
    }
  }
  if ((st = apply(P, s)) != DLPNO_OK) return st;
  if (hipStreamSynchronize(s) != hipSuccess) return fail(DLPNO_ERR_HIP, "autotune: sync failed");
  snprintf(buf, sizeof buf, "autotune best %.3f ms\n", best);
  log += buf;
  P->profiling = prof;
  P->info = describe(P) + log;
  return DLPNO_OK;
}

// ---------------------------------------------------------------------------
// Persistent cache of the autotuner's choices.  A JSON file with one entry per
// (device architecture, precision), written one entry per line:
//   {"entries": [
//   {"arch": "gfx950:sramecc+:xnack-", "precision": 0, "ladder_variant": [0, 4, 7, 9],
//    "proj_variant": [0, 4, 7, 8], "items_per_wave": 6, "two_wave": 1, "workers": 256},
//   ...
//   ]}
// The reader takes the entry lines this writer produces; a file it cannot read
// counts as a miss and is rewritten.
// ---------------------------------------------------------------------------
namespace {

struct CacheEntry {
  std::string arch;
  int precision = -1;
  int ladder[4] = {0, 0, 0, 0}, proj[4] = {0, 0, 0, 0};
  double items_per_wave = 0.0;
  int two_wave = 1, workers = 0;
};

// value text after "key": in line (empty when absent)
static std::string field(const std::string& line, const char* key) {
  const std::string k = std::string("\"") + key + "\":";
  const size_t at = line.find(k);
  if (at == std::string::npos) return "";
  size_t b = at + k.size();
  while (b < line.size() && line[b] == ' ') ++b;
  size_t e = b;
  if (b < line.size() && line[b] == '"') {
    e = line.find('"', b + 1);
    return e == std::string::npos ? "" : line.substr(b + 1, e - b - 1);
  }
  if (b < line.size() && line[b] == '[') {
    e = line.find(']', b);
    return e == std::string::npos ? "" : line.substr(b + 1, e - b - 1);
  }
  while (e < line.size() && line[e] != ',' && line[e] != '}') ++e;
  return line.substr(b, e - b);
}

static bool parse_entry(const std::string& line, CacheEntry& c) {
  c.arch = field(line, "arch");
  const std::string pr = field(line, "precision"), lv = field(line, "ladder_variant"), pv = field(line, "proj_variant"),
                    ipw = field(line, "items_per_wave"), tw = field(line, "two_wave"), wk = field(line, "workers");
  if (c.arch.empty() || pr.empty() || lv.empty() || pv.empty() || ipw.empty() || tw.empty() || wk.empty()) return false;
  c.precision = atoi(pr.c_str());
  if (sscanf(lv.c_str(), "%d , %d , %d , %d", &c.ladder[0], &c.ladder[1], &c.ladder[2], &c.ladder[3]) != 4) return false;
  if (sscanf(pv.c_str(), "%d , %d , %d , %d", &c.proj[0], &c.proj[1], &c.proj[2], &c.proj[3]) != 4) return false;
  c.items_per_wave = atof(ipw.c_str());
  c.two_wave = atoi(tw.c_str());
  c.workers = atoi(wk.c_str());
  for (int t = 0; t < 4; ++t)
    if (c.ladder[t] < 0 || c.ladder[t] >= kNumLadderVariants || kLadderVariants[c.ladder[t]].nt != t + 1 ||
        c.proj[t] < 0 || c.proj[t] >= kNumProjVariants || kProjVariants[c.proj[t]].nt != t + 1)
      return false;
  return c.items_per_wave > 0.0 && c.workers > 0;
}

static std::vector<CacheEntry> read_cache(const char* path) {
  std::vector<CacheEntry> out;
  FILE* f = fopen(path, "r");
  if (!f) return out;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    CacheEntry c;
    if (parse_entry(buf, c)) out.push_back(c);
  }
  fclose(f);
  return out;
}

static bool write_cache(const char* path, const std::vector<CacheEntry>& es) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\"entries\": [\n");
  for (size_t k = 0; k < es.size(); ++k) {
    const CacheEntry& c = es[k];
    fprintf(f,
            "{\"arch\": \"%s\", \"precision\": %d, \"ladder_variant\": [%d, %d, %d, %d], \"proj_variant\": [%d, %d, %d, "
            "%d], \"items_per_wave\": %g, \"two_wave\": %d, \"workers\": %d}%s\n",
            c.arch.c_str(), c.precision, c.ladder[0], c.ladder[1], c.ladder[2], c.ladder[3], c.proj[0], c.proj[1],
            c.proj[2], c.proj[3], c.items_per_wave, c.two_wave, c.workers, k + 1 < es.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" dlpno_status dlpno_autotune_cached(dlpno_plan* P, const double* T, double* R, const char* path,
                                              int32_t* hit, void* stream) {
  if (hit) *hit = 0;
  if (!P || !path || (!T && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan, path or buffer");
  hipStream_t s = (hipStream_t)stream;
  std::vector<CacheEntry> es = read_cache(path);
  for (const CacheEntry& c : es) {
    if (c.arch != P->arch || c.precision != (int)P->opt.precision) continue;
    for (int t = 0; t < 4; ++t) {
      P->tune.ladder_variant[t] = c.ladder[t];
      P->tune.proj_variant[t] = c.proj[t];
    }
    P->tune.items_per_wave = c.items_per_wave;
    P->tune.two_wave = c.two_wave != 0;
    P->workers = c.workers;
    const dlpno_status st = apply(P, s);
    if (st != DLPNO_OK) return st;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(DLPNO_ERR_HIP, "autotune cache: sync failed");
    P->info = describe(P) + "autotune choices read from " + std::string(path) + "\n";
    if (hit) *hit = 1;
    return DLPNO_OK;
  }
  const dlpno_status st = dlpno_autotune(P, T, R, stream);
  if (st != DLPNO_OK) return st;
  CacheEntry c;
  c.arch = P->arch;
  c.precision = (int)P->opt.precision;
  for (int t = 0; t < 4; ++t) {
    c.ladder[t] = P->tune.ladder_variant[t];
    c.proj[t] = P->tune.proj_variant[t];
  }
  c.items_per_wave = P->tune.items_per_wave;
  c.two_wave = P->tune.two_wave ? 1 : 0;
  c.workers = P->workers;
  std::vector<CacheEntry> keep;
  for (const CacheEntry& e : es)
    if (!(e.arch == c.arch && e.precision == c.precision)) keep.push_back(e);
  keep.push_back(c);
  if (!write_cache(path, keep)) return fail(DLPNO_ERR_INVALID_ARG, std::string("cannot write the autotune cache ") + path);
  return DLPNO_OK;
}
