// C ABI of the DLPNO doubles-residual library: descriptor validation, device
// tables, the longest-first work schedule of the grouped kernel, hipGraph
// replay of one iteration, precision copies and phase timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/dlpno.h"
#include "internal.h"
#include "plan_internal.h"
#include "split_internal.h"

using namespace dlpno;

static thread_local std::string g_last_error;

namespace dlpno {
dlpno_status fail(dlpno_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
}  // namespace dlpno

#define HIPCK(expr)                                                                          \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(DLPNO_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

namespace {

int block_code(int s1, int s2) { return s1 == s2 ? s1 : (s1 == 0 ? 2 : 3); }
const int kCodeS1[4] = {0, 1, 0, 1};
const int kCodeS2[4] = {0, 1, 1, 0};
const uint32_t kCodeBit[4] = {DLPNO_AA, DLPNO_BB, DLPNO_AB, DLPNO_BA};

// Block rule (paper Sec. II.A, high-spin cases): s s' kept iff i in occ_s,
// j in occ_s', not (s == s' and i == j), and BA dropped for i == j.
uint32_t rule_mask(int i, int j, const uint8_t* somo) {
  uint32_t m = 0;
  for (int c = 0; c < 4; ++c) {
    const int s1 = kCodeS1[c], s2 = kCodeS2[c];
    const bool in1 = s1 == 0 || !somo[i];
    const bool in2 = s2 == 0 || !somo[j];
    if (!in1 || !in2) continue;
    if (s1 == s2 && i == j) continue;
    if (i == j && c == 3) continue;
    m |= kCodeBit[c];
  }
  return m;
}

int popcount4(uint32_t m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1); }

template <typename T>
dlpno_status dev_alloc(T** p, size_t count, const char* what) {
  *p = nullptr;
  if (count == 0) return DLPNO_OK;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(DLPNO_ERR_OOM, std::string("hipMalloc failed for ") + what + " (" +
                                   std::to_string(count * sizeof(T)) + " bytes)");
  }
  return DLPNO_OK;
}

template <typename T>
dlpno_status upload(T** p, const std::vector<T>& h, const char* what, hipStream_t s) {
  dlpno_status st = dev_alloc(p, h.size(), what);
  if (st != DLPNO_OK) return st;
  if (!h.empty()) HIPCK(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return DLPNO_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// schedule
// ---------------------------------------------------------------------------
namespace dlpno {

// Work of one ladder item per auxiliary function and block, in 16x16x4 MFMA
// times: both stages issue nt x nta x s4 of them.  In FP64 a partial last
// tile (r = s4 - 4 (nt - 1) < 4 k-steps in it) runs as r row strips of the
// four-block 4x4x4 MFMA, each about 0.22 of a 16x16x4 instruction, and with
// r <= kColStrips the last a-tile as r column strips in both stages.
double ladder_block_mfma_per_q(int nt, int ta0, int nta, int dta, int s4, bool strips, bool mirror) {
  const int r = s4 - 4 * (nt - 1);
  const double last = strips && r < 4 ? 0.22 * r : 1.0;
  const bool cs = strips && r <= kColStrips && ta0 + (nta - 1) * dta == nt - 1;
  double st1 = 0.0, st2 = 0.0;
  for (int u = 0; u < nta; ++u) {
    const bool colu = cs && u == nta - 1;
    st1 += (nt - 1 + last) * (colu ? 0.22 * r : 1.0);
    for (int tb = 0; tb < nt; ++tb)
      if (!mirror || tb >= ta0 + u * dta) st2 += colu ? 0.22 * r : tb == nt - 1 ? last : 1.0;
  }
  return s4 * (st1 + st2);
}
double ladder_mfma_per_q(int nt, int nta, int s4, bool strips) {
  // a-tiles 0 .. nta - 1 of a block that computes every tile
  return ladder_block_mfma_per_q(nt, 0, nta, 1, s4, strips, false);
}

// largest compiled variant with this tile shape handling at most maxnb blocks
// (split-only variants only for split-precision items)
int pick_ladder(int nt, int nta, int maxnb, bool split) {
  int best = -1;
  for (int v = 0; v < kNumLadderVariants; ++v) {
    const LadderVariant& V = kLadderVariants[v];
    if (kLadderSplitOnly[v] && !split) continue;
    if (V.nt == nt && V.nta == nta && V.nb <= maxnb && (best < 0 || V.nb > kLadderVariants[best].nb)) best = v;
  }
  if (best >= 0) return best;
  // no variant with this a-tile grouping fits: any of the same tile count
  for (int v = 0; v < kNumLadderVariants; ++v) {
    const LadderVariant& V = kLadderVariants[v];
    if (kLadderSplitOnly[v] && !split) continue;
    if (V.nt == nt && V.nb <= maxnb && (best < 0 || V.nb > kLadderVariants[best].nb)) best = v;
  }
  return best;
}
int pick_proj(int nt, int maxnb) {
  int best = -1;
  for (int v = 0; v < kNumProjVariants; ++v) {
    const ProjVariant& V = kProjVariants[v];
    if (V.nt == nt && V.nb <= maxnb && (best < 0 || V.nb > kProjVariants[best].nb)) best = v;
  }
  return best;
}

// Whether the kernels have a compiled body for an item of this kind and
// variant in precision prec: mirrors the switch statements of run_item and
// grouped_coop_kernel (grouped_impl.h) and split_run_item (split.hip).
bool item_compiled(const Item& it, int prec) {
  const bool fp64 = prec == DLPNO_FP64;
  const int v = it.variant;
  switch (it.kind) {
    case ITEM_LADDER:
      return v >= 0 && v < kNumLadderVariants && !kLadderCoop[v] && (is_split(prec) || !kLadderSplitOnly[v]);
    case ITEM_LADDER2: return fp64 && v >= 0 && v < kNumLadderVariants && kLadderTwoWave[v];
    case ITEM_LADDER4: return fp64 && (v == kLadderCoopPair || v == kLadderCoopOne);
    case ITEM_PROJ2: {
      const int tv = v >> 2, cq = (v & 3) + 1;
      return fp64 && v >= 0 && tv < kNumProjVariants && kProjTwoWave[tv] && cq <= 3;
    }
    case ITEM_PROJ: {
      const int tv = v >> 2, cq = (v & 3) + 1;
      if (v < 0 || tv >= kNumProjVariants) return false;
      // FP64/FP32: three target tiles in pairs of blocks take at most three source tiles
      return is_split(prec) || !(tv == 6 && cq == 4);
    }
    default: return false;
  }
}

struct Cand {
  Item it;
  double cost;
};

// Items by kind in launch order (one set of queues and one launch each),
// longest first within a kind, ties by pair for a deterministic order.  One
// queue per XCD: the items of one (pair, slot) read the same B^Q or S slices
// and go to one queue; groups are dealt out in that order to the
// least-loaded queue, and each queue keeps the longest-first order.
void partition(std::vector<Cand>& cand, Schedule& S, double& maxc) {
  int rank[kKinds];
  for (int k = 0; k < kKinds; ++k) rank[kKindOrder[k]] = k;
  std::stable_sort(cand.begin(), cand.end(), [&](const Cand& a, const Cand& b) {
    if (a.it.kind != b.it.kind) return rank[a.it.kind] < rank[b.it.kind];
    return a.cost > b.cost;
  });
  S.items_h.clear();
  S.items_h.reserve(cand.size());
  for (int kind : kKindOrder) {
    std::vector<std::vector<Item>> qs(kQueues);
    double load[kQueues] = {};
    std::unordered_map<int64_t, int> group_q;
    for (const Cand& c : cand) {
      if (c.it.kind != kind) continue;
      const int64_t key = ((int64_t)c.it.pair << 32) | (uint32_t)c.it.slot;
      auto g = group_q.find(key);
      int q = 0;
      if (g != group_q.end()) {
        q = g->second;
      } else {
        for (int k = 1; k < kQueues; ++k)
          if (load[k] < load[q]) q = k;
        group_q.emplace(key, q);
      }
      qs[q].push_back(c.it);
      load[q] += c.cost;
      maxc = std::max(maxc, c.cost);
    }
    const int32_t base = (int32_t)S.items_h.size();
    for (int k = 0; k < kQueues; ++k) {
      S.qoff[kind][k] = (int32_t)S.items_h.size() - base;
      S.items_h.insert(S.items_h.end(), qs[k].begin(), qs[k].end());
    }
    S.qoff[kind][kQueues] = (int32_t)S.items_h.size() - base;
    S.kind_begin[kind] = base;
    S.kind_count[kind] = S.qoff[kind][kQueues];
  }
}

dlpno_status build_schedule(dlpno_plan* P) {
  const int npairs = P->n_pairs;
  const bool strips = P->opt.precision == DLPNO_FP64;
  const bool two_wave = P->opt.precision == DLPNO_FP64 && P->tune.two_wave;
  // split plans also keep FP64 items over the same slots for their FP64
  // residuals (refinement), in the FP64 launches
  const bool split = P->opt.precision == DLPNO_BF16X2 || P->opt.precision == DLPNO_FP16X2;
  constexpr int kFp64Ladder[4] = {0, 4, 7, kLadderCoopPair};
  std::vector<int> nL(npairs, 0), nP(npairs, 0);
  std::vector<Cand> cand, cand64;
  // total work in MFMA instructions, to size the items
  double total = 0.0;
  for (int p = 0; p < npairs; ++p) {
    const PairDev& pr = P->pairs_h[p];
    if (pr.nblk == 0) continue;
    const int nt = (pr.n + 15) / 16, s4 = (pr.n + 3) / 4;
    total += (double)pr.m * pr.nblk * ladder_mfma_per_q(nt, nt, s4, strips);
    for (int64_t e = P->rowptr_h[p]; e < P->rowptr_h[p + 1]; ++e) {
      const int nq = P->cpl_h[e].nsrc;
      const int ntq = (nq + 15) / 16, s4q = (nq + 3) / 4;
      total += (double)pr.nblk * (nt * ntq + nt * nt) * s4q;
    }
  }
  const int waves = std::max(1, P->workers * 4);
  double target = total / (waves * P->tune.items_per_wave);
  target = std::max(target, (double)P->tune.min_item_mfma);
  P->total_mfma = total;

  for (int p = 0; p < npairs; ++p) {
    const PairDev& pr = P->pairs_h[p];
    if (pr.nblk == 0) continue;
    const int nt = (pr.n + 15) / 16, s4 = (pr.n + 3) / 4;
    // ladder: block groups of the tuned variant, smaller variants of the same
    // tile shape for the remainder
    // the cooperative variants run in a two-wave FP64 launch only; elsewhere
    // four-tile pairs take the one-wave variant 8
    int lv = P->tune.ladder_variant[nt - 1];
    if (kLadderCoop[lv] && !two_wave) lv = 8;
    const LadderVariant V = kLadderVariants[lv];
    // work per wave: a cooperative item is shared by the workgroup's 4 waves
    const double per_q = (double)V.nb * ladder_mfma_per_q(V.nt, V.nta, s4, strips) / (kLadderCoop[lv] ? 4.0 : 1.0);
    int chunks = (int)std::ceil(per_q * pr.m / target);
    chunks = std::max(1, std::min(chunks, pr.m));
    nL[p] = chunks;
    // the items of ladder slot c (Q in [lo, hi)) with variant lvx; tw: the
    // FP64 two-wave launches are in use, stx: FP64 row strips
    auto emit_ladder = [&](std::vector<Cand>& out, int lvx, bool tw, bool stx, int c, int lo, int hi,
                           bool splitx) -> bool {
      const LadderVariant VX = kLadderVariants[lvx];
      for (int b0 = 0; b0 < pr.nblk;) {
        const int v = pick_ladder(nt, VX.nta, std::min(VX.nb, pr.nblk - b0), splitx);
        if (v < 0) return false;
        const LadderVariant W = kLadderVariants[v];
        for (int ta0 = 0; ta0 < nt; ta0 += W.nta) {
          Item it{};
          it.kind = kLadderCoop[v] ? ITEM_LADDER4 : tw && kLadderTwoWave[v] ? ITEM_LADDER2 : ITEM_LADDER;
          it.variant = v;
          it.pair = p;
          it.bslot0 = b0;
          it.slot = c;
          it.ta0 = ta0;
          it.lo = lo;
          it.hi = hi;
          // duration: the blocks' work, counting for an antisymmetric block only
          // the stage-2 tiles it computes; a cooperative item takes as long as
          // its slower block, shared by two waves
          double cost = 0.0;
          for (int b = 0; b < W.nb; ++b) {
            const bool mirror = !(P->opt.flags & DLPNO_FLAG_GENERAL_T) && P->blocks_h[pr.blk0 + b0 + b].anti != 0;
            const double cb = ladder_block_mfma_per_q(W.nt, ta0, W.nta, 1, s4, stx, mirror);
            cost = kLadderCoop[v] ? std::max(cost, cb / 2.0) : cost + cb;
          }
          out.push_back({it, (double)(hi - lo) * cost});
        }
        b0 += W.nb;
      }
      return true;
    };
    for (int c = 0; c < chunks; ++c) {
      const int lo = (int)((int64_t)pr.m * c / chunks), hi = (int)((int64_t)pr.m * (c + 1) / chunks);
      if (!emit_ladder(cand, lv, two_wave, strips, c, lo, hi, split) ||
          (split && !emit_ladder(cand64, kFp64Ladder[nt - 1], true, true, c, lo, hi, false)))
        return fail(DLPNO_ERR_INVALID_ARG, "no ladder tile variant for this block group");
    }
    // projection
    const int64_t e0 = P->rowptr_h[p], e1 = P->rowptr_h[p + 1];
    if (e1 > e0) {
      const int pv = P->tune.proj_variant[nt - 1];
      const ProjVariant U = kProjVariants[pv];
      // chunk the coupling list by cost, never across a change of the source
      // tile count (one compiled body per count)
      std::vector<std::pair<int64_t, int64_t>> ranges;
      double acc = 0.0;
      int64_t start = e0;
      for (int64_t e = e0; e < e1; ++e) {
        const int nq = P->cpl_h[e].nsrc;
        acc += (double)U.nb * (nt * ((nq + 15) / 16) + nt * nt) * 4 * ((nq + 15) / 16);
        const bool cls_end = e + 1 < e1 && (P->cpl_h[e + 1].nsrc + 15) / 16 != (nq + 15) / 16;
        if ((acc >= target || cls_end) && e + 1 < e1) {
          ranges.push_back({start, e + 1});
          start = e + 1;
          acc = 0.0;
        }
      }
      ranges.push_back({start, e1});
      nP[p] = (int)ranges.size();
      for (size_t c = 0; c < ranges.size(); ++c) {
        double cost = 0.0;
        const int cq = (P->cpl_h[ranges[c].first].nsrc + 15) / 16;
        for (int64_t e = ranges[c].first; e < ranges[c].second; ++e) cost += (nt * cq + nt * nt) * 4 * cq;
        // three target tiles with four source tiles: one block per item (two
        // blocks' accumulators and operands do not fit the registers)
        const int nbmax = nt == 3 && cq == 4 ? 1 : U.nb;
        for (int pass = 0; pass < (split ? 2 : 1); ++pass) {
          const bool tw = pass == 1 || two_wave;
          for (int b0 = 0; b0 < pr.nblk;) {
            const int v = pick_proj(nt, std::min(nbmax, pr.nblk - b0));
            if (v < 0) return fail(DLPNO_ERR_INVALID_ARG, "no projection tile variant for this block group");
            Item it{};
            it.kind = tw && kProjTwoWave[v] && cq <= 3 ? ITEM_PROJ2 : ITEM_PROJ;
            it.variant = v * 4 + (cq - 1);
            it.pair = p;
            it.bslot0 = b0;
            it.slot = nL[p] + (int)c;
            it.ta0 = 0;
            it.lo = (int)ranges[c].first;
            it.hi = (int)ranges[c].second;
            (pass == 0 ? cand : cand64).push_back({it, cost * kProjVariants[v].nb});
            b0 += kProjVariants[v].nb;
          }
        }
      }
    }
  }
  // workspace slots
  int64_t ws = 0;
  for (int p = 0; p < npairs; ++p) {
    const PairDev& pr = P->pairs_h[p];
    for (int b = 0; b < pr.nblk; ++b) {
      BlockDev& bk = P->blocks_h[pr.blk0 + b];
      // the ring/exchange contractions of a block own its last slot
      bk.nslot = nL[p] + nP[p] + (P->rx_block.empty() ? 0 : P->rx_block[pr.blk0 + b]);
      bk.slot_proj = nL[p];
      bk.off_ws = ws;
      ws += (int64_t)bk.nslot * pr.n * pr.n;
    }
  }
  P->ws_elems = ws;
  double maxc = 0.0;
  partition(cand, P->sched, maxc);
  double unused = 0.0;
  P->sched64.items_h.clear();
  if (split) partition(cand64, P->sched64, unused);
  P->max_item_mfma = maxc;
  // every item must have a compiled kernel body (an item without one would
  // leave its partial slot stale)
  for (const Item& it : P->sched.items_h)
    if (!item_compiled(it, P->opt.precision))
      return fail(DLPNO_ERR_UNSUPPORTED, "schedule item (kind " + std::to_string(it.kind) + ", variant " +
                                             std::to_string(it.variant) + ") has no compiled kernel body");
  for (const Item& it : P->sched64.items_h)
    if (!item_compiled(it, DLPNO_FP64))
      return fail(DLPNO_ERR_UNSUPPORTED, "FP64 schedule item (kind " + std::to_string(it.kind) + ", variant " +
                                             std::to_string(it.variant) + ") has no compiled kernel body");
  return DLPNO_OK;
}

}  // namespace dlpno

// ---------------------------------------------------------------------------
// device state (re)allocation for the schedule
// ---------------------------------------------------------------------------
dlpno_status dlpno::upload_schedule(dlpno_plan* P, hipStream_t s) {
  if (P->sched.d_items) (void)hipFree(P->sched.d_items);
  if (P->sched64.d_items) (void)hipFree(P->sched64.d_items);
  if (P->d_blocks) (void)hipFree(P->d_blocks);
  if (P->d_ws) (void)hipFree(P->d_ws);
  P->sched.d_items = nullptr;
  P->sched64.d_items = nullptr;
  P->d_blocks = nullptr;
  P->d_ws = nullptr;
  dlpno_status st;
  if ((st = upload(&P->sched.d_items, P->sched.items_h, "work items", s)) != DLPNO_OK) return st;
  if ((st = upload(&P->sched64.d_items, P->sched64.items_h, "FP64 work items", s)) != DLPNO_OK) return st;
  if ((st = upload(&P->d_blocks, P->blocks_h, "block table", s)) != DLPNO_OK) return st;
  if ((st = dev_alloc(&P->d_ws, (size_t)std::max<int64_t>(P->ws_elems, 1), "partial-sum workspace")) != DLPNO_OK)
    return st;
  P->graph_valid = false;
  return DLPNO_OK;
}

std::string dlpno::describe(const dlpno_plan* P) {
  char buf[1024];
  std::string s;
  snprintf(buf, sizeof buf,
           "pairs=%d blocks=%d couplings=%lld (hole-hole %lld) terms=%lld precision=%d workers=%d items=%zu (ladder %d, ladder at two "
           "waves per SIMD %d, cooperative ladder %d, projection %d, projection at two waves per SIMD %d) "
           "max_item/total=%.2e workspace=%.3f GB\n",
           P->n_pairs, P->n_blocks, (long long)P->n_cpl, (long long)P->n_hh, (long long)P->n_terms, (int)P->opt.precision, P->workers,
           P->sched.items_h.size(), P->sched.kind_count[ITEM_LADDER], P->sched.kind_count[ITEM_LADDER2],
           P->sched.kind_count[ITEM_LADDER4], P->sched.kind_count[ITEM_PROJ], P->sched.kind_count[ITEM_PROJ2],
           P->total_mfma > 0 ? P->max_item_mfma / P->total_mfma : 0.0, P->ws_elems * 8.0 / 1e9);
  s += buf;
  snprintf(buf, sizeof buf,
           "ladder variants by tiles: %d %d %d %d%s; projection: %d %d %d %d; items/wave %.1f\n",
           P->tune.ladder_variant[0], P->tune.ladder_variant[1], P->tune.ladder_variant[2], P->tune.ladder_variant[3],
           P->sched.kind_count[ITEM_LADDER2] > 0 ? " (two-wave launch)" : "", P->tune.proj_variant[0],
           P->tune.proj_variant[1], P->tune.proj_variant[2], P->tune.proj_variant[3], P->tune.items_per_wave);
  s += buf;
  if (!P->sched64.items_h.empty()) {
    snprintf(buf, sizeof buf, "FP64 items for refinement residuals: %zu\n", P->sched64.items_h.size());
    s += buf;
  }
  snprintf(buf, sizeof buf, "flops/residual: ladder %.4e projection %.4e quadratic-term weights %.4e\n",
           P->flops_ladder, P->flops_proj, P->flops_quad);
  s += buf;
  if (!P->quad_h.empty()) {
    snprintf(buf, sizeof buf, "quadratic term: %zu couplings, factors S K S^T %.3f GB (%.4e flops, once)\n",
             P->quad_h.size(), P->n_quadG * 8e-9, P->flops_quad_prep);
  } else {
    buf[0] = 0;
  }
  s += buf;
  if (P->qocc) {
    snprintf(buf, sizeof buf,
             "occupied-intermediate quadratic term: %zu contributions, %zu dressed terms, factors %.3f GB (%.4e flops, "
             "once), %.4e flops per residual\n",
             P->occ_ctb_h.size(), P->occ_terms_h.size(), P->n_occG * 8e-9, P->flops_occ_prep, P->flops_occ);
    s += buf;
  }
  if (P->n_ring > 0) {
    snprintf(buf, sizeof buf, "ring/exchange term: %lld couplings, %zu contractions over %zu blocks, %.4e flops\n",
             (long long)P->n_ring, P->rx_terms_h.size(), P->rx_units_h.size(), P->flops_rx);
    s += buf;
  }
  return s;
}

// ---------------------------------------------------------------------------
// plan creation
// ---------------------------------------------------------------------------
extern "C" dlpno_status dlpno_plan_create(const dlpno_problem* prob, const dlpno_inputs* in,
                                          const dlpno_options* opts, void* stream, dlpno_plan** out) {
  g_last_error.clear();
  if (!out) return fail(DLPNO_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!prob || !in) return fail(DLPNO_ERR_INVALID_ARG, "problem or inputs is NULL");
  const int n_occ = prob->n_occ, npairs = prob->n_pairs;
  if (n_occ < 1 || npairs < 0 || prob->n_couplings < 0)
    return fail(DLPNO_ERR_DIM_RANGE, "n_occ must be >= 1, n_pairs and n_couplings >= 0");
  if (!prob->is_somo || !prob->f_a || !prob->f_b || !prob->cpl_rowptr || (npairs > 0 && !prob->pairs) ||
      (prob->n_couplings > 0 && !prob->cpl) || (prob->n_hh > 0 && (!prob->hh_rowptr || !prob->hh)) ||
      (prob->n_ring > 0 && (!prob->ring_rowptr || !prob->ring)))
    return fail(DLPNO_ERR_INVALID_ARG, "a required host array is NULL");
  if (prob->n_ring < 0 || prob->n_ring_ints < 0) return fail(DLPNO_ERR_DIM_RANGE, "n_ring and n_ring_ints must be >= 0");
  dlpno_options opt{};
  opt.precision = DLPNO_FP64;
  opt.diis_max = 8;
  opt.diis_start = 3;
  if (opts) opt = *opts;
  if (opt.precision < DLPNO_FP64 || opt.precision > DLPNO_FP16X2)
    return fail(DLPNO_ERR_INVALID_ARG, "unknown precision");
  if (opt.diis_max < 0 || opt.diis_max > 8) return fail(DLPNO_ERR_INVALID_ARG, "diis_max must be in 0..8");
  if ((opt.flags & ~(DLPNO_FLAG_GENERAL_T | DLPNO_FLAG_QUADRATIC | DLPNO_FLAG_QUADRATIC_OCC)) != 0)
    return fail(DLPNO_ERR_INVALID_ARG, "unknown option flag");
  const bool qocc = (opt.flags & DLPNO_FLAG_QUADRATIC_OCC) != 0;
  const bool quad = (opt.flags & DLPNO_FLAG_QUADRATIC) != 0;
  if (quad && prob->n_hh <= 0) return fail(DLPNO_ERR_INVALID_ARG, "the quadratic term needs hole-hole couplings");
  if (opt.diis_max > 0 && (opt.diis_start < 1 || opt.diis_start > opt.diis_max))
    return fail(DLPNO_ERR_INVALID_ARG, "diis_start must be in 1..diis_max");
  for (int k = 0; k < n_occ; ++k)
    if (prob->is_somo[k] > 1) return fail(DLPNO_ERR_INVALID_ARG, "is_somo entries must be 0 or 1");
  const bool need_inputs = npairs > 0;
  if (need_inputs && (!in->B || !in->K || !in->eps_a || !in->eps_b ||
                     (prob->n_couplings + prob->n_hh + prob->n_ring > 0 && !in->S) ||
                     (prob->n_ring > 0 && !in->ring_ints)))
    return fail(DLPNO_ERR_INVALID_ARG, "a device input pointer is NULL");

  hipStream_t s = (hipStream_t)stream;
  dlpno_plan* P = new dlpno_plan();
  P->opt = opt;
  P->n_occ = n_occ;
  P->n_pairs = npairs;

  P->in = *in;
  P->n_B = prob->n_B;
  P->n_T = prob->n_T;
  P->n_K = prob->n_K;
  P->n_eps = prob->n_eps;
  P->n_S = prob->n_S;
  P->somo.assign(prob->is_somo, prob->is_somo + n_occ);
  auto destroy_fail = [&](dlpno_status st) {
    dlpno_plan_destroy(P);
    return st;
  };

  // ---- pairs ----
  int n_somo_total = 0;
  for (int k = 0; k < n_occ; ++k) n_somo_total += prob->is_somo[k];
  std::map<std::pair<int, int>, int> index;
  P->pairs_h.resize(npairs);
  int nblk_total = 0;
  for (int p = 0; p < npairs; ++p) {
    const dlpno_pair& d = prob->pairs[p];
    if (d.i < 0 || d.j < d.i || d.j >= n_occ)
      return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, "pair " + std::to_string(p) + ": need 0 <= i <= j < n_occ"));
    if (d.npno < 1 || d.npno > 64)
      return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, "pair " + std::to_string(p) + ": npno must be in 1..64"));
    if (d.naux < 1 || d.naux > 65536)
      return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, "pair " + std::to_string(p) + ": naux must be in 1..65536"));
    if (d.n_somo_virt < 0 || d.n_somo_virt >= d.npno || d.n_somo_virt > n_somo_total)
      return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, "pair " + std::to_string(p) +
                                                        ": n_somo_virt must be below npno and at most the SOMO count"));
    if (!index.emplace(std::make_pair(d.i, d.j), p).second)
      return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "pair " + std::to_string(p) + " duplicates an earlier pair"));
    const uint32_t want = rule_mask(d.i, d.j, prob->is_somo);
    if (d.blocks != want)
      return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "pair " + std::to_string(p) +
                                                          ": block mask does not follow the spin-case rule"));
    const int64_t n = d.npno, n2 = n * n, nb = popcount4(want);
    if (d.off_B < 0 || d.off_B + (int64_t)d.naux * n2 > prob->n_B || d.off_T < 0 || d.off_T + nb * n2 > prob->n_T ||
        d.off_K < 0 || d.off_K + n2 > prob->n_K || d.off_eps < 0 || d.off_eps + n > prob->n_eps)
      return destroy_fail(fail(DLPNO_ERR_ALIGNMENT, "pair " + std::to_string(p) + ": offsets exceed the buffers"));
    PairDev& pd = P->pairs_h[p];
    pd.i = d.i;
    pd.j = d.j;
    pd.n = d.npno;
    pd.m = d.naux;
    pd.nblk = (int)nb;
    pd.blk0 = nblk_total;
    pd.off_B = d.off_B;
    pd.off_T = d.off_T;
    pd.off_K = d.off_K;
    pd.off_eps = d.off_eps;
    nblk_total += (int)nb;
  }
  P->n_blocks = nblk_total;
  // ---- blocks ----
  P->blocks_h.resize(nblk_total);
  P->flops_ladder = 0.0;
  for (int p = 0; p < npairs; ++p) {
    const dlpno_pair& d = prob->pairs[p];
    const PairDev& pd = P->pairs_h[p];
    int slot = 0;
    for (int c = 0; c < 4; ++c) {
      if (!(d.blocks & kCodeBit[c])) continue;
      BlockDev& b = P->blocks_h[pd.blk0 + slot];
      b.pair = p;
      b.code = c;
      b.n = pd.n;
      b.s1 = kCodeS1[c];
      b.s2 = kCodeS2[c];
      b.anti = b.s1 == b.s2;
      b.off_T = pd.off_T + (int64_t)slot * pd.n * pd.n;
      b.off_K = pd.off_K;
      b.off_eps = pd.off_eps;
      const double* f1 = b.s1 == 0 ? prob->f_a : prob->f_b;
      const double* f2 = b.s2 == 0 ? prob->f_a : prob->f_b;
      b.fsum = f1[(size_t)d.i * n_occ + d.i] + f2[(size_t)d.j * n_occ + d.j];
      b.w = b.anti ? 0.5 : 1.0;
      b.rows = b.s1 == 0 ? pd.n - d.n_somo_virt : pd.n;
      b.cols = b.s2 == 0 ? pd.n - d.n_somo_virt : pd.n;
      if (d.n_somo_virt > 0) P->somo_virt = true;
      P->flops_ladder += 4.0 * pd.m * (double)pd.n * pd.n * pd.n;
      ++slot;
    }
  }
  // ---- occupied Fock symmetry (a precondition of the vector-Jacobian product) ----
  {
    double fmax = 0.0;
    for (size_t x = 0; x < (size_t)n_occ * n_occ; ++x) fmax = std::max(fmax, std::max(std::fabs(prob->f_a[x]), std::fabs(prob->f_b[x])));
    for (int a = 0; a < n_occ && P->fock_symmetric; ++a)
      for (int b = a + 1; b < n_occ; ++b) {
        const size_t ab = (size_t)a * n_occ + b, ba = (size_t)b * n_occ + a;
        if (std::fabs(prob->f_a[ab] - prob->f_a[ba]) > 1e-12 * fmax ||
            std::fabs(prob->f_b[ab] - prob->f_b[ba]) > 1e-12 * fmax) {
          P->fock_symmetric = false;
          P->vjp_reason = "the occupied Fock matrices are not symmetric (element " + std::to_string(a) + ", " +
                          std::to_string(b) + ")";
          break;
        }
      }
  }
  // ---- couplings and terms ----
  // One merged list per target pair: its occupied-Fock couplings, then its
  // hole-hole ladder couplings.  Both apply -w S_{p,q} X S_{p,q}^T to every
  // target block for which the ordered source (x, y) has a block; the
  // kernels do not distinguish them.
  const int64_t n_fock = prob->n_couplings, n_hh = prob->n_hh;
  if (n_hh < 0) return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, "n_hh must be >= 0"));
  if (n_hh > 0 && (!prob->hh_rowptr || !prob->hh))
    return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "hh_rowptr or hh is NULL with n_hh > 0"));
  std::vector<int64_t> frow(prob->cpl_rowptr, prob->cpl_rowptr + npairs + 1);
  std::vector<int64_t> hrow(npairs + 1, 0);
  if (n_hh > 0) hrow.assign(prob->hh_rowptr, prob->hh_rowptr + npairs + 1);
  if (frow[0] != 0 || frow[npairs] != n_fock)
    return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "cpl_rowptr must start at 0 and end at n_couplings"));
  if (hrow[0] != 0 || hrow[npairs] != n_hh)
    return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "hh_rowptr must start at 0 and end at n_hh"));
  for (int p = 0; p < npairs; ++p) {
    if (frow[p + 1] < frow[p]) return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "cpl_rowptr must be non-decreasing"));
    if (hrow[p + 1] < hrow[p]) return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "hh_rowptr must be non-decreasing"));
  }
  if (n_fock + n_hh > INT32_MAX) return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, "too many couplings"));
  const int64_t n_all = n_fock + n_hh;
  P->n_cpl = n_all;
  P->n_hh = n_hh;
  P->rowptr_h.assign(npairs + 1, 0);
  for (int p = 0; p <= npairs; ++p) P->rowptr_h[p] = frow[p] + hrow[p];
  P->cpl_h.resize(n_all);
  P->cpl_k_h.resize(n_all);
  P->cpl_side_h.resize(n_all);
  P->cpl_l_h.resize(n_all);
  P->terms_h.assign((size_t)n_all * 4, TermDev{-1, 0.0, 0, -1});
  P->flops_proj = 0.0;
  P->n_terms = 0;
  for (int p = 0; p < npairs; ++p) {
    const dlpno_pair& d = prob->pairs[p];
    const PairDev& pd = P->pairs_h[p];
    int64_t out = P->rowptr_h[p];
    // the term of merged coupling `e` (source pair q, ordered source (x, y)
    // with electron spins (s1, s2)) on target block slot `slot`, weight w
    auto add_term = [&](int64_t e, int slot, const dlpno_pair& q, int src_pair, int x, int y, int s1, int s2,
                        double w, bool is_hh) {
      int scode, trans;
      if (x == y) {
        if (s1 == s2) return;                               // Pauli
        scode = 2;
        trans = s1 == 1;
      } else if (x < y) {
        scode = block_code(s1, s2);
        trans = 0;
      } else {
        scode = block_code(s2, s1);
        trans = 1;
      }
      // zero weights are kept where a T-dependent part is added to them
      if (!(q.blocks & kCodeBit[scode]) || (w == 0.0 && !(quad && is_hh) && !(qocc && !is_hh))) return;
      int sslot = 0;
      for (int cc = 0; cc < scode; ++cc)
        if (q.blocks & kCodeBit[cc]) ++sslot;
      const int64_t nq = q.npno;
      TermDev& tm = P->terms_h[(size_t)e * 4 + slot];
      tm.src_off = q.off_T + (int64_t)sslot * nq * nq;
      tm.w = w;
      tm.trans = trans;
      tm.src_blk = P->pairs_h[src_pair].blk0 + sslot;
      P->flops_proj += 2.0 * pd.n * (double)nq * (pd.n + nq);
      ++P->n_terms;
    };
    for (int64_t fe = frow[p]; fe < frow[p + 1]; ++fe, ++out) {
      const dlpno_coupling& c = prob->cpl[fe];
      const std::string where = "coupling " + std::to_string(fe) + " of pair " + std::to_string(p);
      if (c.src_pair < 0 || c.src_pair >= npairs || c.k < 0 || c.k >= n_occ || (c.side != 0 && c.side != 1))
        return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, where + ": src_pair, k or side out of range"));
      const int rep = c.side == 0 ? d.i : d.j, keep = c.side == 0 ? d.j : d.i;
      if (c.k == rep) return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, where + ": k equals the replaced index"));
      const dlpno_pair& q = prob->pairs[c.src_pair];
      if (q.i != std::min(c.k, keep) || q.j != std::max(c.k, keep))
        return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, where + ": source pair does not match (k, side)"));
      if (c.off_S < 0 || c.off_S + (int64_t)q.npno * d.npno > prob->n_S)
        return destroy_fail(fail(DLPNO_ERR_ALIGNMENT, where + ": off_S exceeds the S buffer"));
      CplDev& cd = P->cpl_h[out];
      cd.src = c.src_pair;
      cd.nsrc = q.npno;
      cd.off_S = c.off_S;
      P->cpl_k_h[out] = c.k;
      P->cpl_side_h[out] = c.side;
      P->cpl_l_h[out] = -1;
      // k replaces electron i (side 0) or j (side 1); weight f^s[k][replaced]
      // of the replaced electron's spin s, which needs k occupied in s
      int slot = 0;
      for (int code = 0; code < 4; ++code) {
        if (!(d.blocks & kCodeBit[code])) continue;
        const int s1 = kCodeS1[code], s2 = kCodeS2[code];
        const int sk = c.side == 0 ? s1 : s2;
        const int this_slot = slot++;
        if (sk == 1 && prob->is_somo[c.k]) continue;
        const double* f = sk == 0 ? prob->f_a : prob->f_b;
        const int x = c.side == 0 ? c.k : d.i, y = c.side == 0 ? d.j : c.k;
        add_term(out, this_slot, q, c.src_pair, x, y, s1, s2, f[(size_t)c.k * n_occ + rep], false);
      }
    }
    for (int64_t he = hrow[p]; he < hrow[p + 1]; ++he, ++out) {
      const dlpno_hh_coupling& c = prob->hh[he];
      const std::string where = "hole-hole coupling " + std::to_string(he) + " of pair " + std::to_string(p);
      if (c.src_pair < 0 || c.src_pair >= npairs || c.k < 0 || c.k >= n_occ || c.l < 0 || c.l >= n_occ)
        return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, where + ": src_pair, k or l out of range"));
      const dlpno_pair& q = prob->pairs[c.src_pair];
      if (q.i != std::min(c.k, c.l) || q.j != std::max(c.k, c.l))
        return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, where + ": source pair does not match (k, l)"));
      if (!std::isfinite(c.w)) return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, where + ": weight is not finite"));
      if (c.off_S < 0 || c.off_S + (int64_t)q.npno * d.npno > prob->n_S)
        return destroy_fail(fail(DLPNO_ERR_ALIGNMENT, where + ": off_S exceeds the S buffer"));
      CplDev& cd = P->cpl_h[out];
      cd.src = c.src_pair;
      cd.nsrc = q.npno;
      cd.off_S = c.off_S;
      P->cpl_k_h[out] = c.k;
      P->cpl_side_h[out] = 2;
      P->cpl_l_h[out] = c.l;
      // ordered source (k, l) for spins (s1, s2): k in occ_s1, l in occ_s2;
      // the residual gets +w S T S^T (the kernels apply -weight)
      int slot = 0;
      for (int code = 0; code < 4; ++code) {
        if (!(d.blocks & kCodeBit[code])) continue;
        const int s1 = kCodeS1[code], s2 = kCodeS2[code];
        const int this_slot = slot++;
        if ((s1 == 1 && prob->is_somo[c.k]) || (s2 == 1 && prob->is_somo[c.l])) continue;
        add_term(out, this_slot, q, c.src_pair, c.k, c.l, s1, s2, -c.w, true);
      }
    }
  }
  // device tables: within each target row, couplings ordered by the tile
  // count of the source pair (stable), so projection items are homogeneous
  for (int p = 0; p < npairs; ++p) {
    const int64_t e0 = P->rowptr_h[p], e1 = P->rowptr_h[p + 1];
    std::vector<int64_t> ord;
    for (int64_t e = e0; e < e1; ++e) ord.push_back(e);
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
      return (P->cpl_h[x].nsrc + 15) / 16 < (P->cpl_h[y].nsrc + 15) / 16;
    });
    std::vector<CplDev> c2;
    std::vector<TermDev> t2;
    std::vector<int32_t> k2, s2, l2;
    for (int64_t e : ord) {
      c2.push_back(P->cpl_h[e]);
      k2.push_back(P->cpl_k_h[e]);
      s2.push_back(P->cpl_side_h[e]);
      l2.push_back(P->cpl_l_h[e]);
      for (int b = 0; b < 4; ++b) t2.push_back(P->terms_h[(size_t)e * 4 + b]);
    }
    for (int64_t k = 0; k < (int64_t)ord.size(); ++k) {
      P->cpl_h[e0 + k] = c2[k];
      P->cpl_k_h[e0 + k] = k2[k];
      P->cpl_side_h[e0 + k] = s2[k];
      P->cpl_l_h[e0 + k] = l2[k];
      for (int b = 0; b < 4; ++b) P->terms_h[(size_t)(e0 + k) * 4 + b] = t2[(size_t)k * 4 + b];
    }
  }
  // ---- quadratic term: the hole-hole couplings' T-dependent weights ----
  if (quad) {
    for (int p = 0; p < npairs; ++p) {
      const PairDev& pd = P->pairs_h[p];
      const dlpno_pair& d = prob->pairs[p];
      for (int64_t e = P->rowptr_h[p]; e < P->rowptr_h[p + 1]; ++e) {
        if (P->cpl_side_h[e] != 2) continue;
        QuadCpl qc{};
        qc.off_S = P->cpl_h[e].off_S;
        qc.off_K = prob->pairs[P->cpl_h[e].src].off_K;
        qc.np = pd.n;
        qc.nq = P->cpl_h[e].nsrc;
        qc.transK = P->cpl_k_h[e] > P->cpl_l_h[e];
        qc.off_G = P->n_quadG;
        int slot = 0;
        for (int code = 0; code < 4; ++code) {
          if (!(d.blocks & kCodeBit[code])) continue;
          const int this_slot = slot++;
          const TermDev& tm = P->terms_h[(size_t)e * 4 + this_slot];
          if (tm.src_off < 0) continue;
          const int b = qc.nblk++;
          qc.term[b] = e * 4 + this_slot;
          qc.off_T[b] = pd.off_T + (int64_t)this_slot * pd.n * pd.n;
          qc.w0[b] = tm.w;
          qc.c[b] = kCodeS1[code] == kCodeS2[code] ? -0.5 : -1.0;
          P->flops_quad += 2.0 * pd.n * (double)pd.n;
        }
        if (qc.nblk > 0) {
          P->quad_h.push_back(qc);
          P->n_quadG += (int64_t)pd.n * pd.n;
          P->flops_quad_prep += 2.0 * pd.n * (double)qc.nq * (pd.n + qc.nq);
        }
      }
    }
  }
  // ---- quadratic part of the occupied Fock intermediate ----
  // F^s_mj = sum_{n, s_n} <G_(m,n), T^{s s_n}_(j,n)>, G[e][f] = (m e|n f) over
  // the PNOs of the dotted pair {j, n}: S K_(m,n) S^T through a listed Fock
  // coupling of {j, n} with m replacing j, or K_(j,n) itself for m = j.  It
  // dresses the Fock weights f^s_kj of the listed projection terms and adds
  // -(F^s1_ii + F^s2_jj) T per block.
  P->qocc = qocc;
  std::vector<QuadCpl> occ_prep;   // factors S K S^T built once (the prepare kernel of the quadratic term)
  std::vector<int64_t> occ_tr_off;  // factors stored transposed (their dots then read T row by row)
  std::vector<int32_t> occ_tr_n;
  if (qocc) {
    std::map<std::tuple<int, int, int>, int32_t> keyid;
    auto key_add = [&](int m, int j, int sp) -> int32_t {
      const auto key = std::make_tuple(m, j, sp);
      auto it = keyid.find(key);
      if (it != keyid.end()) return it->second;
      const int32_t id = (int32_t)keyid.size();
      keyid.emplace(key, id);
      return id;
    };
    auto key_find = [&](int m, int j, int sp) -> int32_t {
      auto it = keyid.find(std::make_tuple(m, j, sp));
      return it == keyid.end() ? -1 : it->second;
    };
    P->occ_blk_key_h.assign(2 * (size_t)nblk_total, -1);
    for (int p = 0; p < npairs; ++p) {
      const dlpno_pair& d = prob->pairs[p];
      const PairDev& pd = P->pairs_h[p];
      for (int64_t e = P->rowptr_h[p]; e < P->rowptr_h[p + 1]; ++e) {
        const int side = P->cpl_side_h[e];
        if (side == 2) continue;                           // hole-hole couplings are not dressed
        const int k = P->cpl_k_h[e], rep = side == 0 ? d.i : d.j;
        int slot = 0;
        for (int code = 0; code < 4; ++code) {
          if (!(d.blocks & kCodeBit[code])) continue;
          const int this_slot = slot++;
          const TermDev& tm = P->terms_h[(size_t)e * 4 + this_slot];
          if (tm.src_off < 0) continue;
          const int sp = side == 0 ? kCodeS1[code] : kCodeS2[code];
          P->occ_terms_h.push_back(OccTerm{e * 4 + this_slot, key_add(k, rep, sp), 0, tm.w});
        }
      }
      int slot = 0;
      for (int code = 0; code < 4; ++code) {
        if (!(d.blocks & kCodeBit[code])) continue;
        const int b = pd.blk0 + slot++;
        P->occ_blk_key_h[2 * (size_t)b] = key_add(d.i, d.i, kCodeS1[code]);
        P->occ_blk_key_h[2 * (size_t)b + 1] = key_add(d.j, d.j, kCodeS2[code]);
      }
    }
    std::vector<std::vector<int64_t>> per_key(keyid.size());
    for (int q = 0; q < npairs; ++q) {
      const dlpno_pair& d = prob->pairs[q];
      const int64_t nq = d.npno, nn = nq * nq;
      // one contribution: F^s_(m, j) += <G, T_(j,n)> (G from K of q when from_K)
      auto add = [&](int m, int j, int n, int from_K, int64_t off_G, int trG, const QuadCpl* prep) {
        OccCtb c{};
        c.n = (int32_t)nq;
        c.from_K = from_K;
        c.off_G = off_G;
        bool any = false;
        for (int sp = 0; sp < 2; ++sp) {
          c.key[sp] = key_find(m, j, sp);
          int nb = 0;
          c.off_T[sp][0] = c.off_T[sp][1] = -1;
          c.tr[sp][0] = c.tr[sp][1] = 0;
          if (c.key[sp] < 0) continue;
          for (int sn = 0; sn < 2; ++sn) {
            int code, trT;
            if (d.i == d.j) {
              if (sp == sn) continue;
              code = 2;
              trT = sp == 1;
            } else if (j == d.i) {
              code = block_code(sp, sn);
              trT = 0;
            } else {
              code = block_code(sn, sp);
              trT = 1;
            }
            if (!(d.blocks & kCodeBit[code])) continue;
            int sslot = 0;
            for (int cc = 0; cc < code; ++cc)
              if (d.blocks & kCodeBit[cc]) ++sslot;
            c.off_T[sp][nb] = d.off_T + (int64_t)sslot * nn;
            c.tr[sp][nb] = trT ^ trG;
            ++nb;
            P->flops_occ += 2.0 * (double)nn;
          }
          if (nb > 0) any = true;
        }
        if (!any) return;
        if (prep) {
          QuadCpl qc = *prep;
          qc.off_G = P->n_occG;
          c.off_G = P->n_occG;
          if (trG) {
            occ_tr_off.push_back(P->n_occG);
            occ_tr_n.push_back((int32_t)nq);
          }
          P->n_occG += nn;
          occ_prep.push_back(qc);
          P->flops_occ_prep += 2.0 * nq * (double)qc.nq * (nq + qc.nq);
        }
        const int64_t ci = (int64_t)P->occ_ctb_h.size();
        for (int sp = 0; sp < 2; ++sp)
          if (c.key[sp] >= 0 && c.off_T[sp][0] >= 0) per_key[c.key[sp]].push_back(2 * ci + sp);
        P->occ_ctb_h.push_back(c);
      };
      // m = j: K of the pair itself, (j e|n f) = K_q (j = i) or K_q^T (j = j)
      add(d.i, d.i, d.j, 1, d.off_K, 0, nullptr);
      if (d.j != d.i) add(d.j, d.j, d.i, 1, d.off_K, 1, nullptr);
      // m != j: the listed Fock couplings of q, m replacing j, n kept (a
      // diagonal pair lists each source once per side: it is dotted once)
      for (int64_t e = P->rowptr_h[q]; e < P->rowptr_h[q + 1]; ++e) {
        const int side = P->cpl_side_h[e];
        if (side == 2 || (side == 1 && d.i == d.j)) continue;
        const int m = P->cpl_k_h[e], j = side == 0 ? d.i : d.j, n = side == 0 ? d.j : d.i;
        const int r = P->cpl_h[e].src;
        QuadCpl qc{};
        qc.off_S = P->cpl_h[e].off_S;
        qc.off_K = prob->pairs[r].off_K;
        qc.np = (int32_t)nq;
        qc.nq = P->cpl_h[e].nsrc;
        qc.transK = m > n;
        // for j the pair's second index every block of the dot enters
        // transposed: the factor is stored transposed instead, so that the
        // dots read both operands in the same order
        add(m, j, n, 0, 0, (j == d.j && d.i != d.j) ? 1 : 0, &qc);
      }
    }
    P->occ_key_rowptr_h.assign(per_key.size() + 1, 0);
    for (size_t k = 0; k < per_key.size(); ++k) {
      P->occ_key_rowptr_h[k + 1] = P->occ_key_rowptr_h[k] + (int64_t)per_key[k].size();
      P->occ_key_src_h.insert(P->occ_key_src_h.end(), per_key[k].begin(), per_key[k].end());
    }
  }
  // ---- ring/exchange term ----
  // P(IJ) P(AB) sum_ME t_IM^AE <MB||EJ>: per target block (spins s1, s2 of
  // electrons i, j), role (X, Y) = (i s1, j s2) with sign +1 or (j s2, i s1)
  // with sign -1, orientation (virtual spins (ra, cb) = (s1, s2), added as is,
  // or (s2, s1), added transposed with sign -1) and spin sm of M:
  //   (m e | c y) when cb is the spin of Y, e of spin sm;
  //  -(m y | c e) when sm is the spin of Y, e of spin cb;
  // each with the amplitude t_{X M}^{r e} of the source pair {x, m}: its
  // stored block when (ra, e-spin) are the spins of (X, M), minus its
  // transpose when they are swapped.
  P->n_ring = prob->n_ring;
  P->rx_block.assign(nblk_total, 0);
  if (prob->n_ring > 0) {
    std::vector<int64_t> rrow(prob->ring_rowptr, prob->ring_rowptr + npairs + 1);
    if (rrow[0] != 0 || rrow[npairs] != prob->n_ring)
      return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "ring_rowptr must start at 0 and end at n_ring"));
    for (int p = 0; p < npairs; ++p)
      if (rrow[p + 1] < rrow[p]) return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, "ring_rowptr must be non-decreasing"));
    for (int p = 0; p < npairs; ++p) {
      const dlpno_pair& d = prob->pairs[p];
      const PairDev& pd = P->pairs_h[p];
      std::vector<std::vector<RxTerm>> per_slot(pd.nblk);
      for (int64_t re = rrow[p]; re < rrow[p + 1]; ++re) {
        const dlpno_ring_coupling& c = prob->ring[re];
        const std::string where = "ring coupling " + std::to_string(re) + " of pair " + std::to_string(p);
        if (c.src_pair < 0 || c.src_pair >= npairs || c.m < 0 || c.m >= n_occ || (c.role != 0 && c.role != 1))
          return destroy_fail(fail(DLPNO_ERR_DIM_RANGE, where + ": src_pair, m or role out of range"));
        if (d.i == d.j && c.role != 0)
          return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, where + ": a diagonal target lists role 0 only"));
        const int xr = c.role == 0 ? d.i : d.j;
        const dlpno_pair& q = prob->pairs[c.src_pair];
        if (q.i != std::min(xr, c.m) || q.j != std::max(xr, c.m))
          return destroy_fail(fail(DLPNO_ERR_INVALID_ARG, where + ": source pair does not match (role, m)"));
        const int64_t blk = (int64_t)q.npno * d.npno;
        if (c.off_S < 0 || c.off_S + blk > prob->n_S)
          return destroy_fail(fail(DLPNO_ERR_ALIGNMENT, where + ": off_S exceeds the S buffer"));
        if (c.off_X < 0 || c.off_X + blk > prob->n_ring_ints || c.off_J < 0 || c.off_J + blk > prob->n_ring_ints)
          return destroy_fail(fail(DLPNO_ERR_ALIGNMENT, where + ": off_X or off_J exceeds the ring integral buffer"));
        const int64_t nq = q.npno;
        // stored block of the ordered source (x sx, m sm): slot and transpose, or -1
        auto lookup = [&](int x, int sx, int sm, int& trans) -> int {
          int scode;
          if (x == c.m) {
            if (sx == sm) return -1;
            scode = 2;
            trans = sx == 1;
          } else if (x < c.m) {
            scode = block_code(sx, sm);
            trans = 0;
          } else {
            scode = block_code(sm, sx);
            trans = 1;
          }
          if (!(q.blocks & kCodeBit[scode])) return -1;
          int sslot = 0;
          for (int cc = 0; cc < scode; ++cc)
            if (q.blocks & kCodeBit[cc]) ++sslot;
          return sslot;
        };
        int slot = 0;
        for (int code = 0; code < 4; ++code) {
          if (!(d.blocks & kCodeBit[code])) continue;
          const int this_slot = slot++;
          const int s1 = kCodeS1[code], s2 = kCodeS2[code];
          for (int role = 0; role < 2; ++role) {
            if (d.i != d.j && role != c.role) continue;      // a diagonal target applies each coupling twice
            const int x = role == 0 ? d.i : d.j, sx = role == 0 ? s1 : s2, sy = role == 0 ? s2 : s1;
            for (int orient = 0; orient < 2; ++orient) {
              const int ra = orient == 0 ? s1 : s2, cb = orient == 0 ? s2 : s1;
              const double sgn = (role == 0 ? 1.0 : -1.0) * (orient == 0 ? 1.0 : -1.0);
              for (int sm = 0; sm < 2; ++sm) {
                if (sm == 1 && prob->is_somo[c.m]) continue;   // M occupied: SOMOs are alpha only
                for (int part = 0; part < 2; ++part) {       // 0: X = (m e|c y), 1: J = (m y|c e)
                  const int se = part == 0 ? sm : cb;
                  if (part == 0 ? cb != sy : sm != sy) continue;
                  int trans = 0;
                  double asign;
                  int sslot;
                  if (sx == ra && sm == se) {
                    sslot = lookup(x, sx, sm, trans);
                    asign = 1.0;
                  } else if (sx == se && sm == ra) {
                    sslot = lookup(x, sx, sm, trans);
                    trans ^= 1;
                    asign = -1.0;
                  } else {
                    continue;
                  }
                  if (sslot < 0) continue;
                  RxTerm t{};
                  t.src_off = q.off_T + (int64_t)sslot * nq * nq;
                  t.nq = (int32_t)nq;
                  t.w = sgn * asign * (part == 0 ? 1.0 : -1.0);
                  const int64_t off_W = part == 0 ? c.off_X : c.off_J;
                  // orientation 0: S^T op(T) W;  1: (S^T op(T) W)^T = W^T op(T)^T S
                  if (orient == 0) {
                    t.off_L = c.off_S;
                    t.off_M = off_W;
                    t.flags = kRxM | (trans ? kRxTrans : 0);
                  } else {
                    t.off_L = off_W;
                    t.off_M = c.off_S;
                    t.flags = kRxL | (trans ? 0 : kRxTrans);
                  }
                  per_slot[this_slot].push_back(t);
                  P->flops_rx += 2.0 * pd.n * (double)nq * (nq + pd.n);
                }
              }
            }
          }
        }
      }
      for (int b = 0; b < pd.nblk; ++b) {
        if (per_slot[b].empty()) continue;
        RxUnit u{};
        u.blk = pd.blk0 + b;
        u.t0 = (int64_t)P->rx_terms_h.size();
        P->rx_terms_h.insert(P->rx_terms_h.end(), per_slot[b].begin(), per_slot[b].end());
        u.t1 = (int64_t)P->rx_terms_h.size();
        P->rx_units_h.push_back(u);
        P->rx_block[pd.blk0 + b] = 1;
      }
    }
  }
  // ---- device ----
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  P->device = dev;
  {
    const dlpno_status sst = scratch_init(dev);
    if (sst != DLPNO_OK) return destroy_fail(sst);
  }
  hipDeviceProp_t prop;
  HIPCK(hipGetDeviceProperties(&prop, dev));
  P->num_cu = prop.multiProcessorCount;
  P->arch = prop.gcnArchName;
  P->workers = opt.n_workers > 0 ? opt.n_workers : P->num_cu;
  if (opt.items_per_wave > 0) P->tune.items_per_wave = (double)opt.items_per_wave;
  // FP64 defaults: two-tile pairs take two blocks per item, so that they run
  // in the two-wave ladder launch (the four-block variant's X operands do not
  // fit its LDS slab); four-tile pairs take cooperative items of two blocks
  if (opt.precision == DLPNO_FP64) {
    P->tune.ladder_variant[1] = 4;
    P->tune.ladder_variant[3] = kLadderCoopPair;
  }
  // split defaults: three- and four-tile pairs take two blocks per item
  if (is_split(opt.precision)) {
    P->tune.ladder_variant[2] = 11;
    P->tune.ladder_variant[3] = 12;
  }
  dlpno_status st;
  if ((st = build_schedule(P)) != DLPNO_OK) return destroy_fail(st);
  if ((st = upload(&P->d_pairs, P->pairs_h, "pair table", s)) != DLPNO_OK) return destroy_fail(st);
  if ((st = upload(&P->d_cpl, P->cpl_h, "coupling table", s)) != DLPNO_OK) return destroy_fail(st);
  if ((st = upload(&P->d_terms, P->terms_h, "term table", s)) != DLPNO_OK) return destroy_fail(st);
  if (!P->quad_h.empty()) {
    if ((st = upload(&P->d_quad, P->quad_h, "quadratic-term table", s)) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->d_quadG, P->n_quadG, "quadratic-term factors")) != DLPNO_OK) return destroy_fail(st);
    if (launch_quad_prepare(P->d_quad, (int64_t)P->quad_h.size(), P->in.S, P->in.K, P->d_quadG, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return destroy_fail(fail(DLPNO_ERR_HIP, "quadratic-term factors"));
  }
  if (P->qocc) {
    if ((st = upload(&P->d_occ_ctb, P->occ_ctb_h, "occupied-intermediate contributions", s)) != DLPNO_OK ||
        (st = upload(&P->d_occ_terms, P->occ_terms_h, "occupied-intermediate terms", s)) != DLPNO_OK ||
        (st = upload(&P->d_occ_blk_key, P->occ_blk_key_h, "occupied-intermediate block keys", s)) != DLPNO_OK ||
        (st = upload(&P->d_occ_key_rowptr, P->occ_key_rowptr_h, "occupied-intermediate keys", s)) != DLPNO_OK ||
        (st = upload(&P->d_occ_key_src, P->occ_key_src_h, "occupied-intermediate keys", s)) != DLPNO_OK ||
        (st = dev_alloc(&P->d_occ_dots, std::max<size_t>(2 * P->occ_ctb_h.size(), 1), "occupied-intermediate dots")) !=
            DLPNO_OK ||
        (st = dev_alloc(&P->d_occF, std::max<size_t>(P->occ_key_rowptr_h.size(), 1), "occupied intermediate")) !=
            DLPNO_OK ||
        (st = dev_alloc(&P->d_occ_shift, std::max(nblk_total, 1), "occupied-intermediate shifts")) != DLPNO_OK ||
        (st = dev_alloc(&P->d_occG, (size_t)std::max<int64_t>(P->n_occG, 1), "occupied-intermediate factors")) !=
            DLPNO_OK)
      return destroy_fail(st);
    // the shift is read by every finish; until a residual has formed it, zero
    HIPCK(launch_fill(P->d_occ_shift, 0.0, std::max(nblk_total, 1), s));
    if (!occ_prep.empty()) {
      QuadCpl* d_prep = nullptr;
      if ((st = upload(&d_prep, occ_prep, "occupied-intermediate factor list", s)) != DLPNO_OK) return destroy_fail(st);
      const hipError_t pe = launch_quad_prepare(d_prep, (int64_t)occ_prep.size(), P->in.S, P->in.K, P->d_occG, s);
      int64_t* d_toff = nullptr;
      int32_t* d_tn = nullptr;
      hipError_t te = hipSuccess;
      if (pe == hipSuccess && !occ_tr_off.empty()) {
        if ((st = upload(&d_toff, occ_tr_off, "factor transposes", s)) != DLPNO_OK ||
            (st = upload(&d_tn, occ_tr_n, "factor transposes", s)) != DLPNO_OK) {
          (void)hipFree(d_prep);
          (void)hipFree(d_toff);
          return destroy_fail(st);
        }
        te = launch_transpose_blocks(d_toff, d_tn, (int64_t)occ_tr_off.size(), P->d_occG, s);
      }
      const hipError_t se = hipStreamSynchronize(s);
      (void)hipFree(d_prep);
      (void)hipFree(d_toff);
      (void)hipFree(d_tn);
      if (pe != hipSuccess || te != hipSuccess || se != hipSuccess)
        return destroy_fail(fail(DLPNO_ERR_HIP, "occupied-intermediate factors"));
    }
  }
  if (!P->rx_units_h.empty()) {
    if ((st = upload(&P->d_rx_terms, P->rx_terms_h, "ring term table", s)) != DLPNO_OK) return destroy_fail(st);
    if ((st = upload(&P->d_rx_units, P->rx_units_h, "ring unit table", s)) != DLPNO_OK) return destroy_fail(st);
  }
  if ((st = upload_schedule(P, s)) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_counter, kKinds * kQueues, "queue heads")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_e_block, std::max(1, nblk_total), "block energies")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_f12_block, std::max(1, nblk_total), "F12 block energies")) != DLPNO_OK)
    return destroy_fail(st);
  if ((st = dev_alloc(&P->d_red_partial, 2 * kReduceParts, "reduction scratch")) != DLPNO_OK)
    return destroy_fail(st);
  if ((st = dev_alloc(&P->d_rmax_block, std::max(1, nblk_total), "block residual maxima")) != DLPNO_OK)
    return destroy_fail(st);
  if ((st = dev_alloc(&P->d_nonfinite, 4, "non-finite flag")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_flagz, 1, "zero-amplitude flag")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_hist_iter, 4, "history counter")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_hist, 2 * kHistCap, "history")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_diis, 1, "DIIS state")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_scalars, 8, "scalars")) != DLPNO_OK) return destroy_fail(st);
  if ((st = dev_alloc(&P->d_diis_partial, (size_t)kDiisParts * 8, "DIIS partial sums")) != DLPNO_OK)
    return destroy_fail(st);
  if (opt.diis_max > 0 && P->n_T > 0) {
    if ((st = dev_alloc(&P->d_ring_vecs, (size_t)opt.diis_max * P->n_T, "DIIS vectors")) != DLPNO_OK)
      return destroy_fail(st);
    if ((st = dev_alloc(&P->d_ring_errs, (size_t)opt.diis_max * P->n_T, "DIIS errors")) != DLPNO_OK)
      return destroy_fail(st);
  }
  HIPCK(launch_zero_i32(P->d_nonfinite, 1, s));
  HIPCK(launch_zero_i32(P->d_hist_iter, 1, s));
  HIPCK(launch_diis_reset(P->d_diis, std::max(1, opt.diis_max), std::max(1, opt.diis_start), s));
  if (opt.precision == DLPNO_FP32) {
    if ((st = dev_alloc(&P->B32, (size_t)std::max<int64_t>(P->n_B, 1), "FP32 B")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->S32, (size_t)std::max<int64_t>(P->n_S, 1), "FP32 S")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->T32, (size_t)std::max<int64_t>(P->n_T, 1), "FP32 T")) != DLPNO_OK) return destroy_fail(st);
    if (P->n_B > 0) HIPCK(launch_convert_f32(in->B, P->B32, P->n_B, s));
    if (P->n_S > 0) HIPCK(launch_convert_f32(in->S, P->S32, P->n_S, s));
  }
  if (is_split(opt.precision)) {
    const bool f16 = opt.precision == DLPNO_FP16X2;
    std::vector<int64_t> boff(npairs), toff(nblk_total), soff(P->n_cpl), ctgt(P->n_cpl);
    int64_t nb = 0, nt = 0, ns = 0;
    for (int p = 0; p < npairs; ++p) {
      const PairDev& pd = P->pairs_h[p];
      const int64_t n16 = 16 * ((pd.n + 15) / 16);
      boff[p] = nb;
      if (pd.nblk > 0) nb += (int64_t)pd.m * pd.n * n16;
      for (int b = 0; b < pd.nblk; ++b) {
        toff[pd.blk0 + b] = nt;
        nt += (int64_t)pd.n * n16;
      }
      for (int64_t e = P->rowptr_h[p]; e < P->rowptr_h[p + 1]; ++e) {
        ctgt[e] = p;
        soff[e] = ns;
        ns += (int64_t)pd.n * 16 * ((P->cpl_h[e].nsrc + 15) / 16);
      }
    }
    P->n_Bs = nb;
    P->n_Ts = nt;
    P->n_Ss = ns;
    if ((st = upload(&P->d_pair_boff, boff, "split B offsets", s)) != DLPNO_OK) return destroy_fail(st);
    if ((st = upload(&P->d_blk_toff, toff, "split T offsets", s)) != DLPNO_OK) return destroy_fail(st);
    if ((st = upload(&P->d_cpl_soff, soff, "split S offsets", s)) != DLPNO_OK) return destroy_fail(st);
    if ((st = upload(&P->d_cpl_target, ctgt, "coupling targets", s)) != DLPNO_OK) return destroy_fail(st);
    const size_t one = 1;
    if ((st = dev_alloc(&P->Bs_hi, std::max<size_t>(nb, one), "split B")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->Bs_lo, std::max<size_t>(nb, one), "split B")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->Ss_hi, std::max<size_t>(ns, one), "split S")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->Ss_lo, std::max<size_t>(ns, one), "split S")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->Tts_hi, std::max<size_t>(nt, one), "split T")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->Tts_lo, std::max<size_t>(nt, one), "split T")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->Ts_hi, std::max<size_t>(nt, one), "split T")) != DLPNO_OK) return destroy_fail(st);
    if ((st = dev_alloc(&P->Ts_lo, std::max<size_t>(nt, one), "split T")) != DLPNO_OK) return destroy_fail(st);
    if (f16) {
      if ((st = dev_alloc(&P->d_pair_bscale, std::max(npairs, 1), "B scales")) != DLPNO_OK) return destroy_fail(st);
      if ((st = dev_alloc(&P->d_blk_tscale, std::max(nblk_total, 1), "T scales")) != DLPNO_OK) return destroy_fail(st);
    }
    HIPCK(launch_split_B(P->d_pairs, npairs, in->B, P->d_pair_boff, P->d_pair_bscale, P->Bs_hi, P->Bs_lo, f16, s));
    HIPCK(launch_split_S(P->d_pairs, P->d_cpl_target, P->d_cpl, in->S, P->d_cpl_soff, P->n_cpl, P->Ss_hi,
                         P->Ss_lo, f16, s));
  }
  HIPCK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  HIPCK(hipStreamSynchronize(s));
  P->info = describe(P);
  *out = P;
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_plan_destroy(dlpno_plan* P) {
  if (!P) return DLPNO_OK;
  (void)hipDeviceSynchronize();
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  for (auto& ev : P->events) (void)hipEventDestroy(ev);
  void* ptrs[] = {P->d_pairs, P->d_blocks, P->d_cpl, P->d_terms, P->sched.d_items, P->sched64.d_items, P->d_counter, P->d_ws,
                  P->d_e_block, P->d_f12_block, P->d_red_partial, P->d_rmax_block, P->d_nonfinite, P->d_hist, P->d_diis, P->d_scalars,
                  P->d_diis_partial, P->d_ring_vecs, P->d_ring_errs, P->B32, P->S32, P->T32,
                  P->d_vjp_items, P->d_mixed, P->G32, P->d_pair_boff, P->d_blk_toff, P->d_cpl_soff,
                  P->d_cpl_target, P->d_pair_bscale, P->d_blk_tscale, P->Bs_hi, P->Bs_lo, P->Ss_hi, P->Ss_lo,
                  P->Tts_hi, P->Tts_lo, P->Ts_hi, P->Ts_lo, P->d_mix_r, P->d_mix_delta, P->d_hist_iter, P->d_quad,
                  P->d_quadG, P->d_flagz, P->d_rx_terms, P->d_rx_units, P->d_occ_ctb, P->d_occ_terms,
                  P->d_occ_blk_key, P->d_occ_key_rowptr, P->d_occ_key_src, P->d_occG, P->d_occ_dots, P->d_occF,
                  P->d_occ_shift};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete P;
  return DLPNO_OK;
}

// ---------------------------------------------------------------------------
// phases
// ---------------------------------------------------------------------------
namespace dlpno {

void phase_begin(dlpno_plan* P, int ph, hipStream_t s) {
  if (!P->profiling) return;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  (void)hipEventRecord(a, s);
  P->pending.push_back({ph, a, b});
}
void phase_end(dlpno_plan* P, hipStream_t s) {
  if (!P->profiling || P->pending.empty()) return;
  (void)hipEventRecord(P->pending.back().stop, s);
}
void phase_collect(dlpno_plan* P) {
  for (auto& pe : P->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pe.stop) == hipSuccess && hipEventElapsedTime(&ms, pe.start, pe.stop) == hipSuccess) {
      P->phase_ms[pe.phase] += ms;
      P->phase_n[pe.phase] += 1;
    }
    (void)hipEventDestroy(pe.start);
    (void)hipEventDestroy(pe.stop);
  }
  P->pending.clear();
}

bool is_split(int prec) { return prec == DLPNO_BF16X2 || prec == DLPNO_FP16X2; }

// Waits for the stream and turns the device status word into a status.
dlpno_status read_status(dlpno_plan* P, hipStream_t s) {
  int32_t flag = 0;
  HIPCK(hipMemcpyAsync(&flag, P->d_nonfinite, sizeof flag, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (flag & kErrNoBody) return fail(DLPNO_ERR_HIP, "a work item had no compiled kernel body");
  if (flag & kErrNonfinite) return fail(DLPNO_ERR_NONFINITE, "a residual element was not finite");
  return DLPNO_OK;
}

// the work queues of one kind's launch
WorkQueues queues(const dlpno_plan* P, const Schedule& S, int kind) {
  WorkQueues q{};
  for (int k = 0; k <= kQueues; ++k) q.off[k] = S.qoff[kind][k];
  q.counter = P->d_counter + kind * kQueues;
  return q;
}

// grouped kernel over amplitudes T (FP64 buffer given by the caller) in the
// plan's precision, or in `prec` when given (FP64 residuals of a split plan)
hipError_t run_grouped(dlpno_plan* P, const double* T, hipStream_t s, int prec, bool general, double* ws,
                       bool weights) {
  hipError_t e;
  double* const wsp = ws ? ws : P->d_ws;
  // ring/exchange contractions into the blocks' last slots, in FP64 on the
  // FP64 amplitudes (or corrections) whatever the plan's precision
  if (!P->rx_units_h.empty()) {
    phase_begin(P, 10, s);
    e = launch_ring(P->d_rx_units, (int64_t)P->rx_units_h.size(), P->d_rx_terms, P->d_blocks, T, P->in.S,
                    P->in.ring_ints, wsp, s);
    phase_end(P, s);
    if (e != hipSuccess) return e;
  }
  if (P->sched.items_h.empty()) return hipSuccess;
  if (prec < 0) prec = P->opt.precision;
  // quadratic-term weights from T in FP64 for every residual of T; the
  // correction equations of the mixed solve (weights = false) keep the
  // weights of the last FP64 refinement residual
  if (!P->quad_h.empty() && weights) {
    phase_begin(P, 9, s);
    e = launch_quad_weights(P->d_quad, (int64_t)P->quad_h.size(), P->d_quadG, T, P->d_terms, s);
    phase_end(P, s);
    if (e != hipSuccess) return e;
  }
  // the occupied intermediate from T in FP64: dressed Fock weights and the
  // diagonal shift that the finishing kernel applies; the correction
  // equations of the mixed solve (weights = false) keep those of the last
  // FP64 refinement residual
  if (P->qocc && weights) {
    OccArgs oa{P->d_occ_ctb, (int64_t)P->occ_ctb_h.size(), P->d_occG, P->in.K, P->d_occ_dots, P->d_occ_key_rowptr,
               P->d_occ_key_src, (int64_t)P->occ_key_rowptr_h.size() - 1, P->d_occF, P->d_occ_terms,
               (int64_t)P->occ_terms_h.size(), P->d_terms, P->d_occ_blk_key, P->n_blocks, P->d_occ_shift};
    phase_begin(P, 9, s);
    e = launch_occ_weights(oa, T, s);
    phase_end(P, s);
    if (e != hipSuccess) return e;
  }
  if (prec == DLPNO_FP32) {
    phase_begin(P, 4, s);
    if ((e = launch_convert_f32(T, P->T32, P->n_T, s)) != hipSuccess) return e;
    phase_end(P, s);
  } else if (is_split(prec)) {
    phase_begin(P, 4, s);
    if ((e = launch_split_T(P->d_blocks, P->n_blocks, T, P->d_blk_toff, P->d_blk_tscale, P->Tts_hi, P->Tts_lo,
                            P->Ts_hi, P->Ts_lo, prec == DLPNO_FP16X2, s)) != hipSuccess)
      return e;
    phase_end(P, s);
  }
  if ((e = launch_zero_i32(P->d_counter, kKinds * kQueues, s)) != hipSuccess) return e;
  general = general || (P->opt.flags & DLPNO_FLAG_GENERAL_T) != 0;
  if (is_split(prec)) {
    for (int kind : {ITEM_LADDER, ITEM_PROJ}) {
      if (P->sched.kind_count[kind] == 0) continue;
      SplitArgs a{P->sched.d_items + P->sched.kind_begin[kind], queues(P, P->sched, kind), P->d_pairs, P->d_blocks,
                  P->d_cpl, P->d_terms, P->d_pair_boff, P->d_pair_bscale, P->d_blk_toff, P->d_blk_tscale,
                  P->d_cpl_soff, P->Bs_hi, P->Bs_lo, P->Ss_hi, P->Ss_lo, P->Tts_hi, P->Tts_lo, P->Ts_hi, P->Ts_lo,
                  wsp, general ? 0 : 1, P->d_nonfinite};
      phase_begin(P, kind == ITEM_LADDER ? 0 : 5, s);
      e = launch_split_grouped(a, kind, prec == DLPNO_FP16X2, P->workers, s);
      phase_end(P, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  // each kind in its own launch of the persistent kernel (own queues), so
  // that each is register-allocated alone; the two-wave ladder launch exists
  // in FP64 plans only
  // FP64 residuals of a split plan run its FP64 schedule (same slots)
  const Schedule& S = prec == DLPNO_FP64 && !P->sched64.items_h.empty() ? P->sched64 : P->sched;
  for (int kind : kKindOrder) {
    if (S.kind_count[kind] == 0) continue;
    const Item* items = S.d_items + S.kind_begin[kind];
    const WorkQueues wq = queues(P, S, kind);
    const int phase = kind == ITEM_LADDER    ? 0
                      : kind == ITEM_LADDER2 ? 6
                      : kind == ITEM_LADDER4 ? 7
                      : kind == ITEM_PROJ2   ? 8
                                             : 5;
    phase_begin(P, phase, s);
    if (prec == DLPNO_FP32) {
      GroupedArgs<float> a{items, wq, P->d_pairs, P->d_blocks, P->d_cpl, P->d_terms,
                           P->B32, P->S32, P->T32, wsp, general ? 0 : 1, P->d_nonfinite};
      e = launch_grouped_f32(a, kind, P->workers, s);
    } else {
      GroupedArgs<double> a{items, wq, P->d_pairs, P->d_blocks, P->d_cpl, P->d_terms,
                            P->in.B, P->in.S, T, wsp, general ? 0 : 1, P->d_nonfinite};
      e = launch_grouped_f64(a, kind, P->workers, s);
    }
    phase_end(P, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

FinishArgs finish_args(dlpno_plan* P, const double* T, const double* ws) {
  FinishArgs f{};
  f.blocks = P->d_blocks;
  f.n_blocks = P->n_blocks;
  f.T = T;
  f.K = P->in.K;
  f.eps_a = P->in.eps_a;
  f.eps_b = P->in.eps_b;
  f.ws = ws ? ws : P->d_ws;
  f.e_block = P->d_e_block;
  f.rmax_block = P->d_rmax_block;
  f.nonfinite = P->d_nonfinite;
  f.with_driver = 1;
  f.shift = P->d_occ_shift;
  return f;
}

hipError_t amplitudes_zero(dlpno_plan* P, const double* T, hipStream_t s, bool* zero) {
  hipError_t e;
  int32_t h = 1;
  if ((e = launch_zero_i32(P->d_flagz, 1, s)) != hipSuccess) return e;
  if ((e = launch_any_nonzero(T, P->n_T, P->d_flagz, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&h, P->d_flagz, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *zero = h == 0;
  return hipSuccess;
}

// one full iteration on stream s (capturable: kernels only)
hipError_t enqueue_iteration(dlpno_plan* P, double* T, double* R, double* e_pair, double* e_total, double* rmax,
                             hipStream_t s, const double* drv, int prec, bool record, bool zero_T) {
  hipError_t e;
  const bool diis = P->opt.diis_max > 0;
  if (diis && (e = launch_diis_slot(P->d_diis, s)) != hipSuccess) return e;
  if (!zero_T && (e = run_grouped(P, T, s, prec, false, nullptr, drv == nullptr)) != hipSuccess) return e;
  FinishArgs f = finish_args(P, T);
  f.no_partials = zero_T ? 1 : 0;
  if (zero_T) f.shift = nullptr;     // T = 0: the diagonal part vanishes with the rest
  f.R = R;
  f.drv = drv;
  if (diis) {
    f.ring = P->d_diis;
    f.ring_vecs = P->d_ring_vecs;
    f.ring_errs = P->d_ring_errs;
    f.ring_stride = P->n_T;
  } else {
    f.T_new = T;     // in place: every element is read before it is written by the same thread
  }
  phase_begin(P, 1, s);
  if ((e = launch_finish(f, s)) != hipSuccess) return e;
  phase_end(P, s);
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
  ra.hist = record ? P->d_hist : nullptr;
  ra.iter = record ? P->d_hist_iter : nullptr;
  ra.hist_cap = kHistCap;
  phase_begin(P, 2, s);
  if ((e = launch_reduce(ra, s)) != hipSuccess) return e;
  phase_end(P, s);
  if (diis) {
    phase_begin(P, 3, s);
    if ((e = launch_diis_dots(P->d_ring_errs, P->n_T, P->d_diis, P->d_diis_partial, kDiisParts, s)) != hipSuccess)
      return e;
    if ((e = launch_diis_solve(P->d_diis, P->d_diis_partial, kDiisParts, s)) != hipSuccess) return e;
    if ((e = launch_diis_extrap(P->d_ring_vecs, P->n_T, P->d_diis, T, s)) != hipSuccess) return e;
    phase_end(P, s);
  }
  return hipSuccess;
}

}  // namespace dlpno

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
extern "C" dlpno_status dlpno_residual(dlpno_plan* P, const double* T, double* R, void* stream) {
  if (!P || ((!T || !R) && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)stream;
  HIPCK(run_grouped(P, T, s));
  FinishArgs f = finish_args(P, T);
  f.R = R;
  phase_begin(P, 1, s);
  HIPCK(launch_finish(f, s));
  phase_end(P, s);
  if (P->profiling) phase_collect(P);
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_update(dlpno_plan* P, const double* T, const double* R, double* T_out, double* e_pair,
                                     double* e_total, void* stream) {
  if (!P || ((!T || !R || !T_out) && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)stream;
  UpdateArgs u{P->d_blocks, P->n_blocks, T, R, P->in.K, P->in.eps_a, P->in.eps_b, T_out, P->d_e_block};
  HIPCK(launch_update(u, s));
  ReduceArgs ra{};
  ra.partial = P->d_red_partial;
  ra.pairs = P->d_pairs;
  ra.blocks = P->d_blocks;
  ra.n_blocks = P->n_blocks;
  ra.n_pairs = P->n_pairs;
  ra.e_block = P->d_e_block;
  ra.rmax_block = nullptr;
  ra.e_pair = e_pair;
  ra.e_total = e_total;
  HIPCK(launch_reduce(ra, s));
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_f12_energy(dlpno_plan* P, const double* T, const double* W, const double* scalars,
                                         double* e_pair, double* e_total, void* stream) {
  if (!P || ((!T || !W) && P->n_T > 0) || (!scalars && P->n_blocks > 0))
    return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)stream;
  F12Args f{P->d_blocks, P->n_blocks, T, W, scalars, P->d_f12_block};
  HIPCK(launch_f12(f, s));
  ReduceArgs ra{};
  ra.partial = P->d_red_partial;
  ra.pairs = P->d_pairs;
  ra.blocks = P->d_blocks;
  ra.n_blocks = P->n_blocks;
  ra.n_pairs = P->n_pairs;
  ra.e_block = P->d_f12_block;
  ra.rmax_block = nullptr;
  ra.e_pair = e_pair;
  ra.e_total = e_total;
  HIPCK(launch_reduce(ra, s));
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_reset(dlpno_plan* P, void* stream) {
  if (!P) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan");
  hipStream_t s = (hipStream_t)stream;
  HIPCK(launch_diis_reset(P->d_diis, std::max(1, P->opt.diis_max), std::max(1, P->opt.diis_start), s));
  HIPCK(launch_zero_i32(P->d_nonfinite, 1, s));
  HIPCK(launch_zero_i32(P->d_hist_iter, 1, s));
  HIPCK(hipStreamSynchronize(s));
  P->host_iter = 0;
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_iterate(dlpno_plan* P, int32_t n_iter, double* T, double* R, double* e_pair,
                                      double* e_total, double* max_abs_R, void* stream) {
  if (!P || n_iter < 0 || ((!T || !R) && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  // from T = 0 the first residual is the driver alone: its grouped launches
  // (which would add exact zeros) are skipped
  int first = 0;
  if (n_iter > 0 && P->n_T > 0) {
    bool zero = false;
    HIPCK(amplitudes_zero(P, T, s, &zero));
    if (zero) {
      HIPCK(enqueue_iteration(P, T, R, e_pair, e_total, max_abs_R, s, nullptr, -1, true, true));
      first = 1;
    }
  }
  if (P->profiling) {
    for (int k = first; k < n_iter; ++k) HIPCK(enqueue_iteration(P, T, R, e_pair, e_total, max_abs_R, s));
    phase_collect(P);
  } else if (first < n_iter) {
    const void* key[5] = {T, R, e_pair, e_total, max_abs_R};
    if (!P->graph_valid || memcmp(key, P->graph_key, sizeof key) != 0) {
      if (P->gexec) {
        (void)hipGraphExecDestroy(P->gexec);
        P->gexec = nullptr;
      }
      hipGraph_t g;
      HIPCK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t ce = enqueue_iteration(P, T, R, e_pair, e_total, max_abs_R, P->cap_stream);
      hipError_t ee = hipStreamEndCapture(P->cap_stream, &g);
      if (ce != hipSuccess) return fail(DLPNO_ERR_HIP, std::string("capture: ") + hipGetErrorString(ce));
      HIPCK(ee);
      HIPCK(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
      (void)hipGraphDestroy(g);
      memcpy(P->graph_key, key, sizeof key);
      P->graph_valid = true;
    }
    for (int k = first; k < n_iter; ++k) HIPCK(hipGraphLaunch(P->gexec, s));
  }
  P->host_iter += n_iter;
  return read_status(P, s);
}

extern "C" int32_t dlpno_history(const dlpno_plan* P, double* energy, double* max_abs_r, int32_t n) {
  if (!P || n <= 0) return 0;
  const int have = (int)std::min<int64_t>(P->host_iter, kHistCap);
  const int m = std::min(n, have);
  std::vector<double> h(2 * (size_t)std::max(m, 1));
  if (m > 0 && hipMemcpy(h.data(), P->d_hist, 2 * sizeof(double) * m, hipMemcpyDeviceToHost) != hipSuccess) return 0;
  for (int k = 0; k < m; ++k) {
    if (energy) energy[k] = h[2 * k];
    if (max_abs_r) max_abs_r[k] = h[2 * k + 1];
  }
  return m;
}

extern "C" dlpno_status dlpno_diis_state(const dlpno_plan* P, int32_t* count, int32_t* drops, double* coef,
                                         void* stream) {
  if (!P) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan");
  hipStream_t s = (hipStream_t)stream;
  DiisState st;
  HIPCK(hipMemcpyAsync(&st, P->d_diis, sizeof st, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (count) *count = st.count;
  if (drops) *drops = st.drops;
  if (coef) {
    for (int k = 0; k < 8; ++k) coef[k] = 0.0;
    const int mx = std::max(1, st.max);
    for (int k = 0; k < st.count && k < 8; ++k) coef[k] = st.coef[(st.head - (st.count - 1 - k) + mx) % mx];
  }
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_flop_count(const dlpno_plan* P, double* ladder, double* projection) {
  if (!P) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan");
  if (ladder) *ladder = P->flops_ladder;
  if (projection) *projection = P->flops_proj;
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_ring_flop_count(const dlpno_plan* P, double* flops, int64_t* contractions) {
  if (!P) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan");
  if (flops) *flops = P->flops_rx;
  if (contractions) *contractions = (int64_t)P->rx_terms_h.size();
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_set_profiling(dlpno_plan* P, int32_t enable) {
  if (!P) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan");
  P->profiling = enable != 0;
  for (int k = 0; k < kPhases; ++k) {
    P->phase_ms[k] = 0.0;
    P->phase_n[k] = 0;
  }
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_phase_times(const dlpno_plan* P, double* ms, int64_t* launches, int32_t n) {
  if (!P) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan");
  for (int k = 0; k < n && k < kPhases; ++k) {
    if (ms) ms[k] = P->phase_ms[k];
    if (launches) launches[k] = P->phase_n[k];
  }
  return DLPNO_OK;
}

extern "C" const char* dlpno_plan_info(const dlpno_plan* P) { return P ? P->info.c_str() : ""; }

extern "C" const char* dlpno_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* dlpno_status_string(dlpno_status s) {
  switch (s) {
    case DLPNO_OK: return "ok";
    case DLPNO_ERR_INVALID_ARG: return "invalid argument";
    case DLPNO_ERR_DIM_RANGE: return "dimension out of range";
    case DLPNO_ERR_ALIGNMENT: return "offset outside buffer";
    case DLPNO_ERR_HIP: return "HIP runtime error";
    case DLPNO_ERR_NONFINITE: return "non-finite residual";
    case DLPNO_ERR_NOT_CONVERGED: return "not converged";
    case DLPNO_ERR_OOM: return "out of device memory";
    case DLPNO_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}
