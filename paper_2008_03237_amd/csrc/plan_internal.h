// Plan object of the DLPNO residual library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <algorithm>
#include <vector>

#include "../../include/dlpno.h"
#include "internal.h"

namespace dlpno {

constexpr int kHistCap = 4096;   // iterations kept in the device history
constexpr int kDiisParts = 1024; // workgroups of the DIIS dot-product kernel
constexpr int kPhases = 11;

// schedule choices (set by defaults or the autotuner)
struct Tuning {
  int ladder_variant[4] = {0, 3, 7, 8};   // by tiles of 16 PNOs (1..4); FP64 plans start from 0 4 7 9
  int proj_variant[4] = {0, 4, 7, 8};
  double items_per_wave = 6.0;            // target items per wavefront of the queue
  bool two_wave = true;                   // FP64: the two-wave launches (kLadderTwoWave, kLadderCoop, kProjTwoWave)
  double min_item_mfma = 2048.0;          // smallest item worth scheduling alone
};

// One list of work items with its per-kind queues.
struct Schedule {
  std::vector<Item> items_h;            // items by kind, in launch order (kKindOrder)
  int32_t kind_begin[kKinds] = {}, kind_count[kKinds] = {};
  // per kind: queue k holds items [qoff[kind][k], qoff[kind][k+1]) counted
  // from the kind's first item
  int32_t qoff[kKinds][kQueues + 1] = {};
  Item* d_items = nullptr;
};

struct PendingEvent {
  int phase;
  hipEvent_t start, stop;
};

}  // namespace dlpno

struct dlpno_plan {
  dlpno_options opt{};
  int device = 0, num_cu = 0, workers = 0;
  std::string arch;                     // device architecture name (autotuner cache key)
  int32_t n_occ = 0, n_pairs = 0, n_blocks = 0;
  int64_t n_cpl = 0, n_terms = 0, n_hh = 0;   // couplings (Fock + hole-hole), of them hole-hole
  int64_t n_B = 0, n_T = 0, n_K = 0, n_eps = 0, n_S = 0;
  dlpno_inputs in{};
  std::vector<uint8_t> somo;
  std::vector<dlpno::PairDev> pairs_h;
  std::vector<dlpno::BlockDev> blocks_h;
  bool somo_virt = false;                // some pair has SOMO virtual functions
  std::vector<dlpno::QuadCpl> quad_h;    // hole-hole couplings with quadratic weights
  dlpno::QuadCpl* d_quad = nullptr;
  double* d_quadG = nullptr;             // S K S^T per quadratic coupling (built once)
  int32_t* d_flagz = nullptr;            // flag of amplitudes_zero
  int64_t n_quadG = 0;
  double flops_quad = 0.0;               // the weights' dot products per residual
  double flops_quad_prep = 0.0;          // building the factors S K S^T (once)
  // quadratic part of the occupied Fock intermediate (DLPNO_FLAG_QUADRATIC_OCC)
  bool qocc = false;
  std::vector<dlpno::OccCtb> occ_ctb_h;
  std::vector<dlpno::OccTerm> occ_terms_h;
  std::vector<int32_t> occ_blk_key_h;
  std::vector<int64_t> occ_key_rowptr_h, occ_key_src_h;
  int64_t n_occG = 0;
  dlpno::OccCtb* d_occ_ctb = nullptr;
  dlpno::OccTerm* d_occ_terms = nullptr;
  int32_t* d_occ_blk_key = nullptr;
  int64_t* d_occ_key_rowptr = nullptr;
  int64_t* d_occ_key_src = nullptr;
  double* d_occG = nullptr;
  double* d_occ_dots = nullptr;
  double* d_occF = nullptr;
  double* d_occ_shift = nullptr;
  double flops_occ = 0.0, flops_occ_prep = 0.0;
  // ring/exchange term: contractions per target block (units), last partial slot
  std::vector<dlpno::RxTerm> rx_terms_h;
  std::vector<dlpno::RxUnit> rx_units_h;
  std::vector<uint8_t> rx_block;         // per block: 1 = has ring contractions (owns the last slot)
  dlpno::RxTerm* d_rx_terms = nullptr;
  dlpno::RxUnit* d_rx_units = nullptr;
  int64_t n_ring = 0;
  double flops_rx = 0.0;
  std::vector<dlpno::CplDev> cpl_h;
  std::vector<dlpno::TermDev> terms_h;
  std::vector<int64_t> rowptr_h;
  // k and side of each coupling (order of cpl_h); side 2 marks a hole-hole
  // coupling, whose ordered source is (k, l)
  std::vector<int32_t> cpl_k_h, cpl_side_h, cpl_l_h;
  // preconditions of the vector-Jacobian product (the transposed residual is
  // evaluated by the forward kernels): symmetric occupied Fock matrices
  // (checked at creation), a reverse for every coupling with a term and
  // transposed overlap blocks on it (checked at the first product)
  bool fock_symmetric = true;
  int vjp_checked = 0;                        // 0 not yet, 1 satisfied, -1 violated
  std::string vjp_reason;
  dlpno::Schedule sched;                // the plan's precision
  dlpno::Schedule sched64;              // split plans: FP64 items over the same slots (refinement residuals)
  dlpno::Tuning tune;
  double flops_ladder = 0.0, flops_proj = 0.0, total_mfma = 0.0, max_item_mfma = 0.0;
  int64_t ws_elems = 0;
  // device tables and buffers
  dlpno::PairDev* d_pairs = nullptr;
  dlpno::BlockDev* d_blocks = nullptr;
  dlpno::CplDev* d_cpl = nullptr;
  dlpno::TermDev* d_terms = nullptr;
  int32_t* d_counter = nullptr;        // queue heads: kQueues per kind
  double* d_ws = nullptr;
  double* d_e_block = nullptr;
  double* d_f12_block = nullptr;        // F12 pair energy per block
  double* d_red_partial = nullptr;      // energy/max|R| reduction scratch, 2 kReduceParts
  double* d_rmax_block = nullptr;
  int32_t* d_nonfinite = nullptr;
  int32_t* d_hist_iter = nullptr;   // iterations recorded in the history
  double* d_hist = nullptr;
  dlpno::DiisState* d_diis = nullptr;
  double* d_scalars = nullptr;
  double* d_diis_partial = nullptr;
  double* d_ring_vecs = nullptr;
  double* d_ring_errs = nullptr;
  float* B32 = nullptr;
  float* S32 = nullptr;
  float* T32 = nullptr;
  // split precision
  int64_t n_Bs = 0, n_Ss = 0, n_Ts = 0;
  int64_t* d_pair_boff = nullptr;
  int64_t* d_blk_toff = nullptr;
  int64_t* d_cpl_soff = nullptr;
  int64_t* d_cpl_target = nullptr;
  float* d_pair_bscale = nullptr;
  float* d_blk_tscale = nullptr;
  uint16_t *Bs_hi = nullptr, *Bs_lo = nullptr, *Ss_hi = nullptr, *Ss_lo = nullptr;
  uint16_t *Tts_hi = nullptr, *Tts_lo = nullptr, *Ts_hi = nullptr, *Ts_lo = nullptr;
  double* d_mix_r = nullptr;       // FP64 residual of the outer refinement
  double* d_mix_delta = nullptr;   // correction of the inner solve
  void* d_vjp_items = nullptr;
  int n_vjp_items = 0;
  float* G32 = nullptr;
  void* d_mixed = nullptr;
  // graph replay
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_valid = false;
  const void* graph_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t host_iter = 0;
  // profiling
  bool profiling = false;
  std::vector<hipEvent_t> events;
  std::vector<dlpno::PendingEvent> pending;
  double phase_ms[dlpno::kPhases] = {};
  int64_t phase_n[dlpno::kPhases] = {};
  std::string info;
};

namespace dlpno {
// plan.hip
dlpno_status fail(dlpno_status s, const std::string& msg);
dlpno_status build_schedule(dlpno_plan* P);
dlpno_status upload_schedule(dlpno_plan* P, hipStream_t s);
// general: the amplitudes may lack the antisymmetry of same-spin blocks
// (cotangents of the vector-Jacobian product), so every tile is computed
// ws: partial-sum workspace to use in place of the plan's own (nullptr: the plan's)
hipError_t run_grouped(dlpno_plan* P, const double* T, hipStream_t s, int prec = -1, bool general = false,
                       double* ws = nullptr, bool weights = true);
FinishArgs finish_args(dlpno_plan* P, const double* T, const double* ws = nullptr);
// noalloc.hip: device address of the static scratch array, once per device
// (called by dlpno_plan_create with the plan's device current)
dlpno_status scratch_init(int device);
hipError_t enqueue_iteration(dlpno_plan* P, double* T, double* R, double* e_pair, double* e_total, double* rmax,
                             hipStream_t s, const double* drv = nullptr, int prec = -1, bool record = true,
                             bool zero_T = false);
// *zero = every element of T is zero (synchronises the stream); then R(T) is
// the driver alone and the grouped launches can be skipped
hipError_t amplitudes_zero(dlpno_plan* P, const double* T, hipStream_t s, bool* zero);
bool is_split(int prec);
dlpno_status read_status(dlpno_plan* P, hipStream_t s);
std::string describe(const dlpno_plan* P);
void phase_begin(dlpno_plan* P, int ph, hipStream_t s);
void phase_end(dlpno_plan* P, hipStream_t s);
void phase_collect(dlpno_plan* P);
}  // namespace dlpno
