// Split-precision (BF16x2 / FP16x2) operands and kernel interface.
#pragma once
#include "internal.h"

namespace dlpno {

struct SplitArgs {
  const Item* items;
  WorkQueues q;
  const PairDev* pairs;
  const BlockDev* blocks;
  const CplDev* cpl;
  const TermDev* terms;
  const int64_t* pair_boff;   // split B offset per pair (n x N16 per Q)
  const float* pair_bscale;   // FP16: power-of-two scale of B_p (null for BF16)
  const int64_t* blk_toff;    // split amplitude offset per block (n x N16)
  const float* blk_tscale;    // FP16: power-of-two scale per block (null for BF16)
  const int64_t* cpl_soff;    // split S offset per coupling (n_target x N16(n_src))
  const uint16_t* B_hi;
  const uint16_t* B_lo;
  const uint16_t* S_hi;
  const uint16_t* S_lo;
  const uint16_t* Tt_hi;      // amplitudes, transposed copy [d][c]
  const uint16_t* Tt_lo;
  const uint16_t* T_hi;       // amplitudes, plain copy [c][d]
  const uint16_t* T_lo;
  double* ws;
  int32_t anti;               // same-spin blocks antisymmetric (see GroupedArgs::anti)
  int32_t* err;               // device status word (see kErrNoBody)
};

// kind: ITEM_LADDER or ITEM_PROJ; every item of `a` must be of that kind
hipError_t launch_split_grouped(const SplitArgs& a, int kind, bool fp16, int workers, hipStream_t s);
hipError_t launch_split_B(const PairDev* pairs, int npairs, const double* B, const int64_t* boff, float* bscale,
                          uint16_t* hi, uint16_t* lo, bool fp16, hipStream_t s);
hipError_t launch_split_S(const PairDev* pairs, const int64_t* cpl_target, const CplDev* cpl, const double* S,
                          const int64_t* soff, int64_t ncpl, uint16_t* hi, uint16_t* lo, bool fp16, hipStream_t s);
hipError_t launch_split_T(const BlockDev* blocks, int nblocks, const double* T, const int64_t* toff, float* tscale,
                          uint16_t* tt_hi, uint16_t* tt_lo, uint16_t* t_hi, uint16_t* t_lo, bool fp16, hipStream_t s);

}  // namespace dlpno
