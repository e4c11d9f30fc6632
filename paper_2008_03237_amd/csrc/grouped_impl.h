// Persistent grouped kernel: every DF ladder and PNO-overlap projection
// contraction of one residual evaluation, over all pairs of uneven PNO and
// auxiliary sizes.  Ladder items and projection items run as separate
// launches of the same persistent kernel (KIND), each with its own queues, so
// that each body is register-allocated alone.  In FP64 the ladder items of
// pairs with at most three PNO tiles run at two waves per SIMD (one B^Q
// buffer, a smaller LDS slab), and those of four-tile pairs in a cooperative
// launch, also at two waves per SIMD, in which a whole workgroup takes one
// item of two blocks and each pair of waves shares one block's X slab.
//
// Both contractions have the "sandwich" form  Out = M X M^T  summed over a
// list of (M, X) pairs:
//   ladder      M = B^Q_p, X = T^{ss'}_p, summed over Q: the DF factorisation
//               (ac|bd) = sum_Q B^Q_ac B^Q_bd of the four-external integrals
//               in the pair's PNO basis;
//   projection  M = S_{p,q}, X = -w op(T_q), summed over the neighbour
//               couplings of the target pair (one overlap set for all spins).
// One wavefront evaluates a sandwich on the 16x16x4 MFMA with the first
// product kept in registers: the accumulator layout of  Y^T = X^T M^T  is,
// after a fixed permutation of its row index, exactly the B-operand layout of
// Out^T = M Y^T, so  Y = M X  never leaves the VGPRs (it is recomputed for
// every Q instead of stored).  With M symmetric (B^Q) the same registers serve
// as the B operand of the first product and the A operand of the second.
//
// Register forms (lane l, r = l & 15, g = l >> 4):
//   M-form  M[t][s]  = M[16 t + r][4 s + g]          (rows: target PNO, cols: inner)
//   X-form  Al[t][s] = X[4 s + g][16 t + perm(r)]
//   output  acc[tb][ta][i] = Out[16 ta + r][16 tb + orow(g, i)]
// The 16x16x4 FP64 MFMA returns output row 4 i + g in register i of lane
// group g (perm = identity, orow = 4 i + g); the FP32 one returns row 4 g + i,
// so its A rows are fed in the order perm(r) = 4 (r & 3) + (r >> 2), after
// which register i again holds rows 4 i + g.  Either way register i of the
// first product is exactly k-step i of the second.
// K-steps of 4 beyond the inner dimension are skipped, so only the M and N
// tile edges are padded to 16; in FP64 the partial last ladder tile runs as
// row strips of 4 (see mfma_strip).  Operands are read with raw buffer loads
// whose resource covers exactly one matrix: reads past its end return zero,
// and the remaining padded reads land inside the same matrix, are finite, and
// only reach rows or columns that are multiplied by those zeros or never
// stored.
//
// Same-spin blocks hold antisymmetric amplitudes, so their contributions are
// antisymmetric: a compile-time block mask limits stage 2 to the tiles on and
// below the diagonal, and store_tiles writes the others mirrored.
//
// The X-form operands live in a per-wave LDS slab (one 8-byte slot per lane
// and operand, conflict free) or, for small tiles, in VGPRs; at one wave per
// SIMD the M operands of B^Q are double-buffered in VGPRs so the next slice is
// in flight while the current one is contracted.  Projection items are
// software-pipelined one (coupling, block) unit ahead.
//
// Work items come from one queue per XCD, each ordered longest-first (see
// next_item); every wave (cooperative launch: every workgroup) pops items with
// one atomic increment until all queues are empty, the exit condition every
// wave reaches.  Each item writes its partial sums to a private workspace
// slot; the finishing kernel adds the slots in a fixed order, so results are
// bitwise reproducible.
#pragma once
#include "internal.h"

#include <type_traits>

namespace dlpno {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename F>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4_t V;
  static __device__ __forceinline__ V op(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, uint32_t off_elems) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off_elems * 8u, 0u, 0));
  }
  // FP64 16x16x4: register i of lane group g holds output row 4 i + g
  static __device__ __forceinline__ int perm(int r) { return r; }
  static __device__ __forceinline__ int orow(int g, int i) { return 4 * i + g; }
};
template <>
struct Mfma<float> {
  typedef f4_t V;
  static __device__ __forceinline__ V op(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t off_elems) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off_elems * 4u, 0u, 0));
  }
  // FP32 16x16x4: register i of lane group g holds output row 4 g + i; feeding
  // A rows in the order pi(r) makes register i hold rows 4 i + g as well
  static __device__ __forceinline__ int perm(int r) { return ((r & 3) << 2) | (r >> 2); }
  static __device__ __forceinline__ int orow(int g, int i) { return 4 * g + i; }
};

// FP64 row strips.  The four-block 4x4x4 FP64 MFMA (lane 16 g + 4 b + v:
// A[m = v][k = g], B[k = g][n = v], D[m = g][n = v] of block b) does a quarter
// of the work of the 16x16x4 one in less than a quarter of its time on
// gfx950.  Given the 16x16x4 B operand register (k in g, 16 columns in r =
// 4 b + v) and an A operand whose four blocks all hold rows 4 j .. 4 j + 3 of
// the 16x16x4 A operand, it returns rows 4 j .. 4 j + 3 of the 16x16x4 product
// in one register laid out like register j of the 16x16x4 accumulator (row
// 4 j + g, column r).  Strips made only of padded rows are not issued, so the
// row dimensions of both sandwich stages are padded to 4 instead of 16.  The
// instruction has no operand broadcast for FP64, so the replicated A operand
// is built with DPP row shifts (bcast_strip) or read from LDS with a
// lane-permuted address (strip_lane).
template <typename F>
struct Strips : std::false_type {};
template <>
struct Strips<double> : std::true_type {};
__device__ __forceinline__ double mfma_strip(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
// lane of a 16x16x4 operand register that holds what lane `lane` needs as the
// A operand of strip j: same g and v, block j
__device__ __forceinline__ int strip_lane(int lane, int j) { return (lane & 0x33) | (j << 2); }
// every block of every row of 16 lanes receives block J of that row:
// row_shl:n reads lane + n, row_shr:n reads lane - n (within the row); the
// bank mask restricts each copy to one block
template <int J, int B>
__device__ __forceinline__ void bcast_block(int& lo, int& hi, int lo0, int hi0) {
  if constexpr (B != J) {
    constexpr int ctrl = B < J ? 0x100 + 4 * (J - B) : 0x110 + 4 * (B - J);
    lo = __builtin_amdgcn_update_dpp(lo, lo0, ctrl, 0xf, 1 << B, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi0, ctrl, 0xf, 1 << B, false);
  }
}
template <int J>
__device__ __forceinline__ double bcast_strip(double x) {
  const int lo0 = __double2loint(x), hi0 = __double2hiint(x);
  int lo = lo0, hi = hi0;
  bcast_block<J, 0>(lo, hi, lo0, hi0);
  bcast_block<J, 1>(lo, hi, lo0, hi0);
  bcast_block<J, 2>(lo, hi, lo0, hi0);
  bcast_block<J, 3>(lo, hi, lo0, hi0);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double bcast_strip(double x, int j) {
  switch (j) {
    case 0: return bcast_strip<0>(x);
    case 1: return bcast_strip<1>(x);
    case 2: return bcast_strip<2>(x);
    default: return bcast_strip<3>(x);
  }
}

// Wave-uniform copies of descriptor fields.  Descriptors are read with vector
// loads (the kernel also writes memory, so they cannot go through the scalar
// cache); broadcasting them from lane 0 tells the compiler they are uniform,
// so resource descriptors, trip counts and branches stay in SGPRs.
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double x) { return __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, x))); }
template <typename T>
__device__ __forceinline__ T* uni(T* p) { return reinterpret_cast<T*>(uni(reinterpret_cast<int64_t>(p))); }

// An item whose (kind, variant) has no compiled body: the plan checks every
// item against the compiled tables when it builds the schedule, so this is
// never reached; if it were, the item's partial slot would be left stale, so
// the wave raises kErrNoBody in the plan's status word instead of skipping
// silently.
__device__ __forceinline__ void no_body(int32_t* err) {
  if ((threadIdx.x & 63) == 0 && err) atomicOr(err, kErrNoBody);
}

// raw buffer resource over [p, p + elems): out-of-range loads return 0
template <typename F>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const F* p, uint32_t elems) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<F*>(uni(p)), (short)0,
                                           (uint32_t)uni((int32_t)(elems * (uint32_t)sizeof(F))), 0x00020000);
}

// Per-wave LDS slab for X-form operands, in 8-byte words: the largest users
// are the 3-tile, 2-block ladder variant (2 * 3 * 12 operands of 64 lanes) and
// the projection (4 * 16 operands).
constexpr int kLdsWaveWords = 72 * 64;
// ... and for the launch at two waves per SIMD (two workgroups per CU): the
// 3-tile one-block ladder variant (3 * 12 operands)
constexpr int kLdsWaveWords2 = 40 * 64;
// ... and per pair of waves in the cooperative four-tile launch (two
// workgroups per CU, two slabs each): 4 * 16 operands
constexpr int kCoopSlabWords = 64 * 64;

// Partial sums of one block into its workspace slot: acc[tb][u] holds the
// Out^T tile with rows in b-tile tb and columns in a-tile ta0 + u dta (row b,
// column a stored at b n + a, coalesced over r).  mirror: the block's result
// is antisymmetric; tiles above the diagonal (tb < ta) were not computed and
// are written as the negated transpose of the tile below it, by whichever item
// owns that tile's a-tile.
// (store_tiles_first: the first NS of the NU accumulator columns)
template <typename F, int NT, int NS, int NU, typename V>
__device__ __forceinline__ void store_tiles_first(double* dst, int n, int ta0, const V (&acc)[NT][NU], bool mirror,
                                                  double scale = 1.0, int dta = 1) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int tb = 0; tb < NT; ++tb)
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int ta = ta0 + u * dta;
      if (mirror && tb < ta) continue;
      const int a = 16 * ta + r;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int bb = 16 * tb + Mfma<F>::orow(g, i);
        if (a < n && bb < n) {
          const double v = (double)acc[tb][u][i] * scale;
          dst[bb * n + a] = v;
          if (mirror && tb > ta) dst[a * n + bb] = -v;
        }
      }
    }
}
template <typename F, int NT, int NU, typename V>
__device__ __forceinline__ void store_tiles(double* dst, int n, int ta0, const V (&acc)[NT][NU], bool mirror,
                                            double scale = 1.0, int dta = 1) {
  store_tiles_first<F, NT, NU, NU>(dst, n, ta0, acc, mirror, scale, dta);
}

// ---------------------------------------------------------------------------
// Ladder item: pair p, NB consecutive blocks, a-tiles TA0 + u DTA for
// u < NTA, Q in [lo, hi).  Partial Out^T[b][a] of sum_Q B^Q T B^Q^T.
// The inner (k) dimension runs over S4 = 4 (NT - 1) + R steps of 4, R in
// 1..4: n is padded to a multiple of 4, and with every trip count known at
// compile time one Q slice is a single basic block that the scheduler can
// interleave (stage 1 of every block is issued before the stage 2 that reads
// it).  REG keeps the X-form operands in VGPRs instead of the LDS slab.
// W2: the launch runs two waves per SIMD (one B^Q buffer, smaller slab).
// COOP: one wave's share of a cooperative item (see ladder_coop).
// ---------------------------------------------------------------------------
template <typename F, int NT, int NB, int NTA, int TA0, int R, bool REG, int MASK, bool W2, int DTA = 1,
          bool COOP = false>
__device__ __forceinline__ void ladder_item(const GroupedArgs<F>& A, const Item& it, double* lds) {
  typedef typename Mfma<F>::V V;
  constexpr int S4 = 4 * (NT - 1) + R;
  constexpr int LW = COOP ? kCoopSlabWords : W2 ? kLdsWaveWords2 : kLdsWaveWords;
  static_assert(NB * NT * S4 * 64 <= LW, "X slab exceeds the wave's LDS");
  // a-tile of accumulator column u
  auto ta = [](int u) { return TA0 + u * DTA; };
  // cooperative items: waves 2h and 2h + 1 take block h of the item and
  // share its X slab (both write it whole, with the same values)
  const int wave = threadIdx.x >> 6;
  const int bslot0 = it.bslot0 + (COOP ? (wave >> 1) : 0);
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4, pr = Mfma<F>::perm(r);
  const PairDev& Pg = A.pairs[it.pair];
  const int n = uni(Pg.n);
  const int blk0 = uni(Pg.blk0);
  const int64_t off_B = uni(Pg.off_B);
  const uint32_t nn = (uint32_t)n * (uint32_t)n;
  F* Al = reinterpret_cast<F*>(lds + (size_t)(COOP ? (wave >> 1) : wave) * LW);
  // FP64 with a partial last tile (R < 4 k-steps in it): the last d-tile of
  // stage 1 and the last b-tile of stage 2 run as R row strips; the X operands
  // of that d-tile are then also kept in the LDS slab, where the strips read
  // them at permuted lanes
  constexpr bool STRIPS = Strips<F>::value && R < 4;
  // Column strips (FP64): when the item's last a-tile is the pair's last tile
  // and holds at most 4 kColStrips PNO columns, that a-tile runs as R strips of
  // four columns (four-block 4x4x4 MFMAs with the B operand broadcast across
  // the blocks) in both stages instead of one 16-wide tile (see the loops).
  constexpr int UL = NTA - 1;                      // accumulator column of the last a-tile
  constexpr bool CS = STRIPS && R <= kColStrips && TA0 + UL * DTA == NT - 1;
  F Ar[REG ? NB : 1][REG ? NT : 1][REG ? S4 : 1];

  // X-form operands of the NB amplitude blocks, once per item
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int64_t off_T = uni(A.blocks[blk0 + bslot0 + b].off_T);
    const __amdgpu_buffer_rsrc_t tr = rsrc(A.T + off_T, nn);
    const uint32_t base = (uint32_t)(g * n + pr);
#pragma unroll
    for (int td = 0; td < NT; ++td)
#pragma unroll
      for (int s = 0; s < S4; ++s) {
        const F v = Mfma<F>::load(tr, base + (uint32_t)(4 * s * n + 16 * td));
        if constexpr (REG) Ar[b][td][s] = v;
        if (!REG || (STRIPS && td == NT - 1)) Al[((b * NT + td) * S4 + s) * 64 + lane] = v;
      }
  }
  auto aop = [&](int b, int td, int s) -> F {
    if constexpr (REG) return Ar[b][td][s];
    else return Al[((b * NT + td) * S4 + s) * 64 + lane];
  };
  // A operand of row strip i of the last d-tile: block i of the X operand
  auto aop_strip = [&](int b, int s, int i) -> F { return Al[((b * NT + NT - 1) * S4 + s) * 64 + strip_lane(lane, i)]; };

  V acc[NB][NT][NTA];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < NTA; ++u) acc[b][t][u] = V{0, 0, 0, 0};
  // column strips of the last a-tile: accC[b][tb][j], lane 16 g + 4 k + v
  // holds Out^T[16 tb + 4 k + g][16 (NT - 1) + 4 j + v]
  constexpr int RC = CS ? R : 1;
  F accC[NB][NT][RC];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int j = 0; j < RC; ++j) accC[b][t][j] = F(0);
  // bit b of MASK: block b is antisymmetric (same spin), stage 2 only for
  // tiles with tb >= ta
  auto mir = [](int b) { return ((MASK >> b) & 1) != 0; };

  // M-form of B^Q: M[t][s] = B^Q[4s + g][16t + r] = B^Q[16t + r][4s + g] (symmetric)
  const F* Bp = A.B + off_B;
  const uint32_t mbase = (uint32_t)(g * n + r);
  // k-steps [s0, s1) of every tile of the M-form of slice Q
  auto loadM_steps = [&](F (&M)[NT][S4], int Q, int s0, int s1) {
    const __amdgpu_buffer_rsrc_t br = rsrc(Bp + (size_t)Q * nn, nn);
#pragma unroll
    for (int s = s0; s < s1; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t) M[t][s] = Mfma<F>::load(br, mbase + (uint32_t)(4 * s * n + 16 * t));
  };
  auto loadM = [&](F (&M)[NT][S4], int Q) { loadM_steps(M, Q, 0, S4); };

  // W2 (one B^Q buffer): once the last d-tile's stage 1 has run, k-steps
  // s < 4 (NT - 1) of M are dead (that d-tile's stage 2 reads only the steps
  // above); they are reloaded there from slice q_next, so most of the next
  // slice is in flight while this one finishes.  Not in cooperative items,
  // whose registers are full without it.
  auto compute = [&](F (&M)[NT][S4], int q_next) {
#pragma unroll
    for (int td = 0; td < NT; ++td) {
      V d1[NB][NTA];
      // column strips of the last a-tile: d1c[b][j] (full d-tile: lane
      // 16 g + 4 k + v = Y^T[16 td + 4 k + g][col 4 j + v]) and, in the last
      // d-tile run as row strips, d1cc[b][i][j] (every block = Y^T[16 td + 4 i
      // + g][col 4 j + v], already the replicated B operand of stage 2)
      F d1c[NB][RC], d1cc[NB][CS ? R : 1][RC];
      // stage 1: Y^T[d][a] = sum_c T[c][d] B^Q[c][a]   (d-tile td, every block)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int u = 0; u < NTA; ++u) d1[b][u] = V{0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < RC; ++j) {
          d1c[b][j] = F(0);
#pragma unroll
          for (int i = 0; i < (CS ? R : 1); ++i) d1cc[b][i][j] = F(0);
        }
#pragma unroll
        for (int s = 0; s < S4; ++s) {
          // B operand of a column strip: columns 4 j .. 4 j + 3 of the last
          // a-tile, broadcast to all four blocks
          F mb[RC];
          if constexpr (CS) {
#pragma unroll
            for (int j = 0; j < RC; ++j) mb[j] = bcast_strip(M[NT - 1][s], j);
          }
          if (STRIPS && td == NT - 1) {
            // strip i = k-step 4 td + i of stage 2; only the R strips with PNO rows
#pragma unroll
            for (int i = 0; i < R; ++i) {
              const F av = aop_strip(b, s, i);
#pragma unroll
              for (int u = 0; u < NTA; ++u) {
                if (CS && u == UL) continue;
                d1[b][u][i] = mfma_strip(av, M[ta(u)][s], d1[b][u][i]);
              }
              if constexpr (CS) {
#pragma unroll
                for (int j = 0; j < RC; ++j) d1cc[b][i][j] = mfma_strip(av, mb[j], d1cc[b][i][j]);
              }
            }
          } else {
            const F av = aop(b, td, s);
#pragma unroll
            for (int u = 0; u < NTA; ++u) {
              if (CS && u == UL) continue;
              d1[b][u] = Mfma<F>::op(av, M[ta(u)][s], d1[b][u]);
            }
            if constexpr (CS) {
#pragma unroll
              for (int j = 0; j < RC; ++j) d1c[b][j] = mfma_strip(av, mb[j], d1c[b][j]);
            }
          }
        }
      }
      if constexpr (W2 && !COOP && NT > 1) {
        if (td == NT - 1) loadM_steps(M, q_next, 0, 4 * (NT - 1));
      }
      // stage 2: Out^T[b][a] += sum_d B^Q[b][d] Y^T[d][a] over this d-tile
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (4 * td + i < S4) {
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if (mir(b)) {
#pragma unroll
              for (int tb = 0; tb < (STRIPS ? NT - 1 : NT); ++tb)
#pragma unroll
                for (int u = 0; u < NTA; ++u)
                  if (tb >= ta(u) && !(CS && u == UL))
                    acc[b][tb][u] = Mfma<F>::op(M[tb][4 * td + i], d1[b][u][i], acc[b][tb][u]);
            } else {
#pragma unroll
              for (int tb = 0; tb < (STRIPS ? NT - 1 : NT); ++tb)
#pragma unroll
                for (int u = 0; u < NTA; ++u)
                  if (!(CS && u == UL)) acc[b][tb][u] = Mfma<F>::op(M[tb][4 * td + i], d1[b][u][i], acc[b][tb][u]);
            }
          }
          if constexpr (STRIPS) {
            // last b-tile: output strip j holds rows 16 (NT - 1) + 4 j + g
#pragma unroll
            for (int j = 0; j < R; ++j) {
              const F mv = bcast_strip(M[NT - 1][4 * td + i], j);
#pragma unroll
              for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int u = 0; u < NTA; ++u)
                  if (!(CS && u == UL)) acc[b][NT - 1][u][j] = mfma_strip(mv, d1[b][u][i], acc[b][NT - 1][u][j]);
            }
          }
          if constexpr (CS) {
            // column strips of the last a-tile: every b-tile as 16 rows (the
            // last one included; its padded rows are never stored), B operand
            // = k-step i of the stage-1 strip, broadcast to all blocks
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
              for (int j = 0; j < RC; ++j) {
                const F yb = (STRIPS && td == NT - 1) ? d1cc[b][i < R ? i : 0][j] : bcast_strip(d1c[b][j], i);
#pragma unroll
                for (int tb = 0; tb < NT; ++tb)
                  if (!mir(b) || tb >= NT - 1) accC[b][tb][j] = mfma_strip(M[tb][4 * td + i], yb, accC[b][tb][j]);
              }
          }
        }
      }
      // keep each d-tile in its own scheduling region (bounded live ranges)
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  if constexpr (W2) {
    // two waves per SIMD: one B^Q buffer, most of the next slice loaded in
    // the last d-tile (the last slice reloads itself there, harmlessly); the
    // other wave covers the rest of the latency
    F M0[NT][S4];
    if constexpr (COOP || NT == 1) {
      for (int Q = it.lo; Q < it.hi; ++Q) {
        loadM(M0, Q);
        compute(M0, Q);
      }
    } else {
      loadM(M0, it.lo);
      for (int Q = it.lo; Q < it.hi; ++Q) {
        const int qn = Q + 1 < it.hi ? Q + 1 : Q;
        compute(M0, qn);
        loadM_steps(M0, qn, 4 * (NT - 1), S4);
      }
    }
  } else {
    F M0[NT][S4], M1[NT][S4];
    loadM(M0, it.lo);
    for (int Q = it.lo; Q < it.hi; Q += 2) {
      if (Q + 1 < it.hi) loadM(M1, Q + 1);
      compute(M0, 0);
      if (Q + 1 >= it.hi) break;
      if (Q + 2 < it.hi) loadM(M0, Q + 2);
      compute(M1, 0);
    }
  }

#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double* dst = A.ws + uni(A.blocks[blk0 + bslot0 + b].off_ws) + (int64_t)it.slot * nn;
    if constexpr (CS) {
      // the a-tiles before the last as 16x16 tiles, the last one from its strips
      if constexpr (NTA > 1) store_tiles_first<F, NT, NTA - 1, NTA>(dst, n, TA0, acc[b], mir(b), 1.0, DTA);
      const int kb = (lane >> 2) & 3, v = lane & 3;
#pragma unroll
      for (int tb = 0; tb < NT; ++tb) {
        if (mir(b) && tb < NT - 1) continue;       // written mirrored by the item of a-tile tb
        const int bb = 16 * tb + 4 * kb + g;
#pragma unroll
        for (int j = 0; j < RC; ++j) {
          const int a = 16 * (NT - 1) + 4 * j + v;
          if (a < n && bb < n) dst[bb * n + a] = (double)accC[b][tb][j];
        }
      }
    } else {
      store_tiles<F>(dst, n, TA0, acc[b], mir(b), 1.0, DTA);
    }
  }
}

// ---------------------------------------------------------------------------
// Projection item: target pair p (NT tiles), NB consecutive blocks, couplings
// [lo, hi) whose source pairs all have NQ tiles of 16.  Per coupling:
// M = S_{p,q}; per target block the term -w S_{p,q} op(T_q) S_{p,q}^T.  The
// source dimension is padded to 16 (zeros from the range-checked loads); with
// NQ fixed at compile time a coupling is one straight-line block.  A block
// without a term for this coupling runs with weight 0 and an empty operand
// range, which keeps the code branch-free.
// ---------------------------------------------------------------------------
template <typename F, int NT, int NB, int NQ, int MASK, bool W2 = false>
__device__ __forceinline__ void proj_item_direct(const GroupedArgs<F>& A, const Item& it, double* lds) {
  typedef typename Mfma<F>::V V;
  constexpr int S16 = 4 * NQ;                 // k-steps of 4 over the padded source index
  constexpr int SL = NQ * S16;                // LDS slots per term
  constexpr int LW = W2 ? kLdsWaveWords2 : kLdsWaveWords;
  static_assert(SL * 64 <= LW, "source operands exceed the wave's LDS");
  constexpr bool BATCH = NB * SL <= LW / 64;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4, pr = Mfma<F>::perm(r);
  const PairDev& Pg = A.pairs[it.pair];
  const int n = uni(Pg.n);
  const int blk0 = uni(Pg.blk0);
  F* Al = reinterpret_cast<F*>(lds + (size_t)(threadIdx.x >> 6) * LW);

  V acc[NB][NT][NT];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u) acc[b][t][u] = V{0, 0, 0, 0};
  // bit b of MASK: target block b is antisymmetric (its sources are same-spin
  // blocks too), so stage 2 runs only for tiles with tb >= ta
  auto mir = [](int b) { return ((MASK >> b) & 1) != 0; };

  for (int e = it.lo; e < it.hi; ++e) {
    const int nq = uni(A.cpl[e].nsrc);
    const int64_t off_S = uni(A.cpl[e].off_S);
    // M-form: M[t][s] = S_{p,q}[16t + r][4s + g] = W[(4s + g) n + 16t + r], W = [c][a]
    const __amdgpu_buffer_rsrc_t sr = rsrc(A.S + off_S, (uint32_t)(nq * n));
    const uint32_t mbase = (uint32_t)(g * n + r);
    F M[NT][S16];
#pragma unroll
    for (int s = 0; s < S16; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t) M[t][s] = Mfma<F>::load(sr, mbase + (uint32_t)(4 * s * n + 16 * t));

    auto load_x = [&](int b, int base_slot) {
      const TermDev& tg = A.terms[(int64_t)e * 4 + it.bslot0 + b];
      const int64_t src_off = uni(tg.src_off);
      const bool valid = src_off >= 0;
      const int trans = uni(tg.trans);
      const F mw = valid ? F(-uni(tg.w)) : F(0);
      const __amdgpu_buffer_rsrc_t xr = rsrc(A.T + (valid ? src_off : 0), valid ? (uint32_t)(nq * nq) : 0u);
      // Al[td][s] = X[4s + g][16 td + perm(r)], X = -w T_q or -w T_q^T
      const uint32_t base = trans ? (uint32_t)(pr * nq + g) : (uint32_t)(g * nq + pr);
      const uint32_t step_s = trans ? 4u : (uint32_t)(4 * nq);
      const uint32_t step_t = trans ? (uint32_t)(16 * nq) : 16u;
#pragma unroll
      for (int td = 0; td < NQ; ++td)
#pragma unroll
        for (int s = 0; s < S16; ++s)
          Al[(base_slot + td * S16 + s) * 64 + lane] =
              mw * Mfma<F>::load(xr, base + (uint32_t)s * step_s + (uint32_t)td * step_t);
    };
    // k-steps of the last source tile past the source's PNOs are skipped
    const int nq4 = (nq + 3) >> 2;
    auto compute_x = [&](int b, int base_slot) {
#pragma unroll
      for (int td = 0; td < NQ; ++td) {
        V d1[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) d1[u] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < S16; ++s) {
          if (s > 4 * (NQ - 1) && s >= nq4) continue;
          const F av = Al[(base_slot + td * S16 + s) * 64 + lane];
#pragma unroll
          for (int u = 0; u < NT; ++u) d1[u] = Mfma<F>::op(av, M[u][s], d1[u]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (4 * td + i > 4 * (NQ - 1) && 4 * td + i >= nq4) continue;
#pragma unroll
          for (int tb = 0; tb < NT; ++tb)
#pragma unroll
            for (int u = 0; u < NT; ++u)
              if (!mir(b) || u <= tb) acc[b][tb][u] = Mfma<F>::op(M[tb][4 * td + i], d1[u][i], acc[b][tb][u]);
        }
      }
    };
    if constexpr (BATCH) {
#pragma unroll
      for (int b = 0; b < NB; ++b) load_x(b, b * SL);
#pragma unroll
      for (int b = 0; b < NB; ++b) compute_x(b, b * SL);
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        load_x(b, 0);
        compute_x(b, 0);
      }
    }
  }

  const int64_t nn = (int64_t)n * n;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double* dst = A.ws + uni(A.blocks[blk0 + it.bslot0 + b].off_ws) + (int64_t)it.slot * nn;
    store_tiles<F>(dst, n, 0, acc[b], mir(b));
  }
}

// Pipelined projection item: the same contractions as proj_item_direct, with
// the loads of the next (coupling, block) unit issued before the current unit
// is contracted, so that one wave per SIMD hides its own memory latency.
// Per coupling the descriptors of the coupling after next are read, the
// next coupling's S operand is loaded into Mn during the last block, and the
// source amplitudes of the next unit are loaded into Xn; Xn is weighted and
// written to the LDS slab at the start of its unit.
template <typename F, int NT, int NB, int NQ, int MASK>
__device__ __forceinline__ void proj_item_pipelined(const GroupedArgs<F>& A, const Item& it, double* lds) {
  typedef typename Mfma<F>::V V;
  constexpr int S16 = 4 * NQ;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4, pr = Mfma<F>::perm(r);
  const PairDev& Pg = A.pairs[it.pair];
  const int n = uni(Pg.n);
  const int blk0 = uni(Pg.blk0);
  F* Al = reinterpret_cast<F*>(lds + (size_t)(threadIdx.x >> 6) * kLdsWaveWords);
  const uint32_t mbase = (uint32_t)(g * n + r);

  // Descriptors of one coupling packed in one VGPR: lane l holds dword l of
  // the coupling record (lanes 0..3) followed by its four term records (lanes
  // 4..27); fields are read with readlane where they are used.
  static_assert(sizeof(CplDev) == 16 && sizeof(TermDev) == 24, "descriptor layout");
  auto load_desc = [&](int e) -> int32_t {
    const int32_t* cw = reinterpret_cast<const int32_t*>(A.cpl + e);
    const int32_t* tw = reinterpret_cast<const int32_t*>(A.terms + (int64_t)e * 4);
    int32_t v = 0;
    if (lane < 4) v = cw[lane];
    else if (lane < 28) v = tw[lane - 4];
    return v;
  };
  auto rd32 = [](int32_t d, int k) -> int32_t { return __builtin_amdgcn_readlane(d, k); };
  auto rd64 = [](int32_t d, int k) -> int64_t {
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(d, k + 1) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane(d, k));
  };
  const int tb0 = 4 + 6 * it.bslot0;            // dword of the item's first term
  auto d_nq = [&](int32_t d) { return rd32(d, 1); };
  auto d_offS = [&](int32_t d) { return rd64(d, 2); };
  auto d_src = [&](int32_t d, int b) { return rd64(d, tb0 + 6 * b); };
  auto d_w = [&](int32_t d, int b) { return __builtin_bit_cast(double, rd64(d, tb0 + 6 * b + 2)); };
  auto d_trans = [&](int32_t d, int b) { return rd32(d, tb0 + 6 * b + 4); };

  // M-form of S_{p,q}: M[t][s] = W[(4s + g) n + 16t + r], W = [c][a]; an
  // empty resource (live = false) makes every load return 0
  auto load_M = [&](F (&M)[NT][S16], int32_t d, bool live) {
    const int nq = d_nq(d);
    const __amdgpu_buffer_rsrc_t sr = rsrc(A.S + d_offS(d), live ? (uint32_t)(nq * n) : 0u);
#pragma unroll
    for (int s = 0; s < S16; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t) M[t][s] = Mfma<F>::load(sr, mbase + (uint32_t)(4 * s * n + 16 * t));
  };
  // X-form of the source block of term b: X[4s + g][16 td + perm(r)], X = T_q or T_q^T
  auto load_X = [&](F (&X)[NQ][S16], int32_t d, int b, bool live) {
    const int64_t src = d_src(d, b);
    const bool valid = live && src >= 0;
    const int nq = d_nq(d);
    const __amdgpu_buffer_rsrc_t xr = rsrc(A.T + (valid ? src : 0), valid ? (uint32_t)(nq * nq) : 0u);
    const int trans = d_trans(d, b);
    const uint32_t base = trans ? (uint32_t)(pr * nq + g) : (uint32_t)(g * nq + pr);
    const uint32_t step_s = trans ? 4u : (uint32_t)(4 * nq);
    const uint32_t step_t = trans ? (uint32_t)(16 * nq) : 16u;
#pragma unroll
    for (int td = 0; td < NQ; ++td)
#pragma unroll
      for (int s = 0; s < S16; ++s) X[td][s] = Mfma<F>::load(xr, base + (uint32_t)s * step_s + (uint32_t)td * step_t);
  };
  // residual gets -w S X S^T; a block without a term for this coupling gets weight 0
  auto store_X = [&](const F (&X)[NQ][S16], int32_t d, int b) {
    const F mw = d_src(d, b) >= 0 ? F(-d_w(d, b)) : F(0);
#pragma unroll
    for (int td = 0; td < NQ; ++td)
#pragma unroll
      for (int s = 0; s < S16; ++s) Al[(td * S16 + s) * 64 + lane] = mw * X[td][s];
  };

  V acc[NB][NT][NT];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u) acc[b][t][u] = V{0, 0, 0, 0};
  // bit b of MASK: target block b is antisymmetric (its sources are same-spin
  // blocks too), so stage 2 runs only for tiles with tb >= ta
  auto mir = [](int b) { return ((MASK >> b) & 1) != 0; };

  // One unit's contractions.  nq4: k-steps of 4 over the source's PNOs; the
  // k-steps of the last 16-wide source tile past it (zero operands) are
  // skipped by wave-uniform branches.
  auto compute = [&](const F (&M)[NT][S16], int b, int nq4) {
#pragma unroll
    for (int td = 0; td < NQ; ++td) {
      V d1[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) d1[u] = V{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < S16; ++s) {
        if (s > 4 * (NQ - 1) && s >= nq4) continue;
        const F av = Al[(td * S16 + s) * 64 + lane];
#pragma unroll
        for (int u = 0; u < NT; ++u) d1[u] = Mfma<F>::op(av, M[u][s], d1[u]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (4 * td + i > 4 * (NQ - 1) && 4 * td + i >= nq4) continue;
#pragma unroll
        for (int tb = 0; tb < NT; ++tb)
#pragma unroll
          for (int u = 0; u < NT; ++u)
            if (!mir(b) || u <= tb) acc[b][tb][u] = Mfma<F>::op(M[tb][4 * td + i], d1[u][i], acc[b][tb][u]);
      }
    }
  };

  // prologue: descriptors of the first two couplings, operands of the first unit
  const int last = it.hi - 1;
  int32_t dc = load_desc(it.lo);
  int32_t dn = load_desc(it.lo + 1 <= last ? it.lo + 1 : last);
  F M[NT][S16], Mn[NT][S16], Xn[NQ][S16];
  load_M(M, dc, true);
  load_X(Xn, dc, 0, true);
  for (int e = it.lo; e <= last; ++e) {
    const bool more = e < last;
    const int32_t dnn = load_desc(e + 2 <= last ? e + 2 : last);
    const int nq4 = (d_nq(dc) + 3) >> 2;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      store_X(Xn, dc, b);
      if (b + 1 < NB) {
        load_X(Xn, dc, b + 1, true);
      } else {
        load_M(Mn, dn, more);
        load_X(Xn, dn, 0, more);
      }
      compute(M, b, nq4);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < S16; ++s) M[t][s] = Mn[t][s];
    dc = dn;
    dn = dnn;
  }

  const int64_t nn = (int64_t)n * n;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double* dst = A.ws + uni(A.blocks[blk0 + it.bslot0 + b].off_ws) + (int64_t)it.slot * nn;
    store_tiles<F>(dst, n, 0, acc[b], mir(b));
  }
}

// Projection item: pipelined where its registers (accumulators, two S
// operands, one block of source amplitudes, the stage-1 product; counted in
// operands) fit without spilling, direct otherwise.
// At two waves per SIMD (W2) the direct form: the other wave covers its
// latency, and the pipelined form's registers would not fit.
template <typename F, int NT, int NB, int NQ, int MASK, bool W2>
__device__ __forceinline__ void proj_item_m(const GroupedArgs<F>& A, const Item& it, double* lds) {
  constexpr int kRegs = 4 * NB * NT * NT + 2 * NT * 4 * NQ + 4 * NQ * NQ + 4 * NT;
  if constexpr (W2) proj_item_direct<F, NT, NB, NQ, MASK, true>(A, it, lds);
  else if constexpr (kRegs <= 170) proj_item_pipelined<F, NT, NB, NQ, MASK>(A, it, lds);
  else proj_item_direct<F, NT, NB, NQ, MASK>(A, it, lds);
}
// The antisymmetry pattern of the item's blocks selects a compiled body (see
// ladder_masked).
template <typename F, int NT, int NB, int NQ, bool W2 = false>
__device__ __forceinline__ void proj_item(const GroupedArgs<F>& A, const Item& it, double* lds) {
  int mask = 0;
  if (A.anti != 0) {
    const int blk0 = uni(A.pairs[it.pair].blk0);
#pragma unroll
    for (int b = 0; b < NB; ++b) mask |= (uni(A.blocks[blk0 + it.bslot0 + b].anti) != 0 ? 1 : 0) << b;
  }
  constexpr int kMirror = NB == 4 ? 3 : (1 << NB) - 1;
  if (mask == kMirror) proj_item_m<F, NT, NB, NQ, kMirror, W2>(A, it, lds);
  else proj_item_m<F, NT, NB, NQ, 0, W2>(A, it, lds);
}

// The antisymmetry pattern of the item's blocks selects a compiled body: for
// four blocks (AA, BB, AB, BA) the first two, otherwise all of them; any
// other pattern computes every tile.
template <typename F, int NT, int NB, int NTA, int TA0, int R, bool REG, bool W2>
__device__ __forceinline__ void ladder_masked(const GroupedArgs<F>& A, const Item& it, double* lds) {
  int mask = 0;
  if (A.anti != 0) {
    const int blk0 = uni(A.pairs[it.pair].blk0);
#pragma unroll
    for (int b = 0; b < NB; ++b) mask |= (uni(A.blocks[blk0 + it.bslot0 + b].anti) != 0 ? 1 : 0) << b;
  }
  constexpr int kMirror = NB == 4 ? 3 : (1 << NB) - 1;
  if (mask == kMirror) ladder_item<F, NT, NB, NTA, TA0, R, REG, kMirror, W2>(A, it, lds);
  else ladder_item<F, NT, NB, NTA, TA0, R, REG, 0, W2>(A, it, lds);
}

// k-steps of 4 in the last 16-wide tile of the pair: R = ceil((n mod 16) / 4), 1..4
#define DLPNO_LADDER_W(NT, NB, NTA, TA0, REG, W2)                                 \
  do {                                                                             \
    switch (rk) {                                                                  \
      case 1: ladder_masked<F, NT, NB, NTA, TA0, 1, REG, W2>(A, it, lds); break;   \
      case 2: ladder_masked<F, NT, NB, NTA, TA0, 2, REG, W2>(A, it, lds); break;   \
      case 3: ladder_masked<F, NT, NB, NTA, TA0, 3, REG, W2>(A, it, lds); break;   \
      default: ladder_masked<F, NT, NB, NTA, TA0, 4, REG, W2>(A, it, lds); break;  \
    }                                                                              \
  } while (0)
#define DLPNO_LADDER(NT, NB, NTA, TA0, REG) DLPNO_LADDER_W(NT, NB, NTA, TA0, REG, false)

template <typename F, int KIND>
__device__ __forceinline__ void run_item(const GroupedArgs<F>& A, const Item& it, double* lds) {
  if constexpr (KIND == ITEM_LADDER) {
    const int n = uni(A.pairs[it.pair].n);
    const int rem = n - 16 * ((n - 1) >> 4);     // 1..16 PNOs in the last tile
    const int rk = (rem + 3) >> 2;
    switch (it.variant) {
      case 0: DLPNO_LADDER(1, 4, 1, 0, true); break;
      case 1: DLPNO_LADDER(1, 2, 1, 0, true); break;
      case 2: DLPNO_LADDER(1, 1, 1, 0, true); break;
      case 3: DLPNO_LADDER(2, 4, 2, 0, false); break;
      case 4: DLPNO_LADDER(2, 2, 2, 0, true); break;
      case 5: DLPNO_LADDER(2, 1, 2, 0, true); break;
      case 6:
        if (it.ta0 == 0) DLPNO_LADDER(2, 4, 1, 0, true);
        else DLPNO_LADDER(2, 4, 1, 1, true);
        break;
      case 7: DLPNO_LADDER(3, 1, 3, 0, false); break;
      case 8:
        if (it.ta0 == 0) DLPNO_LADDER(4, 1, 2, 0, false);
        else DLPNO_LADDER(4, 1, 2, 2, false);
        break;
      default: no_body(A.err); break;
    }
  } else if constexpr (KIND == ITEM_LADDER2) {
    // items of at most three tiles at two waves per SIMD: variants whose X
    // operands fit the smaller LDS slab or the smaller register budget
    const int n = uni(A.pairs[it.pair].n);
    const int rem = n - 16 * ((n - 1) >> 4);
    const int rk = (rem + 3) >> 2;
    switch (it.variant) {
      case 0: DLPNO_LADDER_W(1, 4, 1, 0, true, true); break;
      case 1: DLPNO_LADDER_W(1, 2, 1, 0, true, true); break;
      case 2: DLPNO_LADDER_W(1, 1, 1, 0, true, true); break;
      case 4: DLPNO_LADDER_W(2, 2, 2, 0, false, true); break;
      case 5: DLPNO_LADDER_W(2, 1, 2, 0, false, true); break;
      case 7: DLPNO_LADDER_W(3, 1, 3, 0, false, true); break;
      default: no_body(A.err); break;
    }
  } else if constexpr (KIND == ITEM_PROJ2) {
    // projection items at two waves per SIMD: target and sources of at most
    // three tiles, variants whose registers fit 256 per lane
#define DLPNO_PROJ2(V, NT, NB)                                                       \
  case 4 * V + 0: proj_item<F, NT, NB, 1, true>(A, it, lds); break;                  \
  case 4 * V + 1: proj_item<F, NT, NB, 2, true>(A, it, lds); break;                  \
  case 4 * V + 2: proj_item<F, NT, NB, 3, true>(A, it, lds); break;
    switch (it.variant) {
      DLPNO_PROJ2(0, 1, 4)
      DLPNO_PROJ2(1, 1, 2)
      DLPNO_PROJ2(2, 1, 1)
      DLPNO_PROJ2(4, 2, 2)
      DLPNO_PROJ2(5, 2, 1)
      DLPNO_PROJ2(7, 3, 1)
      default: no_body(A.err); break;
    }
#undef DLPNO_PROJ2
  } else {
    // variant = 4 * (tile variant) + (source tiles - 1)
#define DLPNO_PROJ(V, NT, NB)                                                        \
  case 4 * V + 0: proj_item<F, NT, NB, 1>(A, it, lds); break;                        \
  case 4 * V + 1: proj_item<F, NT, NB, 2>(A, it, lds); break;                        \
  case 4 * V + 2: proj_item<F, NT, NB, 3>(A, it, lds); break;                        \
  case 4 * V + 3: proj_item<F, NT, NB, 4>(A, it, lds); break;
    switch (it.variant) {
      DLPNO_PROJ(0, 1, 4)
      DLPNO_PROJ(1, 1, 2)
      DLPNO_PROJ(2, 1, 1)
      DLPNO_PROJ(3, 2, 4)
      DLPNO_PROJ(4, 2, 2)
      DLPNO_PROJ(5, 2, 1)
      // three target tiles, two blocks: up to three source tiles (the
      // schedule gives four-tile sources one block per item)
      case 4 * 6 + 0: proj_item<F, 3, 2, 1>(A, it, lds); break;
      case 4 * 6 + 1: proj_item<F, 3, 2, 2>(A, it, lds); break;
      case 4 * 6 + 2: proj_item<F, 3, 2, 3>(A, it, lds); break;
      DLPNO_PROJ(7, 3, 1)
      DLPNO_PROJ(8, 4, 1)
      default: no_body(A.err); break;
    }
#undef DLPNO_PROJ
  }
}
#undef DLPNO_LADDER
#undef DLPNO_LADDER_W

// Cooperative four-tile ladder item, run by one workgroup: the item has nbi
// (1 or 2) blocks; waves 2h and 2h + 1 take block h, two a-tiles each: {0, 3}
// and {1, 2} when the block is antisymmetric (five stage-2 tiles each), {0, 1}
// and {2, 3} otherwise.  Waves without a block go straight to the next
// barrier of the launch loop.
template <typename F, int R>
__device__ __forceinline__ void ladder_coop(const GroupedArgs<F>& A, const Item& it, int nbi, double* lds) {
  const int wave = threadIdx.x >> 6, h = wave >> 1, odd = wave & 1;
  if (h >= nbi) return;
  const int blk0 = uni(A.pairs[it.pair].blk0);
  const bool mirror = A.anti != 0 && uni(A.blocks[blk0 + it.bslot0 + h].anti) != 0;
  if (mirror) {
    if (odd) ladder_item<F, 4, 1, 2, 1, R, false, 1, true, 1, true>(A, it, lds);
    else ladder_item<F, 4, 1, 2, 0, R, false, 1, true, 3, true>(A, it, lds);
  } else {
    if (odd) ladder_item<F, 4, 1, 2, 2, R, false, 0, true, 1, true>(A, it, lds);
    else ladder_item<F, 4, 1, 2, 0, R, false, 0, true, 1, true>(A, it, lds);
  }
}

__device__ __forceinline__ Item read_item(const Item& ig) {
  Item it;
  it.kind = uni(ig.kind);
  it.variant = uni(ig.variant);
  it.pair = uni(ig.pair);
  it.bslot0 = uni(ig.bslot0);
  it.slot = uni(ig.slot);
  it.ta0 = uni(ig.ta0);
  it.lo = uni(ig.lo);
  it.hi = uni(ig.hi);
  return it;
}

// One launch processes the items of one kind (KIND), so that the ladder and
// projection bodies are register-allocated separately.
template <typename F, int KIND>
__global__ __launch_bounds__(256, KIND == ITEM_LADDER2 || KIND == ITEM_PROJ2 ? 2 : 1) void grouped_kernel(
    GroupedArgs<F> A) {
  __shared__ double lds[4 * (KIND == ITEM_LADDER2 || KIND == ITEM_PROJ2 ? kLdsWaveWords2 : kLdsWaveWords)];
  int q = blockIdx.x % kQueues, left = kQueues;
  for (;;) {
    const int idx = next_item(A.q, q, left);
    if (idx < 0) break;
    run_item<F, KIND>(A, read_item(A.items[idx]), lds);
  }
}

// Cooperative launch over the four-tile ladder items (ITEM_LADDER4), two
// workgroups per CU.  Wave 0 pops an item for its workgroup and passes it on
// through LDS between two barriers; every wave passes both barriers of every
// round, and all leave the loop in the same round.
template <typename F>
__global__ __launch_bounds__(256, 2) void grouped_coop_kernel(GroupedArgs<F> A) {
  __shared__ double lds[2 * kCoopSlabWords];
  __shared__ int32_t next;
  int q = blockIdx.x % kQueues, left = kQueues;
  for (;;) {
    __syncthreads();                     // the previous item's slabs are free
    if (threadIdx.x < 64) {
      const int i = next_item(A.q, q, left);
      if (threadIdx.x == 0) next = i;
    }
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(next);
    if (idx < 0) break;
    const Item it = read_item(A.items[idx]);
    const int n = uni(A.pairs[it.pair].n);
    const int rk = (n - 16 * ((n - 1) >> 4) + 3) >> 2;
    const int nbi = it.variant == kLadderCoopPair ? 2 : 1;
    switch (rk) {
      case 1: ladder_coop<F, 1>(A, it, nbi, lds); break;
      case 2: ladder_coop<F, 2>(A, it, nbi, lds); break;
      case 3: ladder_coop<F, 3>(A, it, nbi, lds); break;
      default: ladder_coop<F, 4>(A, it, nbi, lds); break;
    }
  }
}

}  // namespace dlpno
