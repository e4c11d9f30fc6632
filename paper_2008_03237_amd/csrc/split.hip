// Split-precision (BF16x2 / FP16x2) ladder and projection contractions.
//
// Every operand x is carried as hi + lo with hi = round(x), lo = round(x - hi)
// in BF16 or FP16, and a product as hi*hi + hi*lo + lo*hi on the 16x16x32
// MFMA (two 16-wide inner tiles per instruction) with FP32 accumulation (the lo*lo term is below the FP32 accumulation
// error).  This keeps about 16 (BF16) or 22 (FP16) significant bits per
// operand while the lo half stays a normal number; the FP64 refinement
// driver (mixed.hip) recovers full accuracy.  FP16 needs power-of-two
// scaling: per pair for B, per block for the amplitudes, and per projection
// item and target block for the weighted stage-1 products; BF16 has the FP32
// exponent range and runs unscaled.
//
// Split operands are stored in zero-padded layouts whose rows are 16-element
// multiples, so every 16x16x16 fragment (4 consecutive inner-index elements
// per lane, one 8-byte load) is either inside the matrix or an exact zero:
//   B_p     per Q: [a][c], n rows x N16 columns          (symmetric B^Q)
//   S_pq    [a][c], n_target rows x N16(n_src) columns   (target x source)
//   T_blk   two copies: T^T [d][c] and T [c][d], n rows x N16 columns
// The accumulator keeps output row 4 g + i in register i of lane group g,
// which is exactly the inner-index order of a 4-element fragment of the next
// product's B operand, so Y^T = X^T M^T is converted to hi/lo in registers and
// fed to Out^T = M Y^T without leaving the VGPRs; two d-tiles make one K = 32
// operand.  Only the K = 32 shape is used: on gfx950 the K = 16 form takes the
// same time per instruction, and chaining the two shapes on one accumulator is
// emitted without the wait states it needs (measured: wrong sums), so odd
// tiles are padded with zero fragments instead.
#include "grouped_impl.h"
#include "plan_internal.h"
#include "split_internal.h"

namespace dlpno {

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef unsigned long long u2_t __attribute__((ext_vector_type(2)));

struct SplitBf16 {
  typedef uint16_t E;
  static __device__ __forceinline__ E cvt(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
  static __device__ __forceinline__ float back(E e) { return (float)__builtin_bit_cast(__bf16, e); }
  static __device__ __forceinline__ f4_t mfma(uint64_t a, uint64_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4_t, a), __builtin_bit_cast(s4_t, b), c, 0,
                                                     0, 0);
  }
  // K = 32 from two K = 16 fragments (the same element order in both operands)
  static __device__ __forceinline__ f4_t mfma32(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8_t, u2_t{a0, a1}),
                                                   __builtin_bit_cast(b8_t, u2_t{b0, b1}), c, 0, 0, 0);
  }
};
struct SplitF16 {
  typedef uint16_t E;
  static __device__ __forceinline__ E cvt(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
  static __device__ __forceinline__ float back(E e) { return (float)__builtin_bit_cast(_Float16, e); }
  static __device__ __forceinline__ f4_t mfma(uint64_t a, uint64_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4_t, a), __builtin_bit_cast(h4_t, b), c, 0, 0,
                                                 0);
  }
  static __device__ __forceinline__ f4_t mfma32(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8_t, u2_t{a0, a1}),
                                                  __builtin_bit_cast(h8_t, u2_t{b0, b1}), c, 0, 0, 0);
  }
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc16(const uint16_t* p, uint32_t elems) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(uni(p)), (short)0, (uint32_t)uni((int32_t)(elems * 2u)),
                                           0x00020000);
}
__device__ __forceinline__ uint64_t frag(__amdgpu_buffer_rsrc_t r, uint32_t off_elems) {
  return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, off_elems * 2u, 0u, 0));
}

// hi/lo of 4 FP32 values packed as two 4-element fragments
template <typename S>
__device__ __forceinline__ void split4(const f4_t v, float scale, uint64_t& hi, uint64_t& lo);
// BF16: packed conversions of element pairs (round to nearest even); a BF16
// value back in FP32 is its bits shifted into the high half
typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));
template <>
__device__ __forceinline__ void split4<SplitBf16>(const f4_t v, float scale, uint64_t& hi, uint64_t& lo) {
  uint32_t h[2], l[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float x0 = v[2 * j] * scale, x1 = v[2 * j + 1] * scale;
    h[j] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{x0, x1}, b2_t));
    const float b0 = __builtin_bit_cast(float, h[j] << 16), b1 = __builtin_bit_cast(float, h[j] & 0xffff0000u);
    l[j] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{x0 - b0, x1 - b1}, b2_t));
  }
  hi = ((uint64_t)h[1] << 32) | h[0];
  lo = ((uint64_t)l[1] << 32) | l[0];
}
template <typename S>
__device__ __forceinline__ void split4(const f4_t v, float scale, uint64_t& hi, uint64_t& lo) {
  uint64_t h = 0, l = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float x = v[j] * scale;
    const typename S::E eh = S::cvt(x);
    const typename S::E el = S::cvt(x - S::back(eh));
    h |= (uint64_t)eh << (16 * j);
    l |= (uint64_t)el << (16 * j);
  }
  hi = h;
  lo = l;
}

template <typename S>
__device__ __forceinline__ f4_t mfma3(uint64_t ah, uint64_t al, uint64_t bh, uint64_t bl, f4_t c) {
  c = S::mfma(ah, bh, c);
  c = S::mfma(ah, bl, c);
  c = S::mfma(al, bh, c);
  return c;
}
// two adjacent 16-wide inner tiles as one K = 32 product (hi*hi + hi*lo + lo*hi)
template <typename S>
__device__ __forceinline__ f4_t mfma3x2(uint64_t ah0, uint64_t ah1, uint64_t al0, uint64_t al1, uint64_t bh0,
                                        uint64_t bh1, uint64_t bl0, uint64_t bl1, f4_t c) {
  c = S::mfma32(ah0, ah1, bh0, bh1, c);
  c = S::mfma32(ah0, ah1, bl0, bl1, c);
  c = S::mfma32(al0, al1, bh0, bh1, c);
  return c;
}

// ---------------------------------------------------------------------------
// ladder item (same schedule as the FP64 kernel; NT inner tiles of 16)
// ---------------------------------------------------------------------------
template <typename S, int NT, int NB, int NTA, int TA0, int MASK>
__device__ __forceinline__ void split_ladder_item(const SplitArgs& A, const Item& it) {
  // bit b of MASK: block b antisymmetric, stage 2 only for tiles with tb >= ta
  auto mir = [](int b) { return ((MASK >> b) & 1) != 0; };
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const PairDev& Pg = A.pairs[it.pair];
  const int n = uni(Pg.n);
  const int blk0 = uni(Pg.blk0);
  const int n16 = 16 * NT;
  const uint32_t slice = (uint32_t)n * (uint32_t)n16;
  const int64_t boff = uni(A.pair_boff[it.pair]);
  const float bs = A.pair_bscale ? __builtin_bit_cast(float, uni(__builtin_bit_cast(int32_t, A.pair_bscale[it.pair]))) : 1.f;

  // amplitude fragments (T^T layout): Af[b][td][kt] = T^T[16 td + r][16 kt + 4 g .. +3]
  uint64_t Ah[NB][NT][NT], Alo[NB][NT][NT];
  float unscale[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int blk = blk0 + it.bslot0 + b;
    const int64_t toff = uni(A.blk_toff[blk]);
    const float ts = A.blk_tscale ? __builtin_bit_cast(float, uni(__builtin_bit_cast(int32_t, A.blk_tscale[blk]))) : 1.f;
    unscale[b] = 1.f / (ts * bs * bs);
    const __amdgpu_buffer_rsrc_t rh = rsrc16(A.Tt_hi + toff, slice);
    const __amdgpu_buffer_rsrc_t rl = rsrc16(A.Tt_lo + toff, slice);
#pragma unroll
    for (int td = 0; td < NT; ++td)
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) {
        const uint32_t o = (uint32_t)((16 * td + r) * n16 + 16 * kt + 4 * g);
        Ah[b][td][kt] = frag(rh, o);
        Alo[b][td][kt] = frag(rl, o);
      }
  }
  f4_t acc[NB][NT][NTA];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < NTA; ++u) acc[b][t][u] = f4_t{0, 0, 0, 0};

  // B^Q fragments: M[t][kt] = B^Q[16 t + r][16 kt + 4 g .. +3].  One slice is
  // only a few hundred cycles of MFMA work here, so QB slices are loaded per
  // batch and the next batch is in flight while the current one is used.
  constexpr int QB = NT == 1 ? 8 : NT == 2 ? 4 : NT == 3 ? 2 : 1;
  auto loadM = [&](uint64_t (&Mh)[QB][NT][NT], uint64_t (&Ml)[QB][NT][NT], int Q0) {
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      // slices past the item's range read as zeros (empty resource)
      const bool in = Q0 + q < it.hi;
      const __amdgpu_buffer_rsrc_t rh = rsrc16(A.B_hi + boff + (size_t)(in ? Q0 + q : 0) * slice, in ? slice : 0u);
      const __amdgpu_buffer_rsrc_t rl = rsrc16(A.B_lo + boff + (size_t)(in ? Q0 + q : 0) * slice, in ? slice : 0u);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) {
          const uint32_t o = (uint32_t)((16 * t + r) * n16 + 16 * kt + 4 * g);
          Mh[q][t][kt] = frag(rh, o);
          Ml[q][t][kt] = frag(rl, o);
        }
    }
  };
  // stage 1 for d-tile td: Y^T[d][a] over the inner index in K = 32 pairs of tiles
  auto stage1 = [&](const uint64_t (&Mh)[NT][NT], const uint64_t (&Ml)[NT][NT], int b, int td, int u) -> f4_t {
    f4_t c = f4_t{0, 0, 0, 0};
#pragma unroll
    for (int kp = 0; kp + 1 < NT; kp += 2)
      c = mfma3x2<S>(Ah[b][td][kp], Ah[b][td][kp + 1], Alo[b][td][kp], Alo[b][td][kp + 1], Mh[TA0 + u][kp],
                     Mh[TA0 + u][kp + 1], Ml[TA0 + u][kp], Ml[TA0 + u][kp + 1], c);
    if constexpr (NT % 2 == 1)   // odd tail: K = 32 with a zero upper half (never mix MFMA shapes on one accumulator)
      c = mfma3x2<S>(Ah[b][td][NT - 1], 0, Alo[b][td][NT - 1], 0, Mh[TA0 + u][NT - 1], 0, Ml[TA0 + u][NT - 1], 0, c);
    return c;
  };
  auto compute = [&](const uint64_t (&Mh)[NT][NT], const uint64_t (&Ml)[NT][NT]) {
    // d-tiles in pairs: the two stage-1 tiles form one K = 32 operand of stage 2
#pragma unroll
    for (int tp = 0; tp + 1 < NT; tp += 2) {
      uint64_t yh[NB][NTA][2], yl[NB][NTA][2];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int u = 0; u < NTA; ++u)
#pragma unroll
          for (int h = 0; h < 2; ++h) split4<S>(stage1(Mh, Ml, b, tp + h, u), 1.f, yh[b][u][h], yl[b][u][h]);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int u = 0; u < NTA; ++u)
#pragma unroll
          for (int tb = 0; tb < NT; ++tb)
            if (!mir(b) || tb >= TA0 + u)
              acc[b][tb][u] = mfma3x2<S>(Mh[tb][tp], Mh[tb][tp + 1], Ml[tb][tp], Ml[tb][tp + 1], yh[b][u][0],
                                         yh[b][u][1], yl[b][u][0], yl[b][u][1], acc[b][tb][u]);
    }
    if constexpr (NT % 2 == 1) {
      constexpr int td = NT - 1;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int u = 0; u < NTA; ++u) {
          uint64_t yh, yl;
          split4<S>(stage1(Mh, Ml, b, td, u), 1.f, yh, yl);
#pragma unroll
          for (int tb = 0; tb < NT; ++tb)
            if (!mir(b) || tb >= TA0 + u)
              acc[b][tb][u] = mfma3x2<S>(Mh[tb][td], 0, Ml[tb][td], 0, yh, 0, yl, 0, acc[b][tb][u]);
        }
    }
  };
  auto compute_batch = [&](const uint64_t (&Mh)[QB][NT][NT], const uint64_t (&Ml)[QB][NT][NT], int Q0) {
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      if (Q0 + q < it.hi) compute(Mh[q], Ml[q]);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  uint64_t M0h[QB][NT][NT], M0l[QB][NT][NT], M1h[QB][NT][NT], M1l[QB][NT][NT];
  loadM(M0h, M0l, it.lo);
  for (int Q = it.lo; Q < it.hi; Q += 2 * QB) {
    if (Q + QB < it.hi) loadM(M1h, M1l, Q + QB);
    compute_batch(M0h, M0l, Q);
    if (Q + QB >= it.hi) break;
    if (Q + 2 * QB < it.hi) loadM(M0h, M0l, Q + 2 * QB);
    compute_batch(M1h, M1l, Q + QB);
  }
  const int64_t nn = (int64_t)n * n;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double* dst = A.ws + uni(A.blocks[blk0 + it.bslot0 + b].off_ws) + (int64_t)it.slot * nn;
    // FP32 accumulator layout: row 4 g + i
    store_tiles<float>(dst, n, TA0, acc[b], mir(b), (double)unscale[b]);
  }
}

// ---------------------------------------------------------------------------
// projection item: per coupling S fragments, per term source fragments
// ---------------------------------------------------------------------------
template <typename S, int NT, int NB, int MASK>
__device__ __forceinline__ void split_proj_item(const SplitArgs& A, const Item& it) {
  auto mir = [](int b) { return ((MASK >> b) & 1) != 0; };
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const PairDev& Pg = A.pairs[it.pair];
  const int n = uni(Pg.n);
  const int blk0 = uni(Pg.blk0);
  float tscale[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
    tscale[b] = A.blk_tscale
                    ? __builtin_bit_cast(float, uni(__builtin_bit_cast(int32_t, A.blk_tscale[blk0 + it.bslot0 + b])))
                    : 1.f;
  // FP16: the stage-1 product Y of a term is split after scaling by
  // -w tscale / qs (Fock weight, target over source block scale).  Those
  // factors span orders of magnitude, so per target block they are first
  // normalised by a power of two psc that puts the item's largest one in
  // [256, 512): |Y| <= n_q * 512 < 65504 (|S| <= 1, scaled |X| <= 1), so the
  // hi half cannot overflow, and the dominant terms keep their lo halves out
  // of the FP16 subnormals.  The accumulator is unscaled by tscale * psc.
  float psc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) psc[b] = 1.f;
  if (A.blk_tscale) {
    float wmax[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) wmax[b] = 0.f;
    for (int e = it.lo; e < it.hi; ++e) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const TermDev& tg = A.terms[(int64_t)e * 4 + it.bslot0 + b];
        if (uni(tg.src_off) < 0) continue;
        const float qs = __builtin_bit_cast(float, uni(__builtin_bit_cast(int32_t, A.blk_tscale[uni(tg.src_blk)])));
        wmax[b] = fmaxf(wmax[b], fabsf((float)uni(tg.w)) * (tscale[b] / qs));
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (wmax[b] > 0.f) {
        int ex;
        (void)frexpf(wmax[b], &ex);
        psc[b] = ldexpf(1.f, min(100, max(-100, 9 - ex)));
      }
    }
  }
  f4_t acc[NB][NT][NT];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u) acc[b][t][u] = f4_t{0, 0, 0, 0};

  for (int e = it.lo; e < it.hi; ++e) {
    const int nq = uni(A.cpl[e].nsrc);
    const int NQ = (nq + 15) >> 4;
    const int nq16 = 16 * NQ;
    const int64_t soff = uni(A.cpl_soff[e]);
    const __amdgpu_buffer_rsrc_t sh = rsrc16(A.S_hi + soff, (uint32_t)(n * nq16));
    const __amdgpu_buffer_rsrc_t sl = rsrc16(A.S_lo + soff, (uint32_t)(n * nq16));
    // S_{p,q} fragments: M[t][kt] = S[16 t + r][16 kt + 4 g .. +3]
    uint64_t Mh[NT][4], Ml[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        if (kt < NQ) {
          const uint32_t o = (uint32_t)((16 * t + r) * nq16 + 16 * kt + 4 * g);
          Mh[t][kt] = frag(sh, o);
          Ml[t][kt] = frag(sl, o);
        } else {
          Mh[t][kt] = 0;
          Ml[t][kt] = 0;
        }
      }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const TermDev& tg = A.terms[(int64_t)e * 4 + it.bslot0 + b];
      const int64_t src_off = uni(tg.src_off);
      if (src_off < 0) continue;
      const int sblk = uni(tg.src_blk);
      const int trans = uni(tg.trans);
      const float w = (float)uni(tg.w);
      const float qs = A.blk_tscale ? __builtin_bit_cast(float, uni(__builtin_bit_cast(int32_t, A.blk_tscale[sblk]))) : 1.f;
      // X^T fragments: X = T_q (take the T^T copy) or X = T_q^T (take the T copy)
      const int64_t toff = uni(A.blk_toff[sblk]);
      const uint16_t* xh = trans ? A.T_hi : A.Tt_hi;
      const uint16_t* xl = trans ? A.T_lo : A.Tt_lo;
      const __amdgpu_buffer_rsrc_t xrh = rsrc16(xh + toff, (uint32_t)(nq * nq16));
      const __amdgpu_buffer_rsrc_t xrl = rsrc16(xl + toff, (uint32_t)(nq * nq16));
      // rescale Y to the target block's scale with the Fock weight folded in
      // (and the item's power-of-two normalisation, FP16)
      const float ysc = -w * (tscale[b] / qs) * psc[b];
      // source d-tiles in pairs (one K = 32 operand of stage 2); every product
      // is a K = 32 MFMA, absent tiles are zero fragments
#pragma unroll
      for (int tp = 0; tp < 4; tp += 2) {
        if (tp < NQ) {
          uint64_t yh[NT][2], yl[NT][2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int td = tp + h;
            uint64_t Xh[4], Xl[4];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
              if (td < NQ && kt < NQ) {
                const uint32_t o = (uint32_t)((16 * td + r) * nq16 + 16 * kt + 4 * g);
                Xh[kt] = frag(xrh, o);
                Xl[kt] = frag(xrl, o);
              } else {
                Xh[kt] = 0;
                Xl[kt] = 0;
              }
            }
#pragma unroll
            for (int u = 0; u < NT; ++u) {
              f4_t c = f4_t{0, 0, 0, 0};
#pragma unroll
              for (int kp = 0; kp < 4; kp += 2)
                if (kp < NQ)
                  c = mfma3x2<S>(Xh[kp], Xh[kp + 1], Xl[kp], Xl[kp + 1], Mh[u][kp], Mh[u][kp + 1], Ml[u][kp],
                                 Ml[u][kp + 1], c);
              split4<S>(c, ysc, yh[u][h], yl[u][h]);
            }
          }
#pragma unroll
          for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
              if (!mir(b) || tb >= u)
                acc[b][tb][u] = mfma3x2<S>(Mh[tb][tp], Mh[tb][tp + 1], Ml[tb][tp], Ml[tb][tp + 1], yh[u][0],
                                           yh[u][1], yl[u][0], yl[u][1], acc[b][tb][u]);
        }
      }
    }
  }
  const int64_t nn = (int64_t)n * n;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double* dst = A.ws + uni(A.blocks[blk0 + it.bslot0 + b].off_ws) + (int64_t)it.slot * nn;
    store_tiles<float>(dst, n, 0, acc[b], mir(b), 1.0 / ((double)tscale[b] * (double)psc[b]));
  }
}

// the antisymmetry pattern of the item's blocks selects a compiled body (as
// in the FP64 kernel: four blocks AA, BB, AB, BA mirror the first two)
__device__ __forceinline__ int split_mask(const SplitArgs& A, const Item& it, int nb) {
  if (A.anti == 0) return 0;
  const int blk0 = uni(A.pairs[it.pair].blk0);
  int mask = 0;
  for (int b = 0; b < nb; ++b) mask |= (uni(A.blocks[blk0 + it.bslot0 + b].anti) != 0 ? 1 : 0) << b;
  const int mirror = nb == 4 ? 3 : (1 << nb) - 1;
  return mask == mirror ? mirror : 0;
}
template <typename S, int NT, int NB, int NTA, int TA0>
__device__ __forceinline__ void split_ladder_masked(const SplitArgs& A, const Item& it) {
  constexpr int kMirror = NB == 4 ? 3 : (1 << NB) - 1;
  if (split_mask(A, it, NB) == kMirror) split_ladder_item<S, NT, NB, NTA, TA0, kMirror>(A, it);
  else split_ladder_item<S, NT, NB, NTA, TA0, 0>(A, it);
}
template <typename S, int NT, int NB>
__device__ __forceinline__ void split_proj_masked(const SplitArgs& A, const Item& it) {
  constexpr int kMirror = NB == 4 ? 3 : (1 << NB) - 1;
  if (split_mask(A, it, NB) == kMirror) split_proj_item<S, NT, NB, kMirror>(A, it);
  else split_proj_item<S, NT, NB, 0>(A, it);
}

template <typename S, int KIND>
__device__ __forceinline__ void split_run_item(const SplitArgs& A, const Item& it) {
  if constexpr (KIND == ITEM_LADDER) {
    switch (it.variant) {
      case 0: split_ladder_masked<S, 1, 4, 1, 0>(A, it); break;
      case 1: split_ladder_masked<S, 1, 2, 1, 0>(A, it); break;
      case 2: split_ladder_masked<S, 1, 1, 1, 0>(A, it); break;
      case 3: split_ladder_masked<S, 2, 4, 2, 0>(A, it); break;
      case 4: split_ladder_masked<S, 2, 2, 2, 0>(A, it); break;
      case 5: split_ladder_masked<S, 2, 1, 2, 0>(A, it); break;
      case 6:
        if (it.ta0 == 0) split_ladder_masked<S, 2, 4, 1, 0>(A, it);
        else split_ladder_masked<S, 2, 4, 1, 1>(A, it);
        break;
      case 7: split_ladder_masked<S, 3, 1, 3, 0>(A, it); break;
      case 8:
        if (it.ta0 == 0) split_ladder_masked<S, 4, 1, 2, 0>(A, it);
        else split_ladder_masked<S, 4, 1, 2, 2>(A, it);
        break;
      case 11: split_ladder_masked<S, 3, 2, 3, 0>(A, it); break;
      case 12:
        if (it.ta0 == 0) split_ladder_masked<S, 4, 2, 2, 0>(A, it);
        else split_ladder_masked<S, 4, 2, 2, 2>(A, it);
        break;
      default: no_body(A.err); break;
    }
  } else {
    switch (it.variant >> 2) {     // variant = 4 * (tile variant) + (source tiles - 1)
      case 0: split_proj_masked<S, 1, 4>(A, it); break;
      case 1: split_proj_masked<S, 1, 2>(A, it); break;
      case 2: split_proj_masked<S, 1, 1>(A, it); break;
      case 3: split_proj_masked<S, 2, 4>(A, it); break;
      case 4: split_proj_masked<S, 2, 2>(A, it); break;
      case 5: split_proj_masked<S, 2, 1>(A, it); break;
      case 6: split_proj_masked<S, 3, 2>(A, it); break;
      case 7: split_proj_masked<S, 3, 1>(A, it); break;
      case 8: split_proj_masked<S, 4, 1>(A, it); break;
      default: no_body(A.err); break;
    }
  }
}

// one launch per item kind (separate register allocation), as in the FP64
// kernel; the projection launch fits two waves per SIMD (it uses no LDS and
// fewer than 256 registers per lane), which hides more of its load latency
template <typename S, int KIND>
__global__ __launch_bounds__(256, KIND == ITEM_PROJ ? 2 : 1) void split_grouped_kernel(SplitArgs A) {
  int q = blockIdx.x % kQueues, left = kQueues;
  for (;;) {
    const int idx = next_item(A.q, q, left);
    if (idx < 0) break;
    const Item& ig = A.items[idx];
    Item it;
    it.kind = uni(ig.kind);
    it.variant = uni(ig.variant);
    it.pair = uni(ig.pair);
    it.bslot0 = uni(ig.bslot0);
    it.slot = uni(ig.slot);
    it.ta0 = uni(ig.ta0);
    it.lo = uni(ig.lo);
    it.hi = uni(ig.hi);
    split_run_item<S, KIND>(A, it);
  }
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ void split_d(double x, uint16_t& h, uint16_t& l) {
  const typename S::E eh = S::cvt((float)x);
  const typename S::E el = S::cvt((float)(x - (double)S::back(eh)));
  h = eh;
  l = el;
}

__device__ __forceinline__ float pow2_scale(double amax) {
  // power of two s with amax * s in [0.5, 1); 1 when amax is zero
  if (!(amax > 0.0)) return 1.f;
  int e;
  (void)frexp(amax, &e);
  return ldexpf(1.f, -e);
}

__device__ __forceinline__ double block_max(double v) {
  __shared__ double sm[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  v = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
  __syncthreads();
  return v;
}

// B_p (FP64 [Q][a][c]) -> padded split copy, one workgroup per pair
template <typename S>
__global__ __launch_bounds__(256) void split_B_kernel(const PairDev* pairs, const double* B, const int64_t* boff,
                                                      float* bscale, uint16_t* hi, uint16_t* lo, int scaled) {
  const PairDev P = pairs[blockIdx.x];
  if (P.nblk == 0) return;
  const int n = P.n, n16 = 16 * ((n + 15) / 16);
  const int64_t total = (int64_t)P.m * n * n;
  const double* src = B + P.off_B;
  float sc = 1.f;
  if (scaled) {
    double mx = 0.0;
    for (int64_t x = threadIdx.x; x < total; x += 256) mx = fmax(mx, fabs(src[x]));
    sc = pow2_scale(block_max(mx));
    if (threadIdx.x == 0) bscale[blockIdx.x] = sc;
  }
  const int64_t tot16 = (int64_t)P.m * n * n16;
  for (int64_t x = threadIdx.x; x < tot16; x += 256) {
    const int64_t q = x / ((int64_t)n * n16);
    const int rem = (int)(x - q * n * n16);
    const int a = rem / n16, c = rem - a * n16;
    uint16_t h = 0, l = 0;
    if (c < n) split_d<S>(src[(q * n + a) * n + c] * (double)sc, h, l);
    hi[boff[blockIdx.x] + x] = h;
    lo[boff[blockIdx.x] + x] = l;
  }
}

// S of coupling e (FP64 [c][a], n_src x n_tgt) -> [a][c] padded split copy
template <typename S>
__global__ __launch_bounds__(256) void split_S_kernel(const PairDev* pairs, const int64_t* rowptr_target,
                                                      const CplDev* cpl, const double* Sd, const int64_t* soff,
                                                      int64_t ncpl, uint16_t* hi, uint16_t* lo) {
  for (int64_t e = blockIdx.x; e < ncpl; e += gridDim.x) {
    const int p = (int)rowptr_target[e];
    const int n = pairs[p].n, nq = cpl[e].nsrc, nq16 = 16 * ((nq + 15) / 16);
    const double* W = Sd + cpl[e].off_S;
    for (int x = threadIdx.x; x < n * nq16; x += 256) {
      const int a = x / nq16, c = x - a * nq16;
      uint16_t h = 0, l = 0;
      if (c < nq) split_d<S>(W[c * n + a], h, l);
      hi[soff[e] + x] = h;
      lo[soff[e] + x] = l;
    }
  }
}

// amplitudes (FP64 T layout) -> split T^T and T copies, one workgroup per block
template <typename S>
__global__ __launch_bounds__(256) void split_T_kernel(const BlockDev* blocks, const double* T, const int64_t* toff,
                                                      float* tscale, uint16_t* tt_hi, uint16_t* tt_lo,
                                                      uint16_t* t_hi, uint16_t* t_lo, int scaled) {
  const BlockDev bk = blocks[blockIdx.x];
  const int n = bk.n, n16 = 16 * ((n + 15) / 16);
  const double* src = T + bk.off_T;
  float sc = 1.f;
  if (scaled) {
    double mx = 0.0;
    for (int x = threadIdx.x; x < n * n; x += 256) mx = fmax(mx, fabs(src[x]));
    sc = pow2_scale(block_max(mx));
    if (threadIdx.x == 0) tscale[blockIdx.x] = sc;
  }
  const int64_t o = toff[blockIdx.x];
  for (int x = threadIdx.x; x < n * n16; x += 256) {
    const int row = x / n16, col = x - row * n16;
    uint16_t h = 0, l = 0, h2 = 0, l2 = 0;
    if (col < n) {
      split_d<S>(src[col * n + row] * (double)sc, h, l);    // T^T[row][col] = T[col][row]
      split_d<S>(src[row * n + col] * (double)sc, h2, l2);  // T[row][col]
    }
    tt_hi[o + x] = h;
    tt_lo[o + x] = l;
    t_hi[o + x] = h2;
    t_lo[o + x] = l2;
  }
}

hipError_t launch_split_grouped(const SplitArgs& a, int kind, bool fp16, int workers, hipStream_t s) {
  if (kind == ITEM_LADDER) {
    if (fp16) hipLaunchKernelGGL((split_grouped_kernel<SplitF16, ITEM_LADDER>), dim3(workers), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((split_grouped_kernel<SplitBf16, ITEM_LADDER>), dim3(workers), dim3(256), 0, s, a);
  } else {
    if (fp16) hipLaunchKernelGGL((split_grouped_kernel<SplitF16, ITEM_PROJ>), dim3(2 * workers), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((split_grouped_kernel<SplitBf16, ITEM_PROJ>), dim3(2 * workers), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_split_B(const PairDev* pairs, int npairs, const double* B, const int64_t* boff, float* bscale,
                          uint16_t* hi, uint16_t* lo, bool fp16, hipStream_t s) {
  if (npairs == 0) return hipSuccess;
  if (fp16) hipLaunchKernelGGL(split_B_kernel<SplitF16>, dim3(npairs), dim3(256), 0, s, pairs, B, boff, bscale, hi, lo, 1);
  else hipLaunchKernelGGL(split_B_kernel<SplitBf16>, dim3(npairs), dim3(256), 0, s, pairs, B, boff, bscale, hi, lo, 0);
  return hipGetLastError();
}

hipError_t launch_split_S(const PairDev* pairs, const int64_t* cpl_target, const CplDev* cpl, const double* S,
                          const int64_t* soff, int64_t ncpl, uint16_t* hi, uint16_t* lo, bool fp16, hipStream_t s) {
  if (ncpl == 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(ncpl, 65536);
  if (fp16) hipLaunchKernelGGL(split_S_kernel<SplitF16>, dim3(grid), dim3(256), 0, s, pairs, cpl_target, cpl, S, soff, ncpl, hi, lo);
  else hipLaunchKernelGGL(split_S_kernel<SplitBf16>, dim3(grid), dim3(256), 0, s, pairs, cpl_target, cpl, S, soff, ncpl, hi, lo);
  return hipGetLastError();
}

hipError_t launch_split_T(const BlockDev* blocks, int nblocks, const double* T, const int64_t* toff, float* tscale,
                          uint16_t* tt_hi, uint16_t* tt_lo, uint16_t* t_hi, uint16_t* t_lo, bool fp16, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (fp16) hipLaunchKernelGGL(split_T_kernel<SplitF16>, dim3(nblocks), dim3(256), 0, s, blocks, T, toff, tscale, tt_hi, tt_lo, t_hi, t_lo, 1);
  else hipLaunchKernelGGL(split_T_kernel<SplitBf16>, dim3(nblocks), dim3(256), 0, s, blocks, T, toff, tscale, tt_hi, tt_lo, t_hi, t_lo, 0);
  return hipGetLastError();
}

}  // namespace dlpno
