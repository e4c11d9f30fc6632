// Ring/exchange term of the CCSD doubles residual in the pairs' PNO bases.
//
// The spin-orbital term P(IJ) P(AB) sum_ME t_IM^AE <MB||EJ> is the part of
// the doubles residual that is linear in the doubles and couples a target
// pair (i, j) to the pairs {i, m} and {j, m} that share one occupied index
// with it (Sec. II.B.3 solves the CC residual equations in the truncated PNO
// bases).  Reduced to the stored spin blocks, every contribution is one
// contraction
//     Out += w L^T op(T_q) M,
// where T_q is a stored amplitude block of the source pair (n_q x n_q,
// op = transpose or not), and L, M are an overlap block S (source PNOs x
// target PNOs) and an integral block X = (m e | b y) or J = (m y | b e) in the
// same layout, in one order or the other (the second order yields the
// transposed contribution).  The plan lists the contractions of each target
// block (RxTerm), with their signs, grouped into units of one block each.
//
// Partial slots hold their contribution transposed (row b, column a, as the
// grouped kernel writes them), so the kernel evaluates Out^T = M^T op'(T_q) L
// with op' the opposite transposition.  One workgroup of four wavefronts
// takes one unit.  Wave w evaluates the unit's contractions w, w + 4, ... on
// the 16x16x4 FP64 MFMA, one tile of 16 source PNOs at a time:
//   P = op'(T_q)[tile rows] L       (16 x n_p), k over the source's PNOs;
//   Z += M[tile rows]^T P           (n_p x n_p), k over the tile;
// the accumulator of P is, register by register, the B operand of the second
// product (register i of lane group g holds row 4 i + g of the tile), so P
// never leaves the VGPRs.  The four waves' sums are added in a fixed order
// through LDS and written to the block's last partial slot, which the
// finishing kernel adds to the residual: the result is deterministic.
//
// Operands are read with raw buffer loads whose resource covers exactly one
// matrix: reads past its end return zero.  Padding the source index (to
// chunks of four k-steps and tiles of 16) only reaches rows of L or M beyond
// the source's PNOs, which lie past the end of their block and read as zero,
// and elements of the source block that are finite and meet those zeros;
// padding the target index only reaches output rows and columns that are
// never stored.
#include <hip/hip_runtime.h>

#include "grouped_impl.h"
#include "internal.h"

namespace dlpno {
namespace {

typedef Mfma<double>::V V;

template <int NT>
__device__ __forceinline__ void ring_unit(const RxUnit& u, const RxTerm* __restrict__ terms, const BlockDev& bk,
                                          const double* T, const double* S, const double* Ri, double* ws,
                                          double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int n = uni(bk.n);
  V Z[NT][NT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) Z[a][b] = V{0, 0, 0, 0};

  for (int64_t k = u.t0 + wave; k < u.t1; k += 4) {
    const RxTerm t = terms[k];
    const int nq = uni(t.nq);
    const int flags = uni(t.flags);
    const double w = uni(t.w);
    const int nqt = (nq + 15) >> 4, nq4 = (nq + 3) >> 2;
    // the slot holds Out^T = M^T op(T)^T L: the first product takes L, the
    // second M, and the source block enters with the opposite transposition
    const __amdgpu_buffer_rsrc_t xr = rsrc(T + uni(t.src_off), (uint32_t)(nq * nq));
    const __amdgpu_buffer_rsrc_t br = rsrc(((flags & kRxL) ? Ri : S) + uni(t.off_L), (uint32_t)(nq * n));
    const __amdgpu_buffer_rsrc_t ar = rsrc(((flags & kRxM) ? Ri : S) + uni(t.off_M), (uint32_t)(nq * n));
    const bool tr = (flags & kRxTrans) == 0;
    // op'(T)[16 td + r][4 s + g]: element (row, col) of T, or (col, row) when transposed
    const uint32_t xa = tr ? (uint32_t)g * nq + r : (uint32_t)r * nq + g;
    const uint32_t xs = tr ? 4u * nq : 4u;         // per k-step
    const uint32_t xt = tr ? 16u : 16u * nq;       // per source tile
    // per source tile td: P = op'(T)[td rows] L, then Z += M[td rows]^T P,
    // with k-step i of the second product in register i of P (br: B operand
    // of the first product, ar: A operand of the second)
#pragma unroll
    for (int td = 0; td < 4; ++td) {
      if (td >= nqt) break;
      V Pt[NT];
#pragma unroll
      for (int b = 0; b < NT; ++b) Pt[b] = V{0, 0, 0, 0};
      // k-steps in chunks of four: the chunk's operands are loaded together,
      // then multiplied.  Steps past the source's PNOs read rows of L beyond
      // its end (zero), so the last chunk needs no predicate.
      for (int s0 = 0; s0 < nq4; s0 += 4) {
        double xv[4], lb[4][NT];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int s = s0 + u;
          xv[u] = Mfma<double>::load(xr, xa + (uint32_t)s * xs + (uint32_t)td * xt);
#pragma unroll
          for (int b = 0; b < NT; ++b) lb[u][b] = Mfma<double>::load(br, (uint32_t)(4 * s + g) * n + 16 * b + r);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int b = 0; b < NT; ++b) Pt[b] = Mfma<double>::op(w * xv[u], lb[u][b], Pt[b]);
      }
      // rows of M past the source's PNOs are zero (beyond its end)
      double la[4][NT];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int a = 0; a < NT; ++a) la[i][a] = Mfma<double>::load(ar, (uint32_t)(16 * td + 4 * i + g) * n + 16 * a + r);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = 0; b < NT; ++b) Z[a][b] = Mfma<double>::op(la[i][a], Pt[b][i], Z[a][b]);
    }
  }

  // fixed-order sum of the four waves: ((w0 + w1) + w2) + w3
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    if (wave == step) {
#pragma unroll
      for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            double* x = lds + ((a * NT + b) * 4 + i) * 64 + lane;
            const double v = step == 0 ? Z[a][b][i] : *x + Z[a][b][i];
            if (step < 3) {
              *x = v;
            } else {
              const int row = 16 * a + 4 * i + g, col = 16 * b + r;
              if (row < n && col < n) ws[(int64_t)row * n + col] = v;
            }
          }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256, 2) void ring_kernel(const RxUnit* __restrict__ units, int64_t n_units,
                                                  const RxTerm* __restrict__ terms,
                                                  const BlockDev* __restrict__ blocks, const double* T,
                                                  const double* S, const double* Ri, double* ws) {
  __shared__ double lds[4 * 4 * 4 * 64];
  for (int64_t x = blockIdx.x; x < n_units; x += gridDim.x) {
    const RxUnit u = units[x];
    const BlockDev bk = blocks[u.blk];
    const int64_t nn = (int64_t)bk.n * bk.n;
    double* dst = ws + bk.off_ws + (int64_t)(bk.nslot - 1) * nn;
    switch ((bk.n + 15) >> 4) {
      case 1: ring_unit<1>(u, terms, bk, T, S, Ri, dst, lds); break;
      case 2: ring_unit<2>(u, terms, bk, T, S, Ri, dst, lds); break;
      case 3: ring_unit<3>(u, terms, bk, T, S, Ri, dst, lds); break;
      default: ring_unit<4>(u, terms, bk, T, S, Ri, dst, lds); break;
    }
  }
}

}  // namespace

hipError_t launch_ring(const RxUnit* units, int64_t n_units, const RxTerm* terms, const BlockDev* blocks,
                       const double* T, const double* S, const double* ring_ints, double* ws, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  const int64_t grid = std::min<int64_t>(n_units, (int64_t)1 << 20);
  hipLaunchKernelGGL(ring_kernel, dim3((unsigned)grid), dim3(256), 0, s, units, n_units, terms, blocks, T, S,
                     ring_ints, ws);
  return hipGetLastError();
}

}  // namespace dlpno
