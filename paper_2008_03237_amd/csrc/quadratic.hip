// Weights of the quadratic CCSD term on the hole-hole couplings.
//
// The spin-orbital term 1/4 sum_KLCD <KL||CD> t_IJ^CD t_KL^AB is the
// hole-hole ladder 1/2 sum_KL W_KLIJ t_KL^AB with <KL||IJ> replaced by
// W_KLIJ = 1/2 sum_CD <KL||CD> t_IJ^CD (the CCSD W_mnij intermediate without
// its singles parts, Sec. II.B.3 solves the CC residual equations in the PNO
// bases).  Per spin block s s' of the target pair p and ordered occupied pair
// (k, l) of the coupling, W adds c <K_(k,l), S_pq^T T_p S_pq> to the weight
// (k i | l j), c = 1/2 same spin, 1 opposite spin, where K_(k,l)[c][d] =
// (k c | l d) over the source pair's PNOs (K_q, or its transpose for k > l)
// and S_pq maps the target's PNOs onto the source's: the integrals in the
// target's PNOs are taken as the projection S_pq K_(k,l) S_pq^T.
//
// One workgroup per coupling: the overlap block in LDS, then per target block
// Z = T_p S_pq (n_p x n_q), U = S_pq^T Z and <K, U>, reduced in a fixed order;
// the new weight is written into the coupling's term of that block, which the
// projection launches of the same residual then read.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dlpno {
namespace {

constexpr int kLdq = 65;

__global__ __launch_bounds__(256, 2) void quad_weights_kernel(const QuadCpl* __restrict__ list, int64_t n,
                                                              const double* __restrict__ S,
                                                              const double* __restrict__ K,
                                                              const double* __restrict__ T,
                                                              TermDev* __restrict__ terms) {
  __shared__ double W[64 * kLdq];   // W[c][a] = S_pq[a][c] (the stored overlap block)
  __shared__ double Z[64 * kLdq];   // T_p staged, then Z = T_p S_pq
  __shared__ double red[4];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
    const QuadCpl q = list[it];
    const int np_ = q.np, nq = q.nq;
    __syncthreads();
    if (lane < np_)
      for (int c = w; c < nq; c += 4) W[c * kLdq + lane] = S[q.off_S + (int64_t)c * np_ + lane];
    for (int b = 0; b < q.nblk; ++b) {
      __syncthreads();   // W stored; the previous block's Z no longer read
      if (lane < np_)
        for (int a = w; a < np_; a += 4) Z[a * kLdq + lane] = T[q.off_T[b] + (int64_t)a * np_ + lane];
      __syncthreads();
      // Z[a][d] = sum_x T[a][x] S[x][d] = sum_x T[a][x] W[d][x]: rows a = w + 4 i, column d = lane
      double acc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.0;
      if (lane < nq)
        for (int x = 0; x < np_; ++x) {
          const double sv = W[lane * kLdq + x];
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[i] += Z[min(w + 4 * i, 63) * kLdq + x] * sv;
        }
      __syncthreads();
      if (lane < nq)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (w + 4 * i < np_) Z[(w + 4 * i) * kLdq + lane] = acc[i];
      __syncthreads();
      // U[c][d] = sum_a W[c][a] Z[a][d]: rows c = w + 4 i, column d = lane; then <K_(k,l), U>
      double part = 0.0;
      if (lane < nq)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int c = w + 4 * i;
          if (c >= nq) break;
          double u = 0.0;
          for (int a = 0; a < np_; ++a) u += W[c * kLdq + a] * Z[a * kLdq + lane];
          const double kv = q.transK ? K[q.off_K + (int64_t)lane * nq + c] : K[q.off_K + (int64_t)c * nq + lane];
          part += kv * u;
        }
      for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
      if (lane == 0) red[w] = part;
      __syncthreads();
      if (tid == 0) {
        const double dot = ((red[0] + red[1]) + red[2]) + red[3];
        terms[q.term[b]].w = q.w0[b] + q.c[b] * dot;
      }
    }
  }
}

}  // namespace

hipError_t launch_quad_weights(const QuadCpl* list, int64_t n, const double* S, const double* K, const double* T,
                               TermDev* terms, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = n < (1 << 20) ? n : (1 << 20);
  hipLaunchKernelGGL(quad_weights_kernel, dim3((unsigned)grid), dim3(256), 0, s, list, n, S, K, T, terms);
  return hipGetLastError();
}

}  // namespace dlpno
