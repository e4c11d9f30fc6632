// T-dependent weights of the quadratic CCSD terms: the quadratic term on the
// hole-hole couplings, and the quadratic part of the occupied Fock
// intermediate on the occupied-Fock couplings.
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
// The factor G = S_pq K_(k,l) S_pq^T (n_p x n_p) depends only on the plan's
// inputs: it is computed once per coupling when the plan is built (one
// workgroup per coupling, S_pq and K in LDS), and every residual evaluation
// only forms <G, T_p> for the coupling's target blocks (one wave per coupling,
// reduced in a fixed order), writing the new weight into the term table that
// the projection launches of the same residual then read.
//
// The quadratic part of the occupied Fock intermediate, F_MJ = 1/2 sum_NEF
// t_JN^EF <MN||EF>, enters the doubles residual as -P(IJ) sum_M t_IM^AB F_MJ:
// the occupied-Fock projection weights f^s_kj become f^s_kj + F^s_kj and the
// pair itself adds -(F^s_ii + F^s'_jj) T.  Per spin, F^s_mj = sum over n and
// its spin of <G_(m,n), T^{s s_n}_(j,n)>, G[e][f] = (m e | n f) over the PNOs
// of {j, n}, taken as S K_(m,n) S^T of the source pair {m, n} (built once,
// like the factors above; K_(j,n) itself for m = j).  When j is the pair's
// second index the blocks enter the dot transposed, so such factors are
// stored transposed once and every dot but some of diagonal pairs reads the
// factor and the blocks in the same order.  Per residual: one wave per
// contribution forms its dots, one thread per F adds its contributions in
// a fixed order, one thread per term or block writes the dressed weight or
// the diagonal shift that the finishing kernel applies.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "grouped_impl.h"
#include "internal.h"

namespace dlpno {
namespace {

constexpr int kLdq = 65;

__global__ __launch_bounds__(256, 2) void quad_prepare_kernel(const QuadCpl* __restrict__ list, int64_t n,
                                                              const double* __restrict__ S,
                                                              const double* __restrict__ K, double* __restrict__ G) {
  __shared__ double W[64 * kLdq];   // W[c][a] = S_pq[a][c] (the stored overlap block)
  __shared__ double V[64 * kLdq];   // K_q staged, then V = K_(k,l) W
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
    const QuadCpl q = list[it];
    const int np_ = q.np, nq = q.nq;
    __syncthreads();
    if (lane < np_)
      for (int c = w; c < nq; c += 4) W[c * kLdq + lane] = S[q.off_S + (int64_t)c * np_ + lane];
    if (lane < nq)
      for (int c = w; c < nq; c += 4) V[c * kLdq + lane] = K[q.off_K + (int64_t)c * nq + lane];
    __syncthreads();
    // V[c][b] = sum_d K_(k,l)[c][d] W[d][b]: rows c = w + 4 i, column b = lane
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    if (lane < np_)
      for (int d = 0; d < nq; ++d) {
        const double wv = W[d * kLdq + lane];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int c = min(w + 4 * i, 63);
          acc[i] += (q.transK ? V[d * kLdq + c] : V[c * kLdq + d]) * wv;
        }
      }
    __syncthreads();
    if (lane < np_)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (w + 4 * i < nq) V[(w + 4 * i) * kLdq + lane] = acc[i];
    __syncthreads();
    // G[a][b] = sum_c W[c][a] V[c][b]: rows a = w + 4 i, column b = lane
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    if (lane < np_)
      for (int c = 0; c < nq; ++c) {
        const double vv = V[c * kLdq + lane];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] += W[c * kLdq + min(w + 4 * i, 63)] * vv;
      }
    if (lane < np_)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (w + 4 * i < np_) G[q.off_G + (int64_t)(w + 4 * i) * np_ + lane] = acc[i];
  }
}

__global__ __launch_bounds__(256) void quad_weights_kernel(const QuadCpl* __restrict__ list, int64_t n,
                                                           const double* __restrict__ G,
                                                           const double* __restrict__ T,
                                                           TermDev* __restrict__ terms) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < n; e += waves) {
    const QuadCpl q = list[e];
    const int nn = q.np * q.np;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int x = lane; x < nn; x += 64) {
      const double g = G[q.off_G + x];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b < q.nblk) acc[b] += g * T[q.off_T[b] + x];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
      for (int o = 32; o > 0; o >>= 1) acc[b] += __shfl_xor(acc[b], o);
    if (lane == 0)
      for (int b = 0; b < q.nblk; ++b) terms[q.term[b]].w = q.w0[b] + q.c[b] * acc[b];
  }
}

// One wave per contribution: <G, T_b> (or <G^T, T_b>) summed over its blocks
// per spin, in a fixed order.  Every pass issues all its loads before the
// first product: the factor and the (up to four) blocks are read through
// buffer resources that cover exactly one matrix (an absent block has an
// empty one), so reads past the end, or of an absent block, return zero
// without a branch, and the trip count is the same for every lane.
__global__ __launch_bounds__(256) void occ_dots_kernel(const OccCtb* __restrict__ list, int64_t n,
                                                       const double* __restrict__ G, const double* __restrict__ K,
                                                       const double* __restrict__ T, double* __restrict__ dots) {
  constexpr int U = 4;                       // elements per lane and pass
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < n; e += waves) {
    const OccCtb& c = list[e];
    const int nd = uni(c.n);
    const uint32_t nn = (uint32_t)nd * (uint32_t)nd;
    const __amdgpu_buffer_rsrc_t gr = rsrc((uni(c.from_K) ? K : G) + uni(c.off_G), nn);
    __amdgpu_buffer_rsrc_t tr[2][2];
    bool any_tr = false;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int64_t o = uni(c.off_T[sp][b]);
        tr[sp][b] = rsrc(T + (o >= 0 ? o : 0), o >= 0 ? nn : 0u);
        any_tr |= uni(c.tr[sp][b]) != 0;
      }
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (!any_tr) {
      // every block in the factor's order (all but some dots of diagonal
      // pairs)
      for (uint32_t p = 0; p < nn; p += 64 * U) {
        double gv[U], tv[2][2][U];
#pragma unroll
        for (int u = 0; u < U; ++u) gv[u] = Mfma<double>::load(gr, p + 64 * u + lane);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int u = 0; u < U; ++u) tv[sp][b][u] = Mfma<double>::load(tr[sp][b], p + 64 * u + lane);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[sp][b] += gv[u] * tv[sp][b][u];
      }
    } else {
      int trs[2][2];
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int b = 0; b < 2; ++b) trs[sp][b] = uni(c.tr[sp][b]);
      for (uint32_t p = 0; p < nn; p += 64) {
        // x < nn: element (xr, xc) of the factor; past its end the factor
        // reads zero, and the block reads an element of the same block
        // (finite) or, past the block's end, zero
        const uint32_t x = p + lane;
        const uint32_t xr = x / (uint32_t)nd, xc = x - xr * (uint32_t)nd, xt = xc * (uint32_t)nd + xr;
        const double gv = Mfma<double>::load(gr, x);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[sp][b] += gv * Mfma<double>::load(tr[sp][b], trs[sp][b] ? xt : x);
      }
    }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        for (int o = 32; o > 0; o >>= 1) acc[sp][b] += __shfl_xor(acc[sp][b], o);
    if (lane == 0) {
      dots[2 * e] = acc[0][0] + acc[0][1];
      dots[2 * e + 1] = acc[1][0] + acc[1][1];
    }
  }
}

// F per key: its contributions added in CSR order
__global__ __launch_bounds__(256) void occ_f_kernel(const int64_t* __restrict__ rowptr,
                                                    const int64_t* __restrict__ src, int64_t n_keys,
                                                    const double* __restrict__ dots, double* __restrict__ F) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_keys; k += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int64_t x = rowptr[k]; x < rowptr[k + 1]; ++x) v += dots[src[x]];
    F[k] = v;
  }
}

// dressed weights of the listed projection terms, and the per-block shift
__global__ __launch_bounds__(256) void occ_apply_kernel(const OccTerm* __restrict__ ot, int64_t n_ot,
                                                        const double* __restrict__ F, TermDev* __restrict__ terms,
                                                        const int32_t* __restrict__ blk_key, int32_t n_blocks,
                                                        double* __restrict__ shift) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_ot; t += stride)
    terms[ot[t].term].w = ot[t].w0 + F[ot[t].key];
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks; b += stride) {
    const int32_t ki = blk_key[2 * b], kj = blk_key[2 * b + 1];
    shift[b] = (ki >= 0 ? F[ki] : 0.0) + (kj >= 0 ? F[kj] : 0.0);
  }
}

// in-place transposes of square blocks (n <= 64), one workgroup per block
__global__ __launch_bounds__(256) void transpose_blocks_kernel(const int64_t* __restrict__ offs,
                                                               const int32_t* __restrict__ ns, int64_t count,
                                                               double* __restrict__ G) {
  __shared__ double tile[64 * 65];
  for (int64_t b = blockIdx.x; b < count; b += gridDim.x) {
    const int64_t o = offs[b];
    const int nd = ns[b], nn = nd * nd;
    __syncthreads();
    for (int x = threadIdx.x; x < nn; x += blockDim.x) {
      const int r = x / nd, c = x - r * nd;
      tile[r * 65 + c] = G[o + x];
    }
    __syncthreads();
    for (int x = threadIdx.x; x < nn; x += blockDim.x) {
      const int r = x / nd, c = x - r * nd;
      G[o + x] = tile[c * 65 + r];
    }
  }
}

}  // namespace

hipError_t launch_transpose_blocks(const int64_t* offs, const int32_t* ns, int64_t count, double* G, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t grid = count < (1 << 20) ? count : (1 << 20);
  hipLaunchKernelGGL(transpose_blocks_kernel, dim3((unsigned)grid), dim3(256), 0, s, offs, ns, count, G);
  return hipGetLastError();
}

hipError_t launch_occ_weights(const OccArgs& a, const double* T, hipStream_t s) {
  if (a.n_ctb > 0) {
    const int64_t blocks = (a.n_ctb + 3) / 4;
    const int64_t grid = blocks < (1 << 20) ? blocks : (1 << 20);
    hipLaunchKernelGGL(occ_dots_kernel, dim3((unsigned)grid), dim3(256), 0, s, a.ctb, a.n_ctb, a.G, a.K, T, a.dots);
  }
  if (a.n_keys > 0) {
    const int64_t grid = std::min<int64_t>((a.n_keys + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(occ_f_kernel, dim3((unsigned)grid), dim3(256), 0, s, a.key_rowptr, a.key_src, a.n_keys,
                       a.dots, a.F);
  }
  const int64_t m = std::max<int64_t>(a.n_oterms, a.n_blocks);
  if (m > 0) {
    const int64_t grid = std::min<int64_t>((m + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(occ_apply_kernel, dim3((unsigned)grid), dim3(256), 0, s, a.oterms, a.n_oterms, a.F, a.terms,
                       a.blk_key, a.n_blocks, a.shift);
  }
  return hipGetLastError();
}

hipError_t launch_quad_prepare(const QuadCpl* list, int64_t n, const double* S, const double* K, double* G,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = n < (1 << 20) ? n : (1 << 20);
  hipLaunchKernelGGL(quad_prepare_kernel, dim3((unsigned)grid), dim3(256), 0, s, list, n, S, K, G);
  return hipGetLastError();
}

hipError_t launch_quad_weights(const QuadCpl* list, int64_t n, const double* G, const double* T, TermDev* terms,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 3) / 4;
  const int64_t grid = blocks < (1 << 20) ? blocks : (1 << 20);
  hipLaunchKernelGGL(quad_weights_kernel, dim3((unsigned)grid), dim3(256), 0, s, list, n, G, T, terms);
  return hipGetLastError();
}

}  // namespace dlpno
