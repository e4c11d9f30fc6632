// Vector-Jacobian product of the residual.
//
// dT: the residual's linear part is self-adjoint when the occupied Fock
// matrices are symmetric and the overlap block of every coupling is the
// transpose of the block of its reverse coupling (the physical situation):
// the ladder sum_Q B^Q X B^Q^T has the adjoint sum_Q B^Q^T X B^Q (equal for
// symmetric B^Q), the Fock dressing is diagonal, and the projection term read
// by target p from source q is mirrored by the term read by q from p with the
// same weight and transposition.  dT is therefore the grouped kernel run on
// Gbar, finished without the driver:  dT = D o Gbar + partial sums.
//
// dB: for the ladder R = sum_Q B^Q T B^Q^T the gradient with respect to a
// general (unsymmetrised) B^Q is, summed over the pair's blocks,
//   dB^Q = Gbar B^Q T^T + Gbar^T B^Q T.
// Both terms have the form X B^Q Y^T with (X, Y) = (Gbar, T) and
// (Gbar^T, T^T).  One wavefront owns a pair and a range of Q; for every Q it
// forms U = B^Q Y^T on the MFMA and feeds the accumulator straight into
// X U (same register chaining as the forward kernel), so the intermediates
// B^Q T and B^Q T^T are recomputed in registers and never stored.
#include "grouped_impl.h"
#include "plan_internal.h"

#include <algorithm>
#include <string>
#include <vector>

namespace dlpno {

struct DbItem {
  int32_t pair, lo, hi, pad;
};

template <typename F>
struct DbArgs {
  const DbItem* items;
  int32_t n_items;
  const PairDev* pairs;
  const BlockDev* blocks;
  const F* B;
  const F* T;
  const F* G;
  double* dB;
};

template <typename F, int NT>
__device__ __forceinline__ void db_item(const DbArgs<F>& A, const DbItem& it) {
  typedef typename Mfma<F>::V V;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4, pr = Mfma<F>::perm(r);
  const PairDev& Pg = A.pairs[it.pair];
  const int n = uni(Pg.n);
  const int nblk = uni(Pg.nblk);
  const int blk0 = uni(Pg.blk0);
  const int64_t off_B = uni(Pg.off_B);
  const int S4 = (n + 3) >> 2;
  const uint32_t nn = (uint32_t)n * (uint32_t)n;
  for (int Q = it.lo; Q < it.hi; ++Q) {
    const __amdgpu_buffer_rsrc_t br = rsrc(A.B + off_B + (size_t)Q * nn, nn);
    // A operand of U = B^Q Y^T with permuted rows: Ab[td][s] = B^Q[16 td + pi(r)][4 s + g]
    F Ab[NT][4 * NT];
#pragma unroll
    for (int td = 0; td < NT; ++td)
#pragma unroll
      for (int s = 0; s < 4 * NT; ++s)
        Ab[td][s] = Mfma<F>::load(br, (uint32_t)((4 * s + g) * n + 16 * td + pr));
    V acc[NT][NT];   // acc[ta][tc]: dB^Q[16 ta + orow(g, i)][16 tc + r]
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[a][c] = V{0, 0, 0, 0};
    for (int b = 0; b < nblk; ++b) {
      const int64_t off_T = uni(A.blocks[blk0 + b].off_T);
      const __amdgpu_buffer_rsrc_t tr = rsrc(A.T + off_T, nn);
      const __amdgpu_buffer_rsrc_t gr = rsrc(A.G + off_T, nn);
#pragma unroll
      for (int term = 0; term < 2; ++term) {
#pragma unroll
        for (int td = 0; td < NT; ++td) {
          V d1[NT];
#pragma unroll
          for (int c = 0; c < NT; ++c) d1[c] = V{0, 0, 0, 0};
          // stage 1: U[d][c] = sum_e B[d][e] Y[c][e];  Y = T (term 0) or T^T (term 1)
#pragma unroll
          for (int s = 0; s < 4 * NT; ++s) {
            if (s < S4) {
#pragma unroll
              for (int c = 0; c < NT; ++c) {
                const uint32_t off = term == 0 ? (uint32_t)((16 * c + r) * n + 4 * s + g)
                                               : (uint32_t)((4 * s + g) * n + 16 * c + r);
                d1[c] = Mfma<F>::op(Ab[td][s], Mfma<F>::load(tr, off), d1[c]);
              }
            }
          }
          // stage 2: dB[a][c] += sum_d X[a][d] U[d][c];  X = Gbar (term 0) or Gbar^T (term 1)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int sp = 4 * td + i;
            if (sp < S4) {
              const int d = 4 * sp + g;
#pragma unroll
              for (int a = 0; a < NT; ++a) {
                const uint32_t off = term == 0 ? (uint32_t)((16 * a + r) * n + d) : (uint32_t)(d * n + 16 * a + r);
                F x = Mfma<F>::load(gr, off);
                x = d < n ? x : F(0);
#pragma unroll
                for (int c = 0; c < NT; ++c) acc[a][c] = Mfma<F>::op(x, d1[c][i], acc[a][c]);
              }
            }
          }
        }
      }
    }
    double* dst = A.dB + off_B + (size_t)Q * nn;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const int col = 16 * c + r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * a + Mfma<F>::orow(g, i);
          if (row < n && col < n) dst[row * n + col] = (double)acc[a][c][i];
        }
      }
  }
}

template <typename F>
__global__ __launch_bounds__(256) void db_kernel(DbArgs<F> A) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= A.n_items) return;
  const DbItem& ig = A.items[w];
  DbItem it;
  it.pair = uni(ig.pair);
  it.lo = uni(ig.lo);
  it.hi = uni(ig.hi);
  const int nt = (uni(A.pairs[it.pair].n) + 15) >> 4;
  switch (nt) {
    case 1: db_item<F, 1>(A, it); break;
    case 2: db_item<F, 2>(A, it); break;
    case 3: db_item<F, 3>(A, it); break;
    default: db_item<F, 4>(A, it); break;
  }
}

__global__ void zero_f64_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.0;
}

}  // namespace dlpno

using namespace dlpno;

extern "C" dlpno_status dlpno_residual_vjp(dlpno_plan* P, const double* T, const double* G, double* dT, double* dB,
                                           void* stream) {
  if (!P || ((!T || !G || !dT) && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)stream;
  // dT = D o G + (ladder + projection)(G)
  if (run_grouped(P, G, s, -1, true) != hipSuccess) return fail(DLPNO_ERR_HIP, "vjp launch failed");
  FinishArgs f = finish_args(P, G);
  f.R = dT;
  f.with_driver = 0;
  if (launch_finish(f, s) != hipSuccess) return fail(DLPNO_ERR_HIP, "vjp launch failed");
  if (!dB) return DLPNO_OK;
  // dB items: every pair with blocks, Q split into ranges of at most 64
  if (!P->d_vjp_items) {
    std::vector<DbItem> items;
    for (int p = 0; p < P->n_pairs; ++p) {
      const PairDev& pr = P->pairs_h[p];
      if (pr.nblk == 0) continue;
      for (int lo = 0; lo < pr.m; lo += 64) items.push_back({p, lo, std::min(pr.m, lo + 64), 0});
    }
    std::stable_sort(items.begin(), items.end(), [&](const DbItem& a, const DbItem& b) {
      const PairDev &x = P->pairs_h[a.pair], &y = P->pairs_h[b.pair];
      return (double)x.n * x.n * x.n * x.nblk * (a.hi - a.lo) > (double)y.n * y.n * y.n * y.nblk * (b.hi - b.lo);
    });
    P->n_vjp_items = (int)items.size();
    if (!items.empty()) {
      if (hipMalloc(&P->d_vjp_items, items.size() * sizeof(DbItem)) != hipSuccess) {
        P->d_vjp_items = nullptr;
        return DLPNO_ERR_OOM;
      }
      if (hipMemcpy(P->d_vjp_items, items.data(), items.size() * sizeof(DbItem), hipMemcpyHostToDevice) != hipSuccess)
        return fail(DLPNO_ERR_HIP, "vjp launch failed");
    }
  }
  // pairs without blocks keep dB = 0
  hipLaunchKernelGGL(zero_f64_kernel, dim3(4096), dim3(256), 0, s, dB, P->n_B);
  if (hipGetLastError() != hipSuccess) return fail(DLPNO_ERR_HIP, "vjp launch failed");
  if (P->n_vjp_items == 0) return DLPNO_OK;
  const int grid = (P->n_vjp_items + 3) / 4;
  if (P->opt.precision == DLPNO_FP32) {
    // G in FP32 (T32 holds G after run_grouped); T converted into the spare buffer
    if (!P->G32) {
      if (hipMalloc(&P->G32, (size_t)std::max<int64_t>(P->n_T, 1) * sizeof(float)) != hipSuccess) {
        P->G32 = nullptr;
        return DLPNO_ERR_OOM;
      }
    }
    if (launch_convert_f32(G, P->G32, P->n_T, s) != hipSuccess) return fail(DLPNO_ERR_HIP, "vjp launch failed");
    if (launch_convert_f32(T, P->T32, P->n_T, s) != hipSuccess) return fail(DLPNO_ERR_HIP, "vjp launch failed");
    DbArgs<float> a{(const DbItem*)P->d_vjp_items, P->n_vjp_items, P->d_pairs, P->d_blocks, P->B32, P->T32, P->G32, dB};
    hipLaunchKernelGGL(db_kernel<float>, dim3(grid), dim3(256), 0, s, a);
  } else {
    DbArgs<double> a{(const DbItem*)P->d_vjp_items, P->n_vjp_items, P->d_pairs, P->d_blocks, P->in.B, T, G, dB};
    hipLaunchKernelGGL(db_kernel<double>, dim3(grid), dim3(256), 0, s, a);
  }
  if (hipGetLastError() != hipSuccess) return fail(DLPNO_ERR_HIP, "vjp launch failed");
  return DLPNO_OK;
}
