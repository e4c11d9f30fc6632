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

// One coupling and its reverse: S_e is [c][a] (rows n_src x cols n_tgt), the
// reverse's block [a][c] must be its transpose.
struct SPair {
  int64_t off_e, off_r;
  int32_t rows, cols;
};

// Sets *bad when an element of a reverse block differs from the transposed
// element by more than 1e-12 of the larger of the two; one workgroup per pair.
__global__ __launch_bounds__(256) void s_transpose_check_kernel(const SPair* pr, int64_t n, const double* S, int32_t* bad) {
  for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    const SPair q = pr[k];
    bool wrong = false;
    for (int idx = threadIdx.x; idx < q.rows * q.cols; idx += 256) {
      const int c = idx / q.cols, a = idx - c * q.cols;
      const double x = S[q.off_e + idx], y = S[q.off_r + (int64_t)a * q.rows + c];
      if (!(fabs(x - y) <= 1e-12 * fmax(fabs(x), fabs(y)))) wrong = true;
    }
    if (wrong) atomicOr(bad, 1);
  }
}

// The transposed residual is evaluated by the forward kernels (see the top of
// this file), which is valid when f^s is symmetric (checked at plan creation)
// and every coupling that carries a term has a reverse coupling whose overlap
// block is its transpose.  Checked once, at the first product; the result is
// kept in the plan.
static dlpno_status check_vjp_preconditions(dlpno_plan* P, hipStream_t s) {
  if (P->vjp_checked != 0) return P->vjp_checked > 0 ? DLPNO_OK : fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
  P->vjp_checked = -1;
  if (!P->quad_h.empty()) {
    P->vjp_reason = "vector-Jacobian product: not available with the quadratic term";
    return fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
  }
  if (P->qocc) {
    P->vjp_reason = "vector-Jacobian product: not available with the occupied-intermediate quadratic term";
    return fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
  }
  if (P->n_ring > 0) {
    P->vjp_reason = "vector-Jacobian product: not available with the ring/exchange term";
    return fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
  }
  if (P->somo_virt) {
    P->vjp_reason = "vector-Jacobian product: not available with SOMO virtual functions";
    return fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
  }
  if (!P->fock_symmetric) {
    P->vjp_reason = "vector-Jacobian product: " + P->vjp_reason;
    return fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
  }
  std::vector<SPair> pairs;
  for (int p = 0; p < P->n_pairs; ++p) {
    const PairDev& tp = P->pairs_h[p];
    for (int64_t e = P->rowptr_h[p]; e < P->rowptr_h[p + 1]; ++e) {
      bool active = false;
      for (int b = 0; b < 4; ++b) active = active || P->terms_h[(size_t)e * 4 + b].src_off >= 0;
      if (!active) continue;
      const int q = P->cpl_h[e].src, k = P->cpl_k_h[e];
      const PairDev& sq = P->pairs_h[q];
      int64_t rev = -1;
      if (P->cpl_side_h[e] == 2) {
        // hole-hole (p <- ordered (k, l)): target q reads p as the ordered pair
        // that puts i against k and j against l
        const int l = P->cpl_l_h[e];
        for (int64_t f = P->rowptr_h[q]; f < P->rowptr_h[q + 1] && rev < 0; ++f) {
          if (P->cpl_side_h[f] != 2 || P->cpl_h[f].src != p) continue;
          const int x = P->cpl_k_h[f], y = P->cpl_l_h[f];
          if ((sq.i == k && sq.j == l && x == tp.i && y == tp.j) || (sq.i == l && sq.j == k && x == tp.j && y == tp.i))
            rev = f;
        }
      } else {
        // reverse: target q reads p with rep replacing k (on the side where q holds k)
        const int rep = P->cpl_side_h[e] == 0 ? tp.i : tp.j;
        for (int64_t f = P->rowptr_h[q]; f < P->rowptr_h[q + 1] && rev < 0; ++f) {
          if (P->cpl_side_h[f] == 2 || P->cpl_h[f].src != p || P->cpl_k_h[f] != rep) continue;
          if ((P->cpl_side_h[f] == 0 ? sq.i : sq.j) == k) rev = f;
        }
      }
      if (rev < 0) {
        P->vjp_reason = "vector-Jacobian product: coupling " + std::to_string(e) + " (pair " + std::to_string(p) +
                        " from pair " + std::to_string(q) + ") has no reverse coupling";
        return fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
      }
      if (e < rev) pairs.push_back({P->cpl_h[e].off_S, P->cpl_h[rev].off_S, sq.n, tp.n});
    }
  }
  if (!pairs.empty()) {
    SPair* d_pairs = nullptr;
    int32_t* d_bad = nullptr;
    if (hipMalloc(&d_pairs, pairs.size() * sizeof(SPair)) != hipSuccess || hipMalloc(&d_bad, sizeof(int32_t)) != hipSuccess) {
      if (d_pairs) (void)hipFree(d_pairs);
      (void)hipGetLastError();
      return fail(DLPNO_ERR_OOM, "vector-Jacobian product: overlap check buffers");
    }
    int32_t bad = 0;
    hipError_t e1 = hipMemcpyAsync(d_pairs, pairs.data(), pairs.size() * sizeof(SPair), hipMemcpyHostToDevice, s);
    if (e1 == hipSuccess) e1 = hipMemcpyAsync(d_bad, &bad, sizeof bad, hipMemcpyHostToDevice, s);
    if (e1 == hipSuccess) {
      const int grid = (int)std::min<size_t>(pairs.size(), 65536);
      hipLaunchKernelGGL(s_transpose_check_kernel, dim3(grid), dim3(256), 0, s, d_pairs, (int64_t)pairs.size(),
                         P->in.S, d_bad);
      e1 = hipGetLastError();
    }
    if (e1 == hipSuccess) e1 = hipMemcpyAsync(&bad, d_bad, sizeof bad, hipMemcpyDeviceToHost, s);
    if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
    (void)hipFree(d_pairs);
    (void)hipFree(d_bad);
    if (e1 != hipSuccess) return fail(DLPNO_ERR_HIP, std::string("vector-Jacobian product: overlap check: ") + hipGetErrorString(e1));
    if (bad) {
      P->vjp_reason = "vector-Jacobian product: the overlap block of a reverse coupling is not the transpose of its coupling's";
      return fail(DLPNO_ERR_UNSUPPORTED, P->vjp_reason);
    }
  }
  P->vjp_checked = 1;
  return DLPNO_OK;
}

}  // namespace dlpno

using namespace dlpno;

extern "C" dlpno_status dlpno_residual_vjp(dlpno_plan* P, const double* T, const double* G, double* dT, double* dB,
                                           void* stream) {
  if (!P || ((!T || !G || !dT) && P->n_T > 0)) return fail(DLPNO_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)stream;
  const dlpno_status pre = check_vjp_preconditions(P, s);
  if (pre != DLPNO_OK) return pre;
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
        (void)hipGetLastError();
        return fail(DLPNO_ERR_OOM, "vector-Jacobian product: dB work items");
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
        (void)hipGetLastError();
        return fail(DLPNO_ERR_OOM, "vector-Jacobian product: FP32 cotangent copy");
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
