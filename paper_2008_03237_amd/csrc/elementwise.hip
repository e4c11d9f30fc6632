// Fock dressing, Jacobi update, pair energies, reductions and DIIS.
//
// All of it is FP64 and HBM-bound: one workgroup per stored spin block reads
// its amplitudes, driver, denominators and the partial sums of the grouped
// kernel once, and writes R and the updated amplitudes once.  Reductions run
// in a fixed order (wavefront shuffles, then LDS across the four waves), so
// every result is bitwise reproducible.
#include "internal.h"

#include <math.h>

namespace dlpno {

constexpr int kEwThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// block-wide sum/max over 256 threads in a fixed order
__device__ __forceinline__ void block_sum_max(double& s, double& m) {
  __shared__ double ls[4], lm[4];
  s = wave_sum(s);
  m = wave_max(m);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    ls[w] = s;
    lm[w] = m;
  }
  __syncthreads();
  s = ((ls[0] + ls[1]) + ls[2]) + ls[3];
  m = fmax(fmax(lm[0], lm[1]), fmax(lm[2], lm[3]));
}

// R = K^{ss'} + D o T + sum of partial slots;  optional T' = T - R / D,
// energy w <K^{ss'}, T'>, max |R|, DIIS error T' - T.
__global__ __launch_bounds__(kEwThreads) void finish_kernel(FinishArgs a) {
  const int blk = blockIdx.x;
  const BlockDev bk = a.blocks[blk];
  const int n = bk.n;
  const int nn = n * n;
  const double* ea = (bk.s1 == 0 ? a.eps_a : a.eps_b) + bk.off_eps;
  const double* eb = (bk.s2 == 0 ? a.eps_a : a.eps_b) + bk.off_eps;
  const double* K = a.K + bk.off_K;
  const double* T = a.T + bk.off_T;
  const double* ws = a.ws + bk.off_ws;
  double* Tn = a.T_new;
  double* err = nullptr;
  if (a.ring) {
    const int64_t o = (int64_t)a.ring->head * a.ring_stride;
    Tn = a.ring_vecs + o;
    err = a.ring_errs + o;
  }
  // The partial slots hold Out^T (row b, column a): they are summed with
  // coalesced reads into LDS and read back transposed (n <= 64).
  __shared__ double part[64 * 64];
  const int nslot = a.no_partials ? 0 : bk.nslot;
  for (int idx = threadIdx.x; idx < nn; idx += kEwThreads) {
    // four slots' loads in flight at a time, added in slot order
    double v = 0.0;
    for (int sl = 0; sl < nslot; sl += 4) {
      double p[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = sl + u < nslot ? ws[(int64_t)(sl + u) * nn + idx] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (sl + u < nslot) v += p[u];
    }
    part[idx] = v;
  }
  __syncthreads();
  double esum = 0.0, rmax = 0.0;
  bool bad = false;
  for (int idx = threadIdx.x; idx < nn; idx += kEwThreads) {
    const int x = idx / n, y = idx - x * n;          // element [a = x][b = y]
    // every load of the element is issued before the first use
    const double t = T[idx];
    const double eax = ea[x], eby = eb[y];
    const double k0 = a.with_driver ? K[idx] : 0.0;
    const double k1 = a.with_driver && bk.anti ? K[y * n + x] : 0.0;
    const double dv = a.drv ? a.drv[bk.off_T + idx] : 0.0;
    const double sh = a.shift ? a.shift[blk] : 0.0;
    const double D = (eax + eby) - bk.fsum;
    double kk = 0.0;
    if (a.with_driver) {
      kk = k0;
      if (bk.anti) kk -= k1;
    }
    double r = (a.drv ? dv : kk) + D * t;
    r += part[y * n + x];
    if (a.shift) r -= sh * t;                     // diagonal part of the occupied intermediate
    if (x >= bk.rows || y >= bk.cols) r = 0.0;   // alpha index on a SOMO function
    if (!isfinite(r)) bad = true;
    rmax = fmax(rmax, fabs(r));
    if (a.R) a.R[bk.off_T + idx] = r;
    if (Tn) {
      const double tn = t - r / D;
      Tn[bk.off_T + idx] = tn;
      if (err) err[bk.off_T + idx] = tn - t;
      esum += kk * tn;
    }
  }
  if (bad) atomicOr(a.nonfinite, kErrNonfinite);
  block_sum_max(esum, rmax);
  if (threadIdx.x == 0) {
    if (a.e_block) a.e_block[blk] = bk.w * esum;
    if (a.rmax_block) a.rmax_block[blk] = rmax;
  }
}

// Second-order F12 pair energy of every stored block with the converged
// amplitudes (Sec. II.A: Eq. "Vtilde" without the singles terms, and the
// spin-adapted pair energies that follow Eq. "F12 energy").  Per block:
//   d = <W, T>, x = <W^T, T>        (W = (V + C)^{ij}_{ab} in the block's order)
//   V~ = V + d / 2, V~x = V' + x / 2 (direct and exchanged geminal)
//   same spin:     eps = V~ / 2 + B1 / 16
//   opposite spin: eps = 3/4 V~ + 1/4 V~x + (9 B1 + 3 B2 + 3 B3 + B4) / 64
// One wave per block (four per workgroup, no LDS, so that many blocks are in
// flight): W and T are read coalesced, the transposed T reads hit the lines
// the wave fetches itself.  The sums use a fixed order.
__global__ __launch_bounds__(kEwThreads) void f12_kernel(F12Args a) {
  const int lane = threadIdx.x & 63;
  const int blk = blockIdx.x * (kEwThreads / 64) + (threadIdx.x >> 6);
  if (blk >= a.n_blocks) return;                  // whole waves; no barriers below
  const int n = a.blocks[blk].n;
  const int64_t off = a.blocks[blk].off_T;
  const double* T = a.T + off;
  const double* W = a.W + off;
  const int nn = n * n;
  double d = 0.0, x = 0.0;
#pragma unroll 4
  for (int idx = lane; idx < nn; idx += 64) {
    const int r = idx / n, c = idx - r * n;
    const double w = W[idx];
    d += w * T[idx];
    x += w * T[c * n + r];
  }
  d = wave_sum(d);
  x = wave_sum(x);
  if (lane == 0) {
    const double* sc = a.scal + 6 * (int64_t)blk;
    const double vt = sc[0] + 0.5 * d, vtx = sc[1] + 0.5 * x;
    double e;
    if (a.blocks[blk].s1 == a.blocks[blk].s2) e = 0.5 * vt + sc[2] / 16.0;
    else e = 0.75 * vt + 0.25 * vtx + (9.0 * sc[2] + 3.0 * sc[3] + 3.0 * sc[4] + sc[5]) / 64.0;
    a.e_block[blk] = e;
  }
}

// T' = T - R / D and energies from a given residual.
__global__ __launch_bounds__(kEwThreads) void update_kernel(UpdateArgs a) {
  const int blk = blockIdx.x;
  const BlockDev bk = a.blocks[blk];
  const int n = bk.n;
  const int nn = n * n;
  const double* ea = (bk.s1 == 0 ? a.eps_a : a.eps_b) + bk.off_eps;
  const double* eb = (bk.s2 == 0 ? a.eps_a : a.eps_b) + bk.off_eps;
  const double* K = a.K + bk.off_K;
  double esum = 0.0, dummy = 0.0;
  for (int idx = threadIdx.x; idx < nn; idx += kEwThreads) {
    const int x = idx / n, y = idx - x * n;
    const double D = (ea[x] + eb[y]) - bk.fsum;
    double kk = K[idx];
    if (bk.anti) kk -= K[y * n + x];
    const double tn = a.T[bk.off_T + idx] - a.R[bk.off_T + idx] / D;
    a.T_new[bk.off_T + idx] = tn;
    esum += kk * tn;
  }
  block_sum_max(esum, dummy);
  if (threadIdx.x == 0) a.e_block[blk] = bk.w * esum;
}

// pair energies, total energy, max |R|, iteration history.  Stage 1:
// kReduceParts workgroups, each summing (and taking the maximum of) a fixed
// contiguous range of blocks, and writing the pair energies of a grid-stride
// share of the pairs; stage 2: one wave combines the partial results.  Both
// stages use a fixed order, so the results do not depend on timing.
__global__ __launch_bounds__(kEwThreads) void reduce_parts_kernel(ReduceArgs a) {
  const int g = blockIdx.x;
  const int chunk = (a.n_blocks + kReduceParts - 1) / kReduceParts;
  const int b0 = g * chunk, b1 = min(a.n_blocks, b0 + chunk);
  double s = 0.0, m = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += kEwThreads) {
    s += a.e_block[b];
    if (a.rmax_block) m = fmax(m, a.rmax_block[b]);
  }
  if (a.e_pair) {
    for (int p = g * kEwThreads + threadIdx.x; p < a.n_pairs; p += kReduceParts * kEwThreads) {
      const PairDev P = a.pairs[p];
      double e[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < P.nblk; ++k) e[a.blocks[P.blk0 + k].code] = a.e_block[P.blk0 + k];
      for (int c = 0; c < 4; ++c) a.e_pair[4 * (int64_t)p + c] = e[c];
    }
  }
  block_sum_max(s, m);
  if (threadIdx.x == 0) {
    a.partial[g] = s;
    a.partial[kReduceParts + g] = m;
  }
}

__global__ __launch_bounds__(64) void reduce_final_kernel(ReduceArgs a) {
  static_assert(kReduceParts == 64, "one partial per lane");
  double s = a.partial[threadIdx.x], m = a.partial[kReduceParts + threadIdx.x];
  s = wave_sum(s);
  m = wave_max(m);
  if (threadIdx.x == 0) {
    if (a.e_total) *a.e_total = s;
    if (a.rmax) *a.rmax = m;
    if (a.iter) {
      const int it = *a.iter;
      if (a.hist && it < a.hist_cap) {
        a.hist[2 * it] = s;
        a.hist[2 * it + 1] = m;
      }
      *a.iter = it + 1;
    }
  }
}

// ------------------------------------------------------------------ DIIS
__global__ void diis_reset_kernel(DiisState* st, int max, int start) {
  st->count = 0;
  st->head = max - 1;
  st->max = max;
  st->start = start;
  st->iter = 0;
  st->drops = 0;
  for (int a = 0; a < 8; ++a) {
    st->coef[a] = 0.0;
    for (int b = 0; b < 8; ++b) st->gram[a][b] = 0.0;
  }
}

__global__ void diis_slot_kernel(DiisState* st) {
  st->head = (st->head + 1) % st->max;
  if (st->count < st->max) st->count += 1;
}

// partial[part][k] = sum over this part of err[head] * err[k] for every stored slot k
__global__ __launch_bounds__(256) void diis_dots_kernel(const double* errs, int64_t n, const DiisState* st,
                                                        double* partial) {
  const int cnt = st->count, head = st->head, mx = st->max;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  const double* eh = errs + (int64_t)head * n;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  int64_t so[8];                                    // k-th newest vector
#pragma unroll
  for (int k = 0; k < 8; ++k) so[k] = (int64_t)((head - k + mx) % mx) * n;
  for (int64_t x = lo + threadIdx.x; x < hi; x += 256) {
    // every load of the element is issued before the first product
    const double v = eh[x];
    double e[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) e[k] = k < cnt ? errs[so[k] + x] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < cnt) acc[k] += v * e[k];
  }
  __shared__ double ls[8][4];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double s = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) ls[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int k = threadIdx.x;
    partial[(int64_t)blockIdx.x * 8 + k] = ((ls[k][0] + ls[k][1]) + ls[k][2]) + ls[k][3];
  }
}

// symmetric eigenvalues by cyclic Jacobi (n <= 9), for the condition number.
// The matrix is held in registers: every loop is unrolled to the bound 9 with
// guards on n, so all indices are constants (with run-time indices the
// elements lived in LDS or scratch memory, and each dependent access paid
// its latency on the single thread that runs this).
__device__ void sym_eigs(const double* Ain, int n, double* ev) {
  double A[9][9];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j) A[i][j] = (i < n && j < n) ? Ain[i * 9 + j] : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int p = 0; p < 9; ++p)
#pragma unroll
      for (int q = p + 1; q < 9; ++q)
        if (q < n) off += A[p][q] * A[p][q];
    if (off < 1e-300) break;
#pragma unroll
    for (int p = 0; p < 9; ++p)
#pragma unroll
      for (int q = p + 1; q < 9; ++q) {
        if (q >= n) continue;
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          if (k >= n) continue;
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          if (k >= n) continue;
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
      }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
    if (k < n) ev[k] = A[k][k];
}

// Gram update, bordered system [[G, -1], [-1, 0]] c = [0, -1] with
// G = <e_i, e_j> / max_k <e_k, e_k>, solved by Gaussian elimination with
// partial pivoting; oldest vectors are dropped while the matrix's 2-norm
// condition number exceeds 1e14.  The normalisation leaves c unchanged and
// makes the test one of near linear dependence of the errors, independent of
// their size (unnormalised, the condition number grows like 1 / |e|^2 as the
// iteration converges).
__global__ __launch_bounds__(256) void diis_solve_kernel(DiisState* st, const double* partial, int nparts) {
  const int cnt0 = st->count, head = st->head, mx = st->max;
  // new Gram row: the parts summed by 256 threads (thread t takes parts t,
  // t + 256, ...), then a fixed-order reduction over the threads
  __shared__ double lw[8][4];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    double v = 0.0;
    if (k < cnt0)
      for (int p = threadIdx.x; p < nparts; p += 256) v += partial[(int64_t)p * 8 + k];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lw[k][threadIdx.x >> 6] = v;
  }
  // the small bordered solve runs on one thread with its arrays in LDS:
  // as private arrays with run-time indices they lived in scratch memory,
  // whose latency made this kernel take 0.7 ms
  __shared__ double M[81], E[81], rhs[9], x[9], ev[9];
  __shared__ int sl[8];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < cnt0; ++k) {
    const double s = ((lw[k][0] + lw[k][1]) + lw[k][2]) + lw[k][3];
    const int slot = (head - k + mx) % mx;
    st->gram[head][slot] = s;
    st->gram[slot][head] = s;
  }
  for (int k = 0; k < 8; ++k) st->coef[k] = 0.0;
  if (cnt0 < st->start) {
    st->coef[head] = 1.0;
    return;
  }
  int cnt = cnt0;
  for (;;) {
    // slots oldest -> newest
    for (int k = 0; k < cnt; ++k) sl[k] = (head - (cnt - 1 - k) + mx) % mx;
    const int N = cnt + 1;
    double gscale = 0.0;
    for (int a = 0; a < cnt; ++a) gscale = fmax(gscale, st->gram[sl[a]][sl[a]]);
    if (!(gscale > 0.0)) gscale = 1.0;
    for (int a = 0; a < N; ++a) {
      for (int b = 0; b < N; ++b) {
        double v;
        if (a < cnt && b < cnt) v = st->gram[sl[a]][sl[b]] / gscale;
        else if (a == cnt && b == cnt) v = 0.0;
        else v = -1.0;
        M[a * 9 + b] = v;
        E[a * 9 + b] = v;
      }
      rhs[a] = (a == cnt) ? -1.0 : 0.0;
    }
    if (cnt > 1) {
      sym_eigs(E, N, ev);
      double amax = 0.0, amin = 1e308;
      for (int k = 0; k < N; ++k) {
        amax = fmax(amax, fabs(ev[k]));
        amin = fmin(amin, fabs(ev[k]));
      }
      if (!(amin > 0.0) || amax / amin > 1e14) {
        cnt -= 1;      // drop the oldest
        st->count = cnt;
        st->drops += 1;
        continue;
      }
    }
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < N; ++c) {
      int piv = c;
      for (int rr = c + 1; rr < N; ++rr)
        if (fabs(M[rr * 9 + c]) > fabs(M[piv * 9 + c])) piv = rr;
      if (piv != c) {
        for (int k = 0; k < N; ++k) {
          const double tmp = M[c * 9 + k];
          M[c * 9 + k] = M[piv * 9 + k];
          M[piv * 9 + k] = tmp;
        }
        const double tmp = rhs[c];
        rhs[c] = rhs[piv];
        rhs[piv] = tmp;
      }
      for (int rr = c + 1; rr < N; ++rr) {
        const double f = M[rr * 9 + c] / M[c * 9 + c];
        for (int k = c; k < N; ++k) M[rr * 9 + k] -= f * M[c * 9 + k];
        rhs[rr] -= f * rhs[c];
      }
    }
    for (int c = N - 1; c >= 0; --c) {
      double s = rhs[c];
      for (int k = c + 1; k < N; ++k) s -= M[c * 9 + k] * x[k];
      x[c] = s / M[c * 9 + c];
    }
    for (int k = 0; k < cnt; ++k) st->coef[sl[k]] = x[k];
    return;
  }
}

// T = sum_k coef[k] vec[k], stored slots oldest -> newest
__global__ __launch_bounds__(256) void diis_extrap_kernel(const double* vecs, int64_t n, const DiisState* st,
                                                          double* T) {
  const int cnt = st->count, head = st->head, mx = st->max;
  // oldest to newest; loops unrolled to the bound 8 with guards on the count,
  // so the slots and coefficients stay in registers and every load of an
  // element is issued before the first product
  int64_t so[8];
  double c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int sl = k < cnt ? (head - (cnt - 1 - k) + mx) % mx : 0;
    so[k] = (int64_t)sl * n;
    c[k] = k < cnt ? st->coef[sl] : 0.0;
  }
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < n; x += (int64_t)gridDim.x * 256) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = k < cnt ? vecs[so[k] + x] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < cnt) s += c[k] * v[k];
    T[x] = s;
  }
}

__global__ void convert_f32_kernel(const double* src, float* dst, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < n; x += (int64_t)gridDim.x * 256)
    dst[x] = (float)src[x];
}
__global__ void axpy_kernel(double* y, const double* x, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    y[i] += a * x[i];
}
// Same-spin blocks onto their antisymmetric part: T <- (T - T^T) / 2.  One
// workgroup per block; each thread owns the element pairs (a, b), a < b, it
// updates, so no two threads touch the same element.
__global__ void antisym_kernel(const BlockDev* blocks, double* T) {
  const BlockDev& bk = blocks[blockIdx.x];
  if (!bk.anti) return;
  const int n = bk.n;
  double* X = T + bk.off_T;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int a = idx / n, b = idx % n;
    if (a > b) continue;
    if (a == b) {
      X[idx] = 0.0;
    } else {
      const double v = 0.5 * (X[a * n + b] - X[b * n + a]);
      X[a * n + b] = v;
      X[b * n + a] = -v;
    }
  }
}
__global__ void fill_kernel(double* y, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = v;
}
__global__ void copy_kernel(double* y, const double* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = x[i];
}

static int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

__global__ __launch_bounds__(256) void any_nonzero_kernel(const double* x, int64_t n, int32_t* flag) {
  bool nz = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    nz = nz || !(x[i] == 0.0);
  if (__any(nz) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_any_nonzero(const double* x, int64_t n, int32_t* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(any_nonzero_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

hipError_t launch_finish(const FinishArgs& a, hipStream_t s) {
  if (a.n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_kernel, dim3(a.n_blocks), dim3(kEwThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_f12(const F12Args& a, hipStream_t s) {
  if (a.n_blocks == 0) return hipSuccess;
  const int per = kEwThreads / 64;
  hipLaunchKernelGGL(f12_kernel, dim3((a.n_blocks + per - 1) / per), dim3(kEwThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  if (a.n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(update_kernel, dim3(a.n_blocks), dim3(kEwThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  if (!a.partial) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(kReduceParts), dim3(kEwThreads), 0, s, a);
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_diis_reset(DiisState* st, int max, int start, hipStream_t s) {
  hipLaunchKernelGGL(diis_reset_kernel, dim3(1), dim3(1), 0, s, st, max, start);
  return hipGetLastError();
}
hipError_t launch_diis_slot(DiisState* st, hipStream_t s) {
  hipLaunchKernelGGL(diis_slot_kernel, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}
hipError_t launch_diis_dots(const double* errs, int64_t n, DiisState* st, double* partial, int nparts,
                            hipStream_t s) {
  hipLaunchKernelGGL(diis_dots_kernel, dim3(nparts), dim3(256), 0, s, errs, n, st, partial);
  return hipGetLastError();
}
hipError_t launch_diis_solve(DiisState* st, const double* partial, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(diis_solve_kernel, dim3(1), dim3(256), 0, s, st, partial, nparts);
  return hipGetLastError();
}
hipError_t launch_diis_extrap(const double* vecs, int64_t n, const DiisState* st, double* T, hipStream_t s) {
  hipLaunchKernelGGL(diis_extrap_kernel, dim3(grid_for(n)), dim3(256), 0, s, vecs, n, st, T);
  return hipGetLastError();
}
hipError_t launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(convert_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, a, n);
  return hipGetLastError();
}
hipError_t launch_antisymmetrize(const BlockDev* blocks, int n_blocks, double* T, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(antisym_kernel, dim3(n_blocks), dim3(256), 0, s, blocks, T);
  return hipGetLastError();
}
hipError_t launch_copy(double* y, const double* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}

}  // namespace dlpno

namespace dlpno {
hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, v, n);
  return hipGetLastError();
}
}  // namespace dlpno
