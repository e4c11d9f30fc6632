// PNO construction (Sec. II.B.2): for every pair, the pair density of its
// first-order amplitude blocks in the pair's domain, the density's
// eigen-decomposition, truncation at T_CutPNO and semicanonicalisation (the
// domain's virtual Fock matrix diagonalised in the kept natural orbitals).
//
// One workgroup of 256 threads per pair; domains of at most 64 functions so
// that the matrix and its eigenvectors live in LDS (2 x 64 x 65 doubles,
// two workgroups per CU).  Both eigenproblems use the parallel cyclic Jacobi
// method: a sweep is N-1 rounds of N/2 disjoint rotations in round-robin
// order (Brent and Luk's ordering; a zero dummy index pads an odd N), each
// round computes its rotations, then updates the 2x2 blocks of the matrix;
// the eigenvector columns take the round's rotations while the next
// round's rotations are computed.  A rotation is
// skipped when |a_pq| <= 1e-16 sqrt(|a_pp a_qq|) (the criterion of Demmel and
// Veselic, which keeps small eigenvalues of a positive semidefinite matrix
// to high relative accuracy); a sweep that skips all of them ends the
// iteration.  Rotation angles follow Rutishauser's formulas.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "plan_internal.h"

namespace {

constexpr int kMaxDim = 64;
constexpr int kLd = 65;          // LDS row stride (doubles)
constexpr int kThreads = 256;
constexpr int kMaxSweeps = 40;
constexpr double kRelTol = 1e-16;

struct JacobiLds {
  double c[kMaxDim / 2], s[kMaxDim / 2], t[kMaxDim / 2], apq[kMaxDim / 2];
  int p[kMaxDim / 2], q[kMaxDim / 2];
  int rotated;   // some rotation of the round is applied
};

// Work of a round, listed once per eigenproblem in registers (no division
// in the rounds): the 2x2 blocks (k, l), k <= l, of A over all 256 threads
// (at most 528 blocks: 3 per thread); the column pairs (row, l) of V over
// the 192 threads of waves 1..3 (at most 2048: 11 per thread).  A is kept
// in its upper triangle only: element {x, y} lives at [min][max].
constexpr int kBlkPerThread = 3;
constexpr int kColPerThread = 11;
static_assert(kBlkPerThread * kThreads >= (kMaxDim / 2) * (kMaxDim / 2 + 1) / 2, "block list");
static_assert(kColPerThread * (kThreads - 64) >= kMaxDim * (kMaxDim / 2), "column list");

__device__ __forceinline__ int upper(int x, int y) { return x < y ? x * kLd + y : y * kLd + x; }

// V <- V J for the rotations in Jr (waves 1..3; vt: this thread's column pairs)
__device__ __forceinline__ void rotate_columns(double* V, const int* vt, const JacobiLds& Jr) {
  double nw[kColPerThread][2];
  int iv[kColPerThread][2];
#pragma unroll
  for (int i = 0; i < kColPerThread; ++i) {
    if (vt[i] >= 0) {
      const int row = vt[i] >> 8, l = vt[i] & 255;
      const double sl = Jr.s[l], cl = Jr.c[l];
      iv[i][0] = row * kLd + Jr.p[l];
      iv[i][1] = row * kLd + Jr.q[l];
      const double vp = V[iv[i][0]], vq = V[iv[i][1]];
      nw[i][0] = cl * vp - sl * vq;
      nw[i][1] = sl * vp + cl * vq;
    }
  }
#pragma unroll
  for (int i = 0; i < kColPerThread; ++i)
    if (vt[i] >= 0) {
      V[iv[i][0]] = nw[i][0];
      V[iv[i][1]] = nw[i][1];
    }
}

// Diagonalises the symmetric m x m matrix A (m even, LDS, stride kLd, both
// triangles on entry; on exit the diagonal holds the eigenvalues and only the
// upper triangle is meaningful) in place, accumulating the rotations into V
// (LDS, initialised by the caller).  Returns the number of sweeps, or -1
// without convergence in kMaxSweeps.  Every thread of the workgroup calls it.
//
// A round: wave 0 computes the round's rotations while waves 1..3 apply the
// previous round's rotations to V (the rotation parameters are double
// buffered), barrier, all threads update A, barrier.  A round whose
// rotations are all skipped leaves A and V alone.  Each thread loads all its
// elements before it stores any, so that their LDS latencies overlap.
__device__ int jacobi(double* A, double* V, int m, JacobiLds* J2) {
  const int tid = threadIdx.x;
  const int half = m / 2;
  if (m < 2) return 0;
  // this thread's blocks (k << 8 | l) and column pairs (row << 8 | l), -1 = none
  int bt[kBlkPerThread], vt[kColPerThread];
  {
    const int nblk = half * (half + 1) / 2;
#pragma unroll
    for (int i = 0; i < kBlkPerThread; ++i) {
      int b = tid + i * kThreads;
      bt[i] = -1;
      if (b < nblk) {
        int k = 0;
        while (b >= half - k) {   // row k holds blocks l = k .. half-1
          b -= half - k;
          ++k;
        }
        bt[i] = k << 8 | (k + b);
      }
    }
    const int u = tid - 64;
#pragma unroll
    for (int i = 0; i < kColPerThread; ++i) {
      const int e = u + i * (kThreads - 64);
      vt[i] = (u >= 0 && e < m * half) ? ((e / half) << 8 | (e % half)) : -1;
    }
  }
  if (tid == 0) J2[0].rotated = J2[1].rotated = 0;
  __syncthreads();
  int gr = 0;              // rounds so far, across sweeps (selects the buffer)
  bool pending = false;    // V still owes the rotations of the previous round
  int result = -1;
  for (int sweep = 0; sweep < kMaxSweeps && result < 0; ++sweep) {
    bool sweep_rot = false;
    for (int r = 0; r < m - 1; ++r, ++gr) {
      JacobiLds& J = J2[gr & 1];
      if (tid < 64) {
        if (tid < half) {
          int p, q;
          if (tid == 0) {
            p = r;
            q = m - 1;
          } else {
            p = r + tid;
            if (p >= m - 1) p -= m - 1;
            q = r - tid;
            if (q < 0) q += m - 1;
            if (p > q) {
              const int x = p;
              p = q;
              q = x;
            }
          }
          const double app = A[p * kLd + p], aqq = A[q * kLd + q], apq = A[p * kLd + q];
          double c = 1.0, s = 0.0, t = 0.0;
          if (apq != 0.0 && fabs(apq) > kRelTol * sqrt(fabs(app) * fabs(aqq))) {
            const double theta = (aqq - app) / (2.0 * apq);
            t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            J.rotated = 1;
          }
          J.p[tid] = p;
          J.q[tid] = q;
          J.c[tid] = c;
          J.s[tid] = s;
          J.t[tid] = t;
          J.apq[tid] = apq;
        }
      } else if (pending) {
        rotate_columns(V, vt, J2[(gr + 1) & 1]);
      }
      __syncthreads();
      const bool any = J.rotated != 0;
      // the other buffer's flag was read in the previous round; it is set
      // again only after the barrier that ends this round
      if (tid == 0) J2[(gr + 1) & 1].rotated = 0;
      pending = any;
      if (any) {
        sweep_rot = true;
        // A <- J^T A J on the 2x2 blocks (rows of rotation k, columns of rotation l)
        double nv[kBlkPerThread][4];
        int ia[kBlkPerThread][4];
#pragma unroll
        for (int i = 0; i < kBlkPerThread; ++i) {
          if (bt[i] >= 0) {
            const int k = bt[i] >> 8, l = bt[i] & 255;
            const int pk = J.p[k], qk = J.q[k];
            if (k == l) {
              ia[i][0] = pk * kLd + pk;
              ia[i][1] = pk * kLd + qk;
              ia[i][3] = qk * kLd + qk;
              const double dd = J.t[k] * J.apq[k];
              nv[i][0] = A[ia[i][0]] - dd;
              nv[i][1] = 0.0;
              nv[i][3] = A[ia[i][3]] + dd;
              ia[i][2] = ia[i][1];
              nv[i][2] = 0.0;
            } else {
              const int pl = J.p[l], ql = J.q[l];
              const double sk = J.s[k], ck = J.c[k], sl = J.s[l], cl = J.c[l];
              ia[i][0] = upper(pk, pl);
              ia[i][1] = upper(pk, ql);
              ia[i][2] = upper(qk, pl);
              ia[i][3] = upper(qk, ql);
              const double a = A[ia[i][0]], bq = A[ia[i][1]], cq = A[ia[i][2]], d = A[ia[i][3]];
              const double a1 = cl * a - sl * bq, b1 = sl * a + cl * bq;
              const double c1 = cl * cq - sl * d, d1 = sl * cq + cl * d;
              nv[i][0] = ck * a1 - sk * c1;
              nv[i][2] = sk * a1 + ck * c1;
              nv[i][1] = ck * b1 - sk * d1;
              nv[i][3] = sk * b1 + ck * d1;
            }
          }
        }
#pragma unroll
        for (int i = 0; i < kBlkPerThread; ++i)
          if (bt[i] >= 0) {
            A[ia[i][0]] = nv[i][0];
            A[ia[i][1]] = nv[i][1];
            A[ia[i][2]] = nv[i][2];
            A[ia[i][3]] = nv[i][3];
          }
      }
      __syncthreads();
    }
    if (!sweep_rot) result = sweep + 1;
  }
  // rotations of the last round still owed to V (only when the sweeps ran out)
  if (pending) {
    if (tid >= 64) rotate_columns(V, vt, J2[(gr + 1) & 1]);
    __syncthreads();
  }
  return result;
}

// rank of value v[r] among v[0..n): descending (or ascending) order, ties by index
__device__ int rank_of(const double* v, int n, int r, bool descending) {
  const double x = v[r];
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    const double y = v[j];
    const bool before = descending ? (y > x) : (y < x);
    rank += before || (y == x && j < r);
  }
  return rank;
}

__global__ __launch_bounds__(kThreads, 2) void pno_build_kernel(const dlpno_pno_pair* __restrict__ pairs,
                                                             int64_t n_pairs, const double* __restrict__ X,
                                                             const double* __restrict__ F, double t_cut,
                                                             double* __restrict__ occ, double* __restrict__ eps,
                                                             double* __restrict__ C, int32_t* __restrict__ n_kept,
                                                             int32_t* __restrict__ sweeps) {
  __shared__ double A[kMaxDim * kLd];
  __shared__ double V[kMaxDim * kLd];
  __shared__ JacobiLds J[2];
  __shared__ double lam[kMaxDim], sred[kThreads];
  __shared__ int order[kMaxDim], ired[kThreads], colsign[kMaxDim];
  __shared__ int s_n, s_bad;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;

  for (int64_t pi = blockIdx.x; pi < n_pairs; pi += gridDim.x) {
    const dlpno_pno_pair d = pairs[pi];
    const int N = d.dim, m = N + (N & 1);
    if (tid == 0) {
      s_n = 0;
      s_bad = 0;
    }

    // ---- pair density: D = sum_b w_b (X X^T + X^T X) / (2 (1 + delta_ij)) ----
    double acc[4][4] = {};
    const int ti = tid >> 4, tj = tid & 15;
    int64_t xo = d.off_X;
    for (int b = 0; b < 4; ++b) {
      if (!(d.blocks & (1 << b))) continue;
      // same spin 1/2, opposite spin 1; a diagonal pair's missing beta-alpha
      // block is the transpose of its alpha-beta block and adds the same
      double wb = b < 2 ? 0.5 : 1.0;
      if (b == 2 && d.diagonal && !(d.blocks & 8)) wb = 2.0;
      __syncthreads();
      for (int e = tid; e < N * N; e += kThreads) {
        const int r = e / N;
        V[r * kLd + (e - r * N)] = X[xo + e];
      }
      __syncthreads();
      xo += (int64_t)N * N;
      if (4 * ti < N && 4 * tj < N) {
        double blk[4][4] = {};
        for (int c = 0; c < N; ++c) {
          double xa[4], xb[4], ya[4], yb[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int a = min(4 * ti + i, N - 1), bb = min(4 * tj + i, N - 1);
            xa[i] = V[a * kLd + c];
            xb[i] = V[bb * kLd + c];
            ya[i] = V[c * kLd + a];
            yb[i] = V[c * kLd + bb];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) blk[i][j] += xa[i] * xb[j] + ya[i] * yb[j];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += wb * blk[i][j];
      }
    }
    __syncthreads();
    const double dscale = 1.0 / (2.0 * (d.diagonal ? 2.0 : 1.0));
    for (int e = tid; e < kMaxDim * kMaxDim; e += kThreads) {
      const int r = e >> 6, c = e & 63;
      if (r < m && c < m) A[r * kLd + c] = 0.0;
      if (r < m && c < m) V[r * kLd + c] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = 4 * ti + i, bb = 4 * tj + j;
        if (a < N && bb < N) {
          const double v = acc[i][j] * dscale;
          bad |= !isfinite(v);
          A[a * kLd + bb] = v;
        }
      }
    if (bad) s_bad = 1;
    __syncthreads();
    int status = 0;
    int sw1 = 0, sw2 = 0;
    if (s_bad) status = -3;
    if (status == 0) {
      sw1 = jacobi(A, V, m, J);
      if (sw1 < 0) status = -1;
    }

    // ---- occupations in descending order, truncation ----
    if (tid < N) lam[tid] = A[tid * kLd + tid];
    __syncthreads();
    if (tid < N) {
      const int rk = rank_of(lam, N, tid, true);
      order[rk] = tid;
      occ[d.off_v + rk] = status == 0 ? lam[tid] : 0.0;
      if (lam[tid] >= t_cut) atomicAdd(&s_n, 1);
    }
    __syncthreads();
    const int n = status == 0 ? s_n : 0;
    const int64_t co = d.off_C;

    if (n > 0) {
      // W = F V_k (N x n) in registers, F staged in A
      for (int e = tid; e < N * N; e += kThreads) {
        const int r = e / N;
        A[r * kLd + (e - r * N)] = F[d.off_F + e];
      }
      __syncthreads();
      double acc16[16];
      const int ok = lane < n ? order[lane] : 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) acc16[i] = 0.0;
      for (int b = 0; b < N; ++b) {
        const double v = V[b * kLd + ok];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc16[i] += A[min(w + 4 * i, N - 1) * kLd + b] * v;
      }
      // the kept natural orbitals go to C until the second eigenproblem is done
      for (int e = tid; e < N * n; e += kThreads) {
        const int r = e / n, k = e - r * n;
        C[co + (int64_t)r * N + k] = V[r * kLd + order[k]];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (w + 4 * i < N && lane < n) A[(w + 4 * i) * kLd + lane] = acc16[i];
      __syncthreads();
      // F_PNO = V_k^T W (n x n)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc16[i] = 0.0;
      for (int a = 0; a < N; ++a) {
        const double wv = A[a * kLd + lane];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc16[i] += V[a * kLd + order[min(w + 4 * i, n - 1)]] * wv;
      }
      __syncthreads();
      const int m2 = n + (n & 1);
      for (int e = tid; e < kMaxDim * kMaxDim; e += kThreads) {
        const int r = e >> 6, c = e & 63;
        if (r < m2 && c < m2) {
          A[r * kLd + c] = 0.0;
          V[r * kLd + c] = r == c ? 1.0 : 0.0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (w + 4 * i < n && lane < n) A[(w + 4 * i) * kLd + lane] = acc16[i];
      __syncthreads();
      sw2 = jacobi(A, V, m2, J);
      if (sw2 < 0) status = -2;

      // orbital energies in ascending order
      if (tid < n) lam[tid] = A[tid * kLd + tid];
      __syncthreads();
      if (tid < n) {
        const int rk = rank_of(lam, n, tid, false);
        order[rk] = tid;
        eps[d.off_v + rk] = lam[tid];
      }
      __syncthreads();
      // C = V_k U (columns in ascending energy), V_k back from C into A
      for (int e = tid; e < N * n; e += kThreads) {
        const int r = e / n, k = e - r * n;
        A[r * kLd + k] = C[co + (int64_t)r * N + k];
      }
      __syncthreads();
      const int uk = order[lane < n ? lane : 0];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc16[i] = 0.0;
      for (int j = 0; j < n; ++j) {
        const double u = V[j * kLd + uk];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc16[i] += A[min(w + 4 * i, N - 1) * kLd + j] * u;
      }
      // sign convention: the largest-magnitude element of each column is
      // positive (the first such row on ties)
      double best = -1.0;
      int bi = 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = w + 4 * i;
        if (r < N && fabs(acc16[i]) > best) {
          best = fabs(acc16[i]);
          bi = r;
        }
      }
      sred[tid] = best;
      ired[tid] = bi;
      __syncthreads();
      if (w == 0) {
        double bv = sred[lane];
        int br = ired[lane];
        for (int x = 1; x < 4; ++x) {
          const double v = sred[x * 64 + lane];
          const int rr = ired[x * 64 + lane];
          if (v > bv || (v == bv && rr < br)) {
            bv = v;
            br = rr;
          }
        }
        ired[lane] = br;
      }
      __syncthreads();
      const int srow = ired[lane];
      const int owner = srow & 3, slot = srow >> 2;
      if (w == owner) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i == slot) v = acc16[i];
        colsign[lane] = v < 0.0 ? -1 : 1;
      }
      __syncthreads();
      const double sg = colsign[lane] < 0 ? -1.0 : 1.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = w + 4 * i;
        if (r < N && lane < n) C[co + (int64_t)r * N + lane] = sg * acc16[i];
      }
    }
    // columns past n, energies past n
    for (int e = tid; e < N * N; e += kThreads) {
      const int r = e / N, k = e - r * N;
      if (k >= n) C[co + (int64_t)r * N + k] = 0.0;
    }
    if (tid < N && tid >= n) eps[d.off_v + tid] = 0.0;
    if (tid == 0) {
      n_kept[pi] = status == 0 ? n : status;
      if (sweeps) {
        sweeps[2 * pi] = sw1;
        sweeps[2 * pi + 1] = sw2;
      }
    }
    __syncthreads();
  }
}

// PNO overlaps of a coupling list: one workgroup per target pair p, C_p in
// LDS.  Per coupling, the shared rows of C_q go through registers into LDS;
// the next coupling's rows are loaded while this one is computed.  Each
// thread computes a tile of S (overlap_tile).  LDS rows are 68 doubles so
// that tiles load as 16-byte pairs.
constexpr int kLdO = 68;
constexpr int kPrefetch = kMaxDim * kMaxDim / kThreads;   // 16 elements per thread

// one coupling of the list, resolved on the host at prepare time so that the
// kernel needs one load per coupling (and issues it a coupling ahead)
struct OverlapItem {
  int64_t base;    // first element of the shared rows of C_q
  int64_t off_S;   // output block
  int32_t Nq, nq;  // source domain size and PNO count
  int32_t L;       // shared rows (0: the windows do not meet)
  int32_t shift;   // first shared row within the target's domain
};

// T x T tile of S per thread on a 16 x 16 grid of tiles (T = 2: blocks of
// at most 32 x 32, every thread busy; T = 4: up to 64 x 64)
template <int T>
__device__ __forceinline__ void overlap_tile(const double* Cq, const double* Cp, int shift, int L, int nq, int np_,
                                             double* out) {
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  if (T * ti >= nq || T * tj >= np_) return;
  double acc[T][T] = {};
  for (int x = 0; x < L; ++x) {
    double qv[T], pv[T];
#pragma unroll
    for (int h = 0; h < T; h += 2) {
      const double2 q = *reinterpret_cast<const double2*>(&Cq[x * kLdO + T * ti + h]);
      const double2 v = *reinterpret_cast<const double2*>(&Cp[(x + shift) * kLdO + T * tj + h]);
      qv[h] = q.x;
      qv[h + 1] = q.y;
      pv[h] = v.x;
      pv[h + 1] = v.y;
    }
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int j = 0; j < T; ++j) acc[i][j] += qv[i] * pv[j];
  }
#pragma unroll
  for (int i = 0; i < T; ++i) {
    const int c = T * ti + i;
    if (c < nq)
#pragma unroll
      for (int j = 0; j < T; ++j)
        if (T * tj + j < np_) out[(int64_t)c * np_ + T * tj + j] = acc[i][j];
  }
}

__global__ __launch_bounds__(kThreads, 2) void pno_overlap_kernel(const dlpno_pno_pair* __restrict__ pairs,
                                                                   const int32_t* __restrict__ nk,
                                                                   const int64_t* __restrict__ rowptr,
                                                                   const OverlapItem* __restrict__ items,
                                                                   int64_t n_pairs, const double* __restrict__ C,
                                                                   double* __restrict__ S) {
  __shared__ __attribute__((aligned(16))) double Cp[kMaxDim * kLdO];
  __shared__ __attribute__((aligned(16))) double Cq[kMaxDim * kLdO];
  const int tid = threadIdx.x;
  // element (row, column) = (w + 4 j, lane) of every C block a thread moves
  const int w = tid >> 6, lane = tid & 63;
  // workgroup it runs on XCD it % 8: each XCD takes a contiguous range of
  // target pairs, so that the source rows that neighbouring targets share
  // are found in its L2
  const int64_t chunk = (n_pairs + 7) / 8;
  for (int64_t it = blockIdx.x; it < 8 * chunk; it += gridDim.x) {
    const int64_t p = (it & 7) * chunk + (it >> 3);
    if (p >= n_pairs) continue;
    const dlpno_pno_pair dp = pairs[p];
    const int Np = dp.dim, np_ = nk[p];
    const int64_t e0 = rowptr[p], e1 = rowptr[p + 1];
    __syncthreads();
    if (lane < np_)
      for (int x = w; x < Np; x += 4) Cp[x * kLdO + lane] = C[dp.off_C + (int64_t)x * Np + lane];
    double pre[kPrefetch];
    OverlapItem cur{}, nxt{};
    if (e0 < e1) {
      cur = items[e0];
      if (e0 + 1 < e1) nxt = items[e0 + 1];
#pragma unroll
      for (int j = 0; j < kPrefetch; ++j) {
        const int x = w + 4 * j;
        pre[j] = (x < cur.L && lane < cur.nq) ? C[cur.base + (int64_t)x * cur.Nq + lane] : 0.0;
      }
    }
    for (int64_t cpl = e0; cpl < e1; ++cpl) {
      const OverlapItem r = cur;
      __syncthreads();   // C_p stored; the previous coupling's rows no longer read
#pragma unroll
      for (int j = 0; j < kPrefetch; ++j) {
        const int x = w + 4 * j;
        if (x < r.L && lane < r.nq) Cq[x * kLdO + lane] = pre[j];
      }
      __syncthreads();
      if (cpl + 1 < e1) {   // rows of the next coupling, in flight during this one
        cur = nxt;
        if (cpl + 2 < e1) nxt = items[cpl + 2];
#pragma unroll
        for (int j = 0; j < kPrefetch; ++j) {
          const int x = w + 4 * j;
          pre[j] = (x < cur.L && lane < cur.nq) ? C[cur.base + (int64_t)x * cur.Nq + lane] : 0.0;
        }
      }
      if (r.nq <= 32 && np_ <= 32)
        overlap_tile<2>(Cq, Cp, r.shift, r.L, r.nq, np_, S + r.off_S);
      else
        overlap_tile<4>(Cq, Cp, r.shift, r.L, r.nq, np_, S + r.off_S);
    }
  }
}

}  // namespace

struct dlpno_pno_plan {
  int64_t n_pairs = 0;
  dlpno_pno_pair* d_pairs = nullptr;
  std::vector<dlpno_pno_pair> pairs_h;
  int device = 0;
  // coupling list of dlpno_pno_overlap (device copies)
  int32_t* d_nk = nullptr;
  int64_t* d_rowptr = nullptr;
  OverlapItem* d_items = nullptr;
  bool overlap_ready = false;
};

static void free_overlap(dlpno_pno_plan* P) {
  for (void* ptr : {(void*)P->d_nk, (void*)P->d_rowptr, (void*)P->d_items})
    if (ptr) (void)hipFree(ptr);
  P->d_nk = nullptr;
  P->d_rowptr = nullptr;
  P->d_items = nullptr;
  P->overlap_ready = false;
}

using dlpno::fail;

extern "C" dlpno_status dlpno_pno_plan_create(const dlpno_pno_pair* pairs, int64_t n_pairs, int64_t n_X,
                                              int64_t n_F, int64_t n_C, int64_t n_v, dlpno_pno_plan** out) {
  if (!out) return fail(DLPNO_ERR_INVALID_ARG, "pno_plan_create: out is NULL");
  *out = nullptr;
  if (n_pairs < 0 || (n_pairs > 0 && !pairs)) return fail(DLPNO_ERR_INVALID_ARG, "pno_plan_create: pairs");
  for (int64_t p = 0; p < n_pairs; ++p) {
    const dlpno_pno_pair& d = pairs[p];
    const std::string at = "pno pair " + std::to_string(p) + ": ";
    if (d.dim < 1 || d.dim > kMaxDim) return fail(DLPNO_ERR_DIM_RANGE, at + "dim outside 1..64");
    if (d.blocks & ~15) return fail(DLPNO_ERR_INVALID_ARG, at + "block mask");
    if (d.diagonal != 0 && d.diagonal != 1) return fail(DLPNO_ERR_INVALID_ARG, at + "diagonal flag");
    if (d.first < 0) return fail(DLPNO_ERR_DIM_RANGE, at + "negative domain start");
    const int64_t n2 = (int64_t)d.dim * d.dim;
    const int64_t nb = __builtin_popcount((unsigned)d.blocks);
    if (d.off_X < 0 || (nb > 0 && d.off_X + nb * n2 > n_X)) return fail(DLPNO_ERR_ALIGNMENT, at + "X range");
    if (d.off_F < 0 || d.off_F + n2 > n_F) return fail(DLPNO_ERR_ALIGNMENT, at + "F range");
    if (d.off_C < 0 || d.off_C + n2 > n_C) return fail(DLPNO_ERR_ALIGNMENT, at + "C range");
    if (d.off_v < 0 || d.off_v + d.dim > n_v) return fail(DLPNO_ERR_ALIGNMENT, at + "occupation range");
  }
  auto* P = new (std::nothrow) dlpno_pno_plan;
  if (!P) return fail(DLPNO_ERR_OOM, "pno_plan_create: host allocation");
  P->n_pairs = n_pairs;
  P->pairs_h.assign(pairs, pairs + n_pairs);
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return fail(DLPNO_ERR_HIP, "pno_plan_create: hipGetDevice");
  }
  if (n_pairs > 0) {
    if (hipMalloc(&P->d_pairs, n_pairs * sizeof(dlpno_pno_pair)) != hipSuccess) {
      delete P;
      return fail(DLPNO_ERR_OOM, "pno_plan_create: device descriptors");
    }
    if (hipMemcpy(P->d_pairs, pairs, n_pairs * sizeof(dlpno_pno_pair), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(P->d_pairs);
      delete P;
      return fail(DLPNO_ERR_HIP, "pno_plan_create: descriptor upload");
    }
  }
  *out = P;
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_pno_build(dlpno_pno_plan* plan, const double* X, const double* F, double t_cut,
                                        double* occ, double* eps, double* C, int32_t* n_kept, int32_t* sweeps,
                                        void* stream) {
  if (!plan) return fail(DLPNO_ERR_INVALID_ARG, "pno_build: plan is NULL");
  if (plan->n_pairs == 0) return DLPNO_OK;
  if (!F || !occ || !eps || !C || !n_kept) return fail(DLPNO_ERR_INVALID_ARG, "pno_build: NULL buffer");
  if (!std::isfinite(t_cut)) return fail(DLPNO_ERR_INVALID_ARG, "pno_build: t_cut not finite");
  const int64_t grid = plan->n_pairs < (1 << 20) ? plan->n_pairs : (1 << 20);
  hipLaunchKernelGGL(pno_build_kernel, dim3((unsigned)grid), dim3(kThreads), 0, (hipStream_t)stream,
                     plan->d_pairs, plan->n_pairs, X, F, t_cut, occ, eps, C, n_kept, sweeps);
  if (hipGetLastError() != hipSuccess) return fail(DLPNO_ERR_HIP, "pno_build: launch");
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_pno_plan_destroy(dlpno_pno_plan* plan) {
  if (!plan) return DLPNO_OK;
  if (plan->d_pairs) (void)hipFree(plan->d_pairs);
  free_overlap(plan);
  delete plan;
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_pno_overlap_prepare(dlpno_pno_plan* plan, const int32_t* n_kept, const int64_t* rowptr,
                                                  const int32_t* src, const int64_t* off_S, int64_t n_S) {
  if (!plan || !n_kept || !rowptr) return fail(DLPNO_ERR_INVALID_ARG, "pno_overlap_prepare: NULL argument");
  const int64_t P = plan->n_pairs;
  if (rowptr[0] != 0) return fail(DLPNO_ERR_INVALID_ARG, "pno_overlap_prepare: rowptr[0] != 0");
  std::vector<int32_t> nk(P);
  for (int64_t p = 0; p < P; ++p) {
    if (n_kept[p] < 0 || n_kept[p] > plan->pairs_h[p].dim)
      return fail(DLPNO_ERR_DIM_RANGE, "pno_overlap_prepare: n_kept of pair " + std::to_string(p));
    nk[p] = n_kept[p] > 0 ? n_kept[p] : 1;
    if (rowptr[p + 1] < rowptr[p]) return fail(DLPNO_ERR_INVALID_ARG, "pno_overlap_prepare: rowptr not monotonic");
  }
  const int64_t n_cpl = rowptr[P];
  if (n_cpl > 0 && (!src || !off_S)) return fail(DLPNO_ERR_INVALID_ARG, "pno_overlap_prepare: NULL src/off_S");
  for (int64_t p = 0; p < P; ++p)
    for (int64_t e = rowptr[p]; e < rowptr[p + 1]; ++e) {
      if (src[e] < 0 || src[e] >= P) return fail(DLPNO_ERR_DIM_RANGE, "pno_overlap_prepare: source pair out of range");
      if (off_S[e] < 0 || off_S[e] + (int64_t)nk[src[e]] * nk[p] > n_S)
        return fail(DLPNO_ERR_ALIGNMENT, "pno_overlap_prepare: block " + std::to_string(e) + " outside S");
    }
  std::vector<OverlapItem> items(n_cpl);
  for (int64_t p = 0; p < P; ++p) {
    const dlpno_pno_pair& dp = plan->pairs_h[p];
    for (int64_t e = rowptr[p]; e < rowptr[p + 1]; ++e) {
      const dlpno_pno_pair& dq = plan->pairs_h[src[e]];
      const int lo = std::max(dp.first, dq.first), hi = std::min(dp.first + dp.dim, dq.first + dq.dim);
      OverlapItem& it = items[e];
      it.L = std::max(hi - lo, 0);
      it.base = dq.off_C + (int64_t)(it.L > 0 ? lo - dq.first : 0) * dq.dim;
      it.off_S = off_S[e];
      it.Nq = dq.dim;
      it.nq = nk[src[e]];
      it.shift = it.L > 0 ? lo - dp.first : 0;
    }
  }
  free_overlap(plan);
  auto up = [&](void** dst, const void* h, size_t bytes) -> bool {
    if (bytes == 0) return true;
    if (hipMalloc(dst, bytes) != hipSuccess) return false;
    return hipMemcpy(*dst, h, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up((void**)&plan->d_nk, nk.data(), P * sizeof(int32_t)) ||
      !up((void**)&plan->d_rowptr, rowptr, (P + 1) * sizeof(int64_t)) ||
      !up((void**)&plan->d_items, items.data(), n_cpl * sizeof(OverlapItem))) {
    free_overlap(plan);
    return fail(DLPNO_ERR_OOM, "pno_overlap_prepare: device upload");
  }
  plan->overlap_ready = true;
  return DLPNO_OK;
}

extern "C" dlpno_status dlpno_pno_overlap(dlpno_pno_plan* plan, const double* C, double* S, void* stream) {
  if (!plan) return fail(DLPNO_ERR_INVALID_ARG, "pno_overlap: plan is NULL");
  if (!plan->overlap_ready) return fail(DLPNO_ERR_INVALID_ARG, "pno_overlap: no coupling list (call _prepare)");
  if (plan->n_pairs == 0) return DLPNO_OK;
  if (!C || !S) return fail(DLPNO_ERR_INVALID_ARG, "pno_overlap: NULL buffer");
  const int64_t slots = 8 * ((plan->n_pairs + 7) / 8);
  const int64_t grid = slots < (1 << 20) ? slots : (1 << 20);
  hipLaunchKernelGGL(pno_overlap_kernel, dim3((unsigned)grid), dim3(kThreads), 0, (hipStream_t)stream, plan->d_pairs,
                     plan->d_nk, plan->d_rowptr, plan->d_items, plan->n_pairs, C, S);
  if (hipGetLastError() != hipSuccess) return fail(DLPNO_ERR_HIP, "pno_overlap: launch");
  return DLPNO_OK;
}
