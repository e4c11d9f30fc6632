// Internal device tables and kernel launch interfaces of the DLPNO residual library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dlpno {

// Pair table (one per retained pair).
struct PairDev {
  int32_t i, j, n, m;
  int32_t nblk, blk0;        // stored blocks, global index of the first one
  int64_t off_B, off_T, off_K, off_eps;
};

// Block table (one per stored spin block).
struct BlockDev {
  int32_t pair, code, n, anti;   // code 0 AA, 1 BB, 2 AB, 3 BA; anti: driver is K - K^T
  int64_t off_T, off_K, off_eps;
  int32_t s1, s2;                // spins of electron i and j (0 alpha, 1 beta)
  double fsum;                   // f^s1_ii + f^s2_jj
  double w;                      // energy weight (1/2 same spin, 1 opposite spin)
  int64_t off_ws;                // first partial slot of this block (n*n doubles per slot)
  int32_t nslot, slot_proj;      // partial slots; first projection slot (== nslot: none)
  int32_t rows, cols;            // rows / columns inside the virtual spaces of s1 / s2 (the
                                 // others are SOMO functions of an alpha index: residual zero)
};

// Coupling table (CSR order by target pair).
struct CplDev {
  int32_t src, nsrc;
  int64_t off_S;                 // [c][a]: n_src rows x n_target cols
};

// One projection term: coupling e applied to block slot b of its target.
struct TermDev {
  int64_t src_off;               // source block in T; -1 = no term for this block
  double w;                      // Fock weight; residual gets -w S X S^T
  int32_t trans;                 // X = source^T when trans
  int32_t src_blk;               // global index of the source block
};

// One hole-hole coupling whose weights carry the quadratic term (quadratic.hip):
// per active target block, the term to rewrite, the target block in T, the
// static weight -(k i | l j) and the factor -c (c = 1/2 same spin, 1 opposite).
struct QuadCpl {
  int64_t off_S;        // overlap block [c][a], n_q x n_p
  int64_t off_K;        // K of the source pair, n_q x n_q
  int64_t off_G;        // G = S_pq K_(k,l) S_pq^T in the plan's table, n_p x n_p
  int32_t np, nq;
  int32_t transK;       // k > l: K_(k,l) is K_q transposed
  int32_t nblk;         // active target blocks (1..4)
  int64_t term[4];      // index into the term table
  int64_t off_T[4];     // target block in T
  double w0[4], c[4];
};

// Quadratic part of the occupied Fock intermediate (quadratic.hip): one
// contribution <G, T_(j,n)> to F^s_{mj} for each spin s, over the blocks of
// the dotted pair {j, n} with the ordered spins (s, s_n), s_n either spin.
struct OccCtb {
  int64_t off_G;          // G (n x n): in the plan's factor table, or the dotted pair's K (from_K)
  int32_t n, from_K;
  int32_t key[2];         // index of F^s_{mj} for s = 0, 1 (-1: none)
  int64_t off_T[2][2];    // per spin, up to two amplitude blocks (-1: none)
  int32_t tr[2][2];       // 1: the block enters transposed, <G^T, T>
};
// A projection term whose weight the intermediate dresses: w = w0 + F[key].
struct OccTerm {
  int64_t term;           // index into the term table
  int32_t key, pad;
  double w0;              // the occupied Fock element
};

// One contraction of the ring/exchange term (ring.hip):  Out += w L^T op(T_q) M
// with L and M n_q x n_p row-major blocks ([c][a]) read from the overlap
// buffer S or the ring integral buffer, op(T_q) = T_q or T_q^T.
struct RxTerm {
  int64_t src_off;      // source amplitude block in T, n_q x n_q
  int64_t off_L, off_M;
  int32_t nq;
  int32_t flags;        // kRxL / kRxM: that factor is in the ring integral buffer; kRxTrans: op = ^T
  double w;
};
constexpr int32_t kRxL = 1, kRxM = 2, kRxTrans = 4;
// The ring contractions of one target block, summed into its last partial slot.
struct RxUnit {
  int32_t blk;          // global block index
  int32_t pad;
  int64_t t0, t1;       // terms [t0, t1)
};

// ITEM_LADDER2: ladder items of an FP64 plan run by the launch at two waves
// per SIMD (at most three tiles of 16 PNOs and the variants below).
// ITEM_LADDER4: four-tile ladder items of an FP64 plan, each run by a whole
// workgroup (cooperative variants below), also at two waves per SIMD.
// ITEM_PROJ2: projection items of an FP64 plan with targets and sources of
// at most three tiles (variants of kProjTwoWave), at two waves per SIMD.
enum ItemKind { ITEM_LADDER = 0, ITEM_PROJ = 1, ITEM_LADDER2 = 2, ITEM_LADDER4 = 3, ITEM_PROJ2 = 4 };
constexpr int kKinds = 5;
// launch order of the kinds within one residual
constexpr int kKindOrder[kKinds] = {ITEM_LADDER2, ITEM_LADDER4, ITEM_LADDER, ITEM_PROJ2, ITEM_PROJ};

// One scheduled unit of the grouped kernel.
struct Item {
  int32_t kind;
  int32_t variant;               // compiled tile variant (see variants below)
  int32_t pair;
  int32_t bslot0;                // first block slot of the pair handled
  int32_t slot;                  // partial slot written
  int32_t ta0;                   // first a-tile (ladder)
  int32_t lo, hi;                // Q range (ladder) or coupling range (projection)
};

// Work queues of one launch, one per XCD.  The items of one pair and one Q or
// coupling range (one partial slot) read the same B^Q or S slices; the
// schedule puts them in the same queue, so that they run on one XCD at about
// the same time and the repeated reads hit that XCD's L2.
constexpr int kQueues = 8;
struct WorkQueues {
  int32_t off[kQueues + 1];      // queue k holds items [off[k], off[k+1])
  int32_t* counter;              // kQueues heads, zeroed before each launch
};

// Pops the calling wave's next item, or returns -1 once every queue is empty.
// Workgroups are dispatched to the eight XCDs round-robin by workgroup index,
// so a workgroup starts on queue blockIdx.x % kQueues, the one of its own
// XCD.  A wave drains that queue, then the following ones in turn; a failed
// pop moves it on for good, so every wave ends after at most kQueues failed
// pops and every item is taken exactly once.
__device__ __forceinline__ int next_item(const WorkQueues& Q, int& q, int& left) {
  while (left > 0) {
    int idx = 0;
    if ((threadIdx.x & 63) == 0) idx = atomicAdd(Q.counter + q, 1);
    idx = __builtin_amdgcn_readfirstlane(idx) + Q.off[q];
    if (idx < Q.off[q + 1]) return idx;
    q = q + 1 == kQueues ? 0 : q + 1;
    --left;
  }
  return -1;
}

// FP64 ladder: largest number of k-steps of 4 in the last 16-wide tile (that
// is, at most 4 kColStrips PNOs in it) for which the last a-tile runs as
// column strips of the four-block 4x4x4 MFMA.  Each strip costs about 0.22 of
// a 16x16x4 MFMA plus a DPP broadcast of its operand; with three strips the
// broadcasts eat the gain.
constexpr int kColStrips = 2;

// Tile variants compiled into the grouped kernel.
// Ladder: (NT tiles of 16 per PNO index, NB blocks per item, NTA a-tiles per item).
struct LadderVariant { int nt, nb, nta; };
struct ProjVariant { int nt, nb; };
constexpr int kNumLadderVariants = 13;
constexpr LadderVariant kLadderVariants[kNumLadderVariants] = {
    {1, 4, 1}, {1, 2, 1}, {1, 1, 1}, {2, 4, 2}, {2, 2, 2}, {2, 1, 2}, {2, 4, 1}, {3, 1, 3}, {4, 1, 2},
    {4, 2, 4}, {4, 1, 4}, {3, 2, 3}, {4, 2, 2}};
// variants compiled into the split-precision kernel only (two blocks per item
// for three- and four-tile pairs: each B^Q slice serves both)
constexpr bool kLadderSplitOnly[kNumLadderVariants] = {false, false, false, false, false, false, false,
                                                       false, false, false, false, true, true};
// the cooperative variants (FP64 only): a workgroup per item of two blocks
// (kLadderCoopPair) or one
constexpr int kLadderCoopPair = 9, kLadderCoopOne = 10;
constexpr bool kLadderCoop[kNumLadderVariants] = {false, false, false, false, false, false, false, false, false,
                                                  true, true, false, false};
// ladder variants compiled into the two-wave launch: their X operands fit a
// 40-operand LDS slab (or registers) and their registers fit 256 per lane
constexpr bool kLadderTwoWave[kNumLadderVariants] = {true, true, true, false, true, true, false, true, false,
                                                     false, false, false, false};
constexpr int kNumProjVariants = 9;
constexpr ProjVariant kProjVariants[kNumProjVariants] = {
    {1, 4}, {1, 2}, {1, 1}, {2, 4}, {2, 2}, {2, 1}, {3, 2}, {3, 1}, {4, 1}};
// projection variants compiled into the two-wave launch (sources of at most
// three tiles): their accumulators and S operands fit 256 registers per lane
constexpr bool kProjTwoWave[kNumProjVariants] = {true, true, true, false, true, true, false, true, false};

// Arguments of the grouped kernel (templated on the operand type).
template <typename F>
struct GroupedArgs {
  const Item* items;
  WorkQueues q;
  const PairDev* pairs;
  const BlockDev* blocks;
  const CplDev* cpl;
  const TermDev* terms;          // [coupling][4]
  const F* B;
  const F* S;
  const F* T;
  double* ws;
  // 1: same-spin blocks hold antisymmetric amplitudes, so their ladder and
  // projection contributions are antisymmetric too; only the tiles on and
  // below the diagonal are computed and the others are stored mirrored.
  // 0 (vector-Jacobian products, whose cotangents are general): all tiles.
  int32_t anti;
  int32_t* err;                  // device status word: kErrNoBody set by an item without a compiled body
};

// Bits of the device status word (the plan's non-finite flag).
constexpr int32_t kErrNonfinite = 1;   // a residual element was NaN or Inf
constexpr int32_t kErrNoBody = 2;      // a work item had no compiled kernel body (schedule/kernel mismatch)

// grouped_f64.hip, grouped_f32.hip
// kind: ITEM_LADDER or ITEM_PROJ, and in FP64 also ITEM_LADDER2, ITEM_LADDER4
// or ITEM_PROJ2; every item of `a` must be of that kind
hipError_t launch_grouped_f64(const GroupedArgs<double>& a, int kind, int workers, hipStream_t s);
hipError_t launch_grouped_f32(const GroupedArgs<float>& a, int kind, int workers, hipStream_t s);
hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s);
hipError_t launch_quad_prepare(const QuadCpl* list, int64_t n, const double* S, const double* K, double* G,
                               hipStream_t s);
hipError_t launch_quad_weights(const QuadCpl* list, int64_t n, const double* G, const double* T, TermDev* terms,
                               hipStream_t s);
// F^s_{mj} from T (dots per contribution, then per key in CSR order), the
// dressed weights of the listed terms and the per-block diagonal shift
// F^{s1}_ii + F^{s2}_jj
struct OccArgs {
  const OccCtb* ctb;
  int64_t n_ctb;
  const double* G;
  const double* K;
  double* dots;             // [2 n_ctb]
  const int64_t* key_rowptr; // [n_keys + 1] into key_src
  const int64_t* key_src;   // entries of dots, in a fixed order
  int64_t n_keys;
  double* F;                // [n_keys]
  const OccTerm* oterms;
  int64_t n_oterms;
  TermDev* terms;
  const int32_t* blk_key;   // [2 n_blocks]: keys of F^{s1}_ii and F^{s2}_jj (-1: none)
  int32_t n_blocks;
  double* shift;            // [n_blocks]
};
hipError_t launch_occ_weights(const OccArgs& a, const double* T, hipStream_t s);
// G[offs[b] ..] (ns[b] x ns[b]) transposed in place, for every b < count
hipError_t launch_transpose_blocks(const int64_t* offs, const int32_t* ns, int64_t count, double* G, hipStream_t s);
// ring.hip: every unit's ring contractions into its block's last partial slot
hipError_t launch_ring(const RxUnit* units, int64_t n_units, const RxTerm* terms, const BlockDev* blocks,
                       const double* T, const double* S, const double* ring_ints, double* ws, hipStream_t s);

// elementwise.hip
// DIIS on device.  State lives in a small device struct; vectors in rings.
struct DiisState {
  int32_t count;           // stored vectors (<= max)
  int32_t head;            // ring slot of the newest vector
  int32_t max;
  int32_t start;
  int32_t iter;            // iterations done (history index)
  int32_t drops;           // vectors dropped for ill conditioning since the reset
  int32_t pad[2];
  double gram[8][8];       // <e_a, e_b> by ring slot
  double coef[8];          // extrapolation coefficients by ring slot
};
struct FinishArgs {
  const BlockDev* blocks;
  int32_t n_blocks;
  const double* T;         // amplitudes the residual is evaluated at
  const double* K;
  const double* eps_a;
  const double* eps_b;
  const double* ws;
  double* R;               // residual out (may be null when only the update is wanted)
  double* T_new;           // Jacobi update out (null: no update)
  double* e_block;         // per block energy of T_new
  double* rmax_block;      // per block max |R|
  int32_t* nonfinite;      // status word: kErrNonfinite set when a residual element is not finite
  int32_t with_driver;     // 0: R = D o T + partials (linear part only, used by the VJP)
  int32_t no_partials;     // 1: the partial slots are not read (T = 0: the grouped launches add nothing)
  const double* drv;       // when set, replaces the driver: R = drv + D o T + partials
  // DIIS ring: when ring != null, T_new -> ring_vecs[head], err = T_new - T -> ring_errs[head]
  const DiisState* ring;
  double* ring_vecs;
  double* ring_errs;
  int64_t ring_stride;
  const double* shift;     // when set: R -= shift[block] * T (diagonal part of the occupied intermediate)
};
hipError_t launch_finish(const FinishArgs& a, hipStream_t s);
// flag |= 1 when some element of x[0..n) is not zero (NaN included); the caller zeroes flag
hipError_t launch_any_nonzero(const double* x, int64_t n, int32_t* flag, hipStream_t s);

struct UpdateArgs {         // Jacobi from a given residual
  const BlockDev* blocks;
  int32_t n_blocks;
  const double* T;
  const double* R;
  const double* K;
  const double* eps_a;
  const double* eps_b;
  double* T_new;
  double* e_block;
};
hipError_t launch_update(const UpdateArgs& a, hipStream_t s);

// F12 pair energies of every stored block (elementwise.hip, f12_kernel)
struct F12Args {
  const BlockDev* blocks;
  int32_t n_blocks;
  const double* T;         // converged amplitudes
  const double* W;         // (V + C) per block, amplitude layout
  const double* scal;      // [n_blocks][6]: V, V', B1..B4
  double* e_block;         // [n_blocks] out
};
hipError_t launch_f12(const F12Args& a, hipStream_t s);

struct ReduceArgs {
  const PairDev* pairs;
  const BlockDev* blocks;
  int32_t n_blocks;
  int32_t n_pairs;
  const double* e_block;
  const double* rmax_block;
  double* e_pair;          // [4 n_pairs] (may be null)
  double* e_total;         // scalar (may be null)
  double* rmax;            // scalar (may be null)
  double* hist;            // per-iteration history [cap][2], indexed by *iter (may be null)
  int32_t* iter;           // device iteration counter (may be null)
  int32_t hist_cap;
  double* partial;         // [2 kReduceParts] scratch of the two-stage reduction
};
constexpr int kReduceParts = 64;
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);

hipError_t launch_diis_slot(DiisState* st, hipStream_t s);          // advance head before finish
hipError_t launch_diis_dots(const double* errs, int64_t n, DiisState* st, double* partial,
                            int nparts, hipStream_t s);
hipError_t launch_diis_solve(DiisState* st, const double* partial, int nparts, hipStream_t s);
hipError_t launch_diis_extrap(const double* vecs, int64_t n, const DiisState* st, double* T,
                              hipStream_t s);
hipError_t launch_diis_reset(DiisState* st, int max, int start, hipStream_t s);

// precision copies
hipError_t launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s);
hipError_t launch_copy(double* y, const double* x, int64_t n, hipStream_t s);
// same-spin (anti) blocks of T replaced by their antisymmetric part
hipError_t launch_antisymmetrize(const BlockDev* blocks, int n_blocks, double* T, hipStream_t s);
hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t s);

}  // namespace dlpno
