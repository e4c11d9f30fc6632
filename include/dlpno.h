/*
 * dlpno.h -- C ABI of the MI355X open-shell DLPNO doubles-residual library.
 *
 * The library evaluates, for every retained occupied pair p = (i, j) and every
 * stored high-spin block s s' of that pair, the doubles residual in the pair's
 * own PNO basis (the paper solves "the CC residual equations" in the truncated
 * PNO basis, Sec. II.B.3; spin cases per pair class, Sec. II.A; one
 * spin-independent PNO set per pair, Sec. II.B.2 and II.B.4):
 *
 *   R^{ss'}_p = K^{ss'}_p + (eps^s_a + eps^s'_b - f^s_ii - f^s'_jj) T^{ss'}_p
 *             - sum_{k in occ_s,  k != i} f^s_ki  S_{p,kj} T^{ss'}_{kj} S_{kj,p}
 *             - sum_{k in occ_s', k != j} f^s'_kj S_{p,ik} T^{ss'}_{ik} S_{ik,p}
 *             + sum_Q B^Q_p T^{ss'}_p (B^Q_p)^T
 *
 * with K^{AA} = K^{BB} = K_p - K_p^T, K^{AB} = K^{BA} = K_p, and
 * T_{(k,l)}, k > l, the transposed spin-swapped block of (l, k); then the
 * Jacobi update T' = T - R / D, pair energies w <K^{ss'}, T'> (w = 1/2 for
 * same spin, 1 for opposite spin) and Pulay DIIS.
 *
 * Conventions for every entry point:
 *   - device pointers are HIP device memory owned by the caller and must stay
 *     valid until the work queued on `stream` has finished;
 *   - host pointers are read during the call only (the plan copies them);
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream);
 *   - nothing throws or aborts across the ABI: every call returns a status;
 *   - for identical inputs and an identical schedule every result is bitwise
 *     reproducible (no floating point atomics; all reductions run in a fixed
 *     order).  The schedule (worker count, items per wave, the autotuner's
 *     choices) decides how the auxiliary and coupling ranges are cut into
 *     partial sums, so plans with different schedules agree to rounding only;
 *   - a plan is not thread safe; calls on one plan must be serialised.
 */
#ifndef DLPNO_H
#define DLPNO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DLPNO_OK = 0,
  DLPNO_ERR_INVALID_ARG = -1,   /* NULL pointer, bad enum, inconsistent descriptor */
  DLPNO_ERR_DIM_RANGE = -2,     /* npno outside 1..64, naux outside 1..65536, index range */
  DLPNO_ERR_ALIGNMENT = -3,     /* buffer offsets outside the declared buffer sizes */
  DLPNO_ERR_HIP = -4,           /* a HIP runtime call failed */
  DLPNO_ERR_NONFINITE = -5,     /* a residual element was NaN or Inf */
  DLPNO_ERR_NOT_CONVERGED = -6, /* dlpno_solve: no convergence in max_iter, or divergence */
  DLPNO_ERR_OOM = -7,           /* device allocation failed */
  DLPNO_ERR_UNSUPPORTED = -8    /* precision / option not available for this call */
} dlpno_status;

/* Arithmetic of the ladder and projection contractions.  Dressing, Jacobi
 * update, energies and DIIS are always FP64.
 *   FP64     FP64 MFMA
 *   FP32     FP32 MFMA, FP32 copies of B and S made at plan creation
 *   BF16X2   BF16 hi+lo operand splitting on MFMA, FP32 accumulation
 *   FP16X2   FP16 hi+lo splitting with power-of-two scaling, FP32 accumulation */
typedef enum { DLPNO_FP64 = 0, DLPNO_FP32 = 1, DLPNO_BF16X2 = 2, DLPNO_FP16X2 = 3 } dlpno_precision;

/* Spin-block mask bits, also the storage order of a pair's blocks. */
enum { DLPNO_AA = 1, DLPNO_BB = 2, DLPNO_AB = 4, DLPNO_BA = 8 };

/* One retained pair (i <= j).  Offsets are element offsets into the buffers
 * of dlpno_inputs / the amplitude buffers:
 *   off_B   B_p, [Q][a][c], naux x npno x npno, symmetric in (a, c)
 *   off_T   first stored block of the pair in T / R / dT buffers; the stored
 *           blocks follow back to back in the order AA, BB, AB, BA, each
 *           npno x npno row-major [a][b] (a on electron i, b on electron j)
 *   off_K   K_p = (i a | j b), npno x npno row-major
 *   off_eps virtual PNO energies, npno values in eps_a and in eps_b
 * `blocks` must equal the rule of Sec. II.A for (i, j) given is_somo: a block
 * s s' is present iff i in occ_s, j in occ_s' (SOMOs are alpha-occupied only),
 * not (s == s' and i == j), and BA is absent for i == j. */
typedef struct {
  int32_t i, j;
  int32_t npno;      /* 1..64 */
  int32_t naux;      /* 1..65536 */
  uint32_t blocks;   /* DLPNO_AA | DLPNO_BB | DLPNO_AB | DLPNO_BA */
  int32_t n_somo_virt; /* 0, or the number of SOMOs appended to the pair's PNOs (Sec. II.B.4):
                        * the last n_somo_virt of the npno virtual functions are SOMOs, which
                        * are virtual for beta electrons only.  B, K, S and eps cover all npno
                        * functions (the SOMO part of an overlap block is the identity); every
                        * residual element whose alpha virtual index falls on a SOMO function
                        * is zero, and amplitudes must be zero there.  0 <= n_somo_virt <
                        * npno, at most the number of SOMOs. */
  int64_t off_B, off_T, off_K, off_eps;
} dlpno_pair;

/* One projection coupling of a target pair p = (i, j) (CSR row of p):
 *   side 0: occupied k replaces i, source pair {k, j}, weight f^s[k][i]
 *   side 1: occupied k replaces j, source pair {i, k}, weight f^s'[k][j]
 * off_S: the overlap block between the source PNOs (rows, n_src) and the
 * target PNOs (columns, n_target), row-major: element [c][a] = <c_src|a_tgt>.
 * The library applies it to every spin block of the target for which the
 * source block exists (Sec. II.B.2: one overlap set serves all spins). */
typedef struct {
  int32_t src_pair;
  int32_t k;
  int32_t side;
  int32_t reserved;
  int64_t off_S;
} dlpno_coupling;

/* One hole-hole ladder coupling of a target pair p = (i, j) (CSR row of p;
 * the first slice of the CCSD terms beyond the model above): the ordered
 * occupied pair (k, l), whose source pair is {min(k, l), max(k, l)}.  Every
 * target block s s' with k in occ_s and l in occ_s' gets
 *     + w S_{p,kl} T^{ss'}_{(k,l)} S_{kl,p},   w = (k i | l j)  (chemists' notation),
 * with T_{(k,l)} for k > l the transposed s' s block of (l, k) and k = l only
 * for s != s'.  This is the spin-orbital term 1/2 sum_KL <KL||IJ> t_KL^AB of
 * the CCSD doubles residual in the pair's PNOs (Sec. II.B.3 solves the CC
 * residual equations in that basis).  off_S: the overlap block between the
 * source PNOs (rows) and the target PNOs (columns) as in dlpno_coupling; a
 * source equal to the target needs an identity block.  Every ordered (k, l)
 * is one coupling. */
typedef struct {
  int32_t src_pair;
  int32_t k, l;
  int32_t reserved;
  int64_t off_S;
  double w;
} dlpno_hh_coupling;

/* One ring/exchange coupling of a target pair p = (i, j) (CSR row of p; a
 * further slice of the CCSD terms beyond the model above).  role 0 keeps the
 * target's first occupied index, x = i, with y = j; role 1 keeps x = j, with
 * y = i.  m is the replacing occupied orbital and src_pair the retained pair
 * {min(x, m), max(x, m)} (the target itself when m = y).  In
 * dlpno_inputs.ring_ints, two row-major n_src x n_target blocks [e][b]:
 *     X at off_X:  (m e | b y),   J at off_J:  (m y | b e)   (chemists' notation),
 * e over the source's PNOs, b over the target's.  off_S: the overlap block
 * between the source PNOs (rows) and the target PNOs (columns) as in
 * dlpno_coupling (an identity block when the source is the target).  The
 * couplings add the spin-orbital term P(IJ) P(AB) sum_ME t_IM^AE <MB||EJ> of
 * the CCSD doubles residual, <MB||EJ> = (m e | b j) - (m j | b e) within
 * each spin, linear in the amplitudes, to every stored block: per block,
 * spin of M and orientation, terms +-S_{p,q} op(T_q) X or J (and their
 * transposes) over the source blocks that exist.  A diagonal target (i == j)
 * lists role 0 only; each of its couplings serves both index orders.  The
 * contractions run in FP64 on the FP64 amplitudes in every precision (in
 * dlpno_solve_mixed also on the corrections of the low-precision
 * iterations: the term is linear).  The vector-Jacobian product refuses
 * such plans. */
typedef struct {
  int32_t src_pair;
  int32_t m;
  int32_t role;
  int32_t reserved;
  int64_t off_S, off_X, off_J;
} dlpno_ring_coupling;

/* Problem description (all host memory, copied by dlpno_plan_create). */
typedef struct {
  int32_t n_occ;
  int32_t n_pairs;
  int64_t n_couplings;
  const uint8_t* is_somo;          /* [n_occ], 1 = singly occupied */
  const dlpno_pair* pairs;         /* [n_pairs] */
  const int64_t* cpl_rowptr;       /* [n_pairs + 1], CSR by target pair */
  const dlpno_coupling* cpl;       /* [n_couplings] */
  const double* f_a;               /* [n_occ * n_occ] alpha occupied Fock */
  const double* f_b;               /* [n_occ * n_occ] beta occupied Fock */
  int64_t n_B, n_T, n_K, n_eps, n_S; /* element counts of the buffers (bounds checks) */
  int64_t n_hh;                    /* hole-hole ladder couplings (0: no such term) */
  const int64_t* hh_rowptr;        /* [n_pairs + 1], CSR by target pair (may be NULL when n_hh = 0) */
  const dlpno_hh_coupling* hh;     /* [n_hh] */
  int64_t n_ring;                  /* ring/exchange couplings (0: no such term) */
  const int64_t* ring_rowptr;      /* [n_pairs + 1], CSR by target pair (may be NULL when n_ring = 0) */
  const dlpno_ring_coupling* ring; /* [n_ring] */
  int64_t n_ring_ints;             /* element count of dlpno_inputs.ring_ints */
} dlpno_problem;

/* Device inputs (caller-owned, read-only, fixed for the life of the plan). */
typedef struct {
  const double* B;
  const double* S;
  const double* K;
  const double* eps_a;
  const double* eps_b;
  const double* ring_ints;   /* integral blocks of the ring couplings (NULL when n_ring = 0) */
} dlpno_inputs;

typedef struct {
  dlpno_precision precision;
  int32_t diis_max;     /* vectors kept by DIIS, 0 = plain Jacobi, at most 8 */
  int32_t diis_start;   /* first extrapolation once this many are stored (>= 2) */
  int32_t n_workers;    /* persistent workgroups of the one-wave launches (0 = one per
                           compute unit); the two-wave launches use twice as many */
  int32_t items_per_wave; /* items per wavefront the schedule aims at: the work is
                           cut into about n_workers * 4 * items_per_wave items
                           (0 = default, 6; the autotuner may change it) */
  int32_t flags;        /* DLPNO_FLAG_* bits, 0 = defaults */
} dlpno_options;

/* Same-spin (AA, BB) amplitude blocks are antisymmetric in the two virtual
 * indices (Sec. II.A), and so are their ladder and projection contributions:
 * by default only the tiles on and below the diagonal of those contributions
 * are computed and the others are their negated transposes.  With this flag
 * every tile is computed, so the residual is the plain linear map also for
 * amplitudes that lack the antisymmetry.  Vector-Jacobian products always
 * compute every tile. */
#define DLPNO_FLAG_GENERAL_T 1

/* Adds the quadratic CCSD term 1/4 sum_KLCD <KL||CD> t_IJ^CD t_KL^AB over the
 * hole-hole couplings (so n_hh > 0 is required).  Reduced to
 * spin blocks it is the hole-hole ladder with the weights (k i | l j) +
 * c <K_(k,l), S_pq^T T_p S_pq>, c = 1/2 same spin and 1 opposite spin,
 * K_(k,l)[c][d] = (k c | l d) over the source pair's PNOs (its K block, or the
 * transpose for k > l): the integrals in the target's PNOs are taken as the
 * projection S_pq K_(k,l) S_pq^T.  The factors S_pq K_(k,l) S_pq^T are built
 * once by dlpno_plan_create; every residual evaluation of T first computes
 * the weights from T in FP64 (a separate kernel, phase 9 of
 * dlpno_phase_times), so the residual is quadratic in T.  In dlpno_solve_mixed
 * the FP64 refinement residuals compute them and the low-precision iterations
 * on the correction equation keep them.  The vector-Jacobian product refuses
 * such plans. */
#define DLPNO_FLAG_QUADRATIC 2

/* Adds the quadratic part of the occupied Fock intermediate of CCSD,
 * -P(IJ) sum_M t_IM^AB F_MJ with F_MJ = 1/2 sum_NEF t_JN^EF <MN||EF>.  Reduced to spin blocks, F^s_mj = sum over occupied n and its
 * spin of <G_(m,n), T^{s s_n}_(j,n)> with G[e][f] = (m e | n f) over the PNOs
 * of {j, n}, taken as the projection S K_(m,n) S^T of the exchange integrals
 * of {m, n} (transposed for m > n) through the listed occupied-Fock coupling
 * of {j, n} in which m replaces j, and K_(j,n) itself for m = j; the term
 * then dresses the occupied Fock weight of every listed projection term,
 * f^s_kj -> f^s_kj + F^s_kj, and adds -(F^s_ii + F^s'_jj) T to each block.
 * Sums run over the listed couplings only.  The factors S K S^T are built once
 * by dlpno_plan_create; every residual evaluation of T forms F from T first,
 * in FP64 (phase 9 of dlpno_phase_times).  In dlpno_solve_mixed the FP64
 * refinement residuals form it and the low-precision iterations on the
 * correction equation keep it.  The vector-Jacobian product refuses such
 * plans. */
#define DLPNO_FLAG_QUADRATIC_OCC 4

typedef struct dlpno_plan dlpno_plan;   /* opaque, owned by the library */

/* Validates the descriptors (ranges, offsets against the buffer sizes, the
 * block rule, CSR monotonicity and coupling consistency), builds the device
 * tables, the work schedule and the workspace.  Precision copies of B and S
 * are made here.  Synchronous.  opts may be NULL (FP64, DIIS 8/3). */
dlpno_status dlpno_plan_create(const dlpno_problem* prob, const dlpno_inputs* in,
                               const dlpno_options* opts, void* stream, dlpno_plan** out);
dlpno_status dlpno_plan_destroy(dlpno_plan* plan);

/* R = residual(T) for every stored block.  T, R: device, n_T doubles.  The
 * same-spin blocks of T must be antisymmetric unless the plan was created
 * with DLPNO_FLAG_GENERAL_T.  Asynchronous: a non-finite residual element is
 * reported by the next dlpno_iterate or dlpno_solve_mixed.  Every work item
 * of the schedule is checked against the compiled kernel bodies when the
 * plan is built (DLPNO_ERR_UNSUPPORTED there); should an item still reach a
 * kernel without a body, the device raises a flag that those calls report as
 * DLPNO_ERR_HIP. */
dlpno_status dlpno_residual(dlpno_plan* plan, const double* T, double* R, void* stream);

/* dlpno_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results (bitwise equal to dlpno_residual on the same
 * plan), with the partial-sum workspace taken from a static device array of
 * the library - 256 MiB (2^25 doubles) per GPU, held until the process ends -
 * instead of the plan's.  The call itself allocates nothing (no hipMalloc,
 * no events; phase timing is skipped).  The caller passes T and R (device,
 * n_T doubles) as for dlpno_residual.  A plan whose partial sums exceed the
 * array gets DLPNO_ERR_DIM_RANGE (fewer workers or items per wave make fewer
 * partial slots).  All calls on one GPU share the array: calls that overlap
 * in time there (other streams or threads) race.  Asynchronous. */
dlpno_status dlpno_residual_noalloc(dlpno_plan* plan, const double* T, double* R, void* stream);

/* T_out = T - R / D; e_pair[4 p + c] = energy of block c (0 AA, 1 BB, 2 AB,
 * 3 BA) of pair p computed with T_out (0 for absent blocks); *e_total = sum.
 * All device pointers; e_pair has 4 n_pairs doubles.  T_out may equal T. */
dlpno_status dlpno_update(dlpno_plan* plan, const double* T, const double* R, double* T_out,
                          double* e_pair, double* e_total, void* stream);

/* Second-order F12 correction with the (converged) amplitudes T (Sec. II.A:
 * Eq. "Vtilde" without its singles terms, and the spin-adapted pair energies
 * that follow Eq. "F12 energy").  For every stored block, in that block's
 * electron order:
 *   V~  = V  + 1/2 sum_ab W_ab T_ab      (direct geminal)
 *   V~x = V' + 1/2 sum_ab W_ba T_ab      (exchanged geminal)
 *   same spin:     eps = 1/2 V~ + 1/16 B1
 *   opposite spin: eps = 3/4 V~ + 1/4 V~x + 9/64 B1 + 3/64 B2 + 3/64 B3 + 1/64 B4
 * T, W: device, n_T doubles in the amplitude layout (W = V + C over the
 * pair's PNOs); scalars: device, 6 doubles per stored block in block order
 * (pairs in order, blocks AA, BB, AB, BA): V, V', B1, B2, B3, B4 (V' and
 * B2..B4 unused for same spin).  e_pair: 4 n_pairs doubles, by block code,
 * 0 for absent blocks; *e_total = their sum in a fixed order.  Device
 * pointers, caller-owned; asynchronous on stream.  NULL buffers with
 * nonzero sizes give DLPNO_ERR_INVALID_ARG. */
dlpno_status dlpno_f12_energy(dlpno_plan* plan, const double* T, const double* W, const double* scalars,
                              double* e_pair, double* e_total, void* stream);

/* n_iter iterations of: R = residual(T); T' = T - R/D; energies of T';
 * DIIS on (T', T' - T) (when enabled); T <- extrapolated T'.  One hipGraph per
 * iteration, replayed.  T is in/out; R, e_pair, e_total, max_abs_R receive
 * the last iteration's values (device).  Blocks until done and returns
 * DLPNO_ERR_NONFINITE if any residual element was not finite.  DIIS history
 * persists across calls until dlpno_reset.  When every element of T is zero
 * on entry, the first residual is the driver K^{ss'} alone (its ladder and
 * projection terms vanish exactly) and its grouped launches are skipped; the
 * same holds for the first refinement step of dlpno_solve_mixed. */
dlpno_status dlpno_iterate(dlpno_plan* plan, int32_t n_iter, double* T, double* R,
                           double* e_pair, double* e_total, double* max_abs_R, void* stream);

/* DIIS state after the last iteration (Pulay extrapolation of the amplitude
 * vectors T' with errors T' - T).  The bordered system
 *   [[G, -1], [-1, 0]] [c; -lambda] = [0; -1],  G_ab = <e_a, e_b> / max_k <e_k, e_k>,
 * is solved for the extrapolation coefficients; while its 2-norm condition
 * number exceeds 1e14 the oldest vector is dropped.  Outputs (host, any may be
 * NULL): *count = vectors kept, *drops = vectors dropped since the last reset,
 * coef[0..7] = coefficients oldest -> newest for the kept vectors (coef[count-1]
 * = 1 and the others 0 before extrapolation starts), zeros after them.
 * Waits for the work queued on `stream`. */
dlpno_status dlpno_diis_state(const dlpno_plan* plan, int32_t* count, int32_t* drops, double* coef, void* stream);

/* Iterates (as dlpno_iterate, checking every second iteration) until
 * max|R| < tol_r and the total energy changed by less than tol_e since the
 * previous iteration (DLPNO_OK), or at most max_iter iterations.  Returns
 * DLPNO_ERR_NOT_CONVERGED when max_iter is reached first, and as soon as max|R|
 * exceeds 1e3 times its smallest value of the call (the iteration diverges;
 * the buffers hold that iteration's values).  *n_done (host, may be NULL) =
 * iterations run.  Synchronous. */
dlpno_status dlpno_solve(dlpno_plan* plan, int32_t max_iter, double tol_r, double tol_e, double* T, double* R,
                         double* e_pair, double* e_total, double* max_abs_R, int32_t* n_done, void* stream);

/* Checkpoint of the iteration state, to resume an interrupted solve: the
 * amplitudes T (device, n_T doubles), the DIIS history (vectors, errors,
 * Gram matrix, coefficients) and the energy/max|R| history, copied to or from
 * caller-owned host memory of dlpno_checkpoint_size bytes.  A checkpoint
 * loads only into a plan with the same sizes and DIIS options; resuming gives
 * bitwise the iterations the saved plan would have run.  Synchronous. */
dlpno_status dlpno_checkpoint_size(const dlpno_plan* plan, size_t* bytes);
dlpno_status dlpno_checkpoint_save(const dlpno_plan* plan, const double* T, void* dst, void* stream);
dlpno_status dlpno_checkpoint_load(dlpno_plan* plan, double* T, const void* src, void* stream);

/* Clears the DIIS history and the iteration counter. */
dlpno_status dlpno_reset(dlpno_plan* plan, void* stream);

/* Per-iteration history of the last dlpno_iterate calls (host arrays of
 * length >= n): total energy and max |R|.  Returns the number written. */
int32_t dlpno_history(const dlpno_plan* plan, double* energy, double* max_abs_r, int32_t n);

/* Vector-Jacobian product of the residual: for Gbar = dL/dR,
 *   dT = D o Gbar + sum_Q (B^Q)^T Gbar B^Q + (projection terms)^T Gbar,
 *   dB^Q_p = sum_blocks (Gbar B^Q T^T + Gbar^T B^Q T)   (general, unsymmetrised B).
 * The projection transpose is evaluated by gathering over the couplings of
 * each source pair; this requires the data the physics guarantees: f^s
 * symmetric (to 1e-12 of its largest element), every coupling that carries a
 * term paired with a reverse coupling (q <- p) whose S block is the transpose
 * of (p <- q) (to 1e-12 relative).  The first call checks both (the overlap
 * blocks on the device; synchronous that once) and keeps the result; a plan
 * whose data violates them gets DLPNO_ERR_UNSUPPORTED from every call.
 * dT: n_T doubles; dB: n_B doubles (NULL skips it).  X^Q = B^Q T is recomputed
 * inside the kernel, never stored.  Asynchronous otherwise. */
dlpno_status dlpno_residual_vjp(dlpno_plan* plan, const double* T, const double* Gbar,
                                double* dT, double* dB, void* stream);

/* Mixed-precision solve (plan precision BF16X2, FP16X2 or FP32): n_outer
 * refinement steps, each computing the FP64 residual r = R(T) and then
 * n_inner low-precision Jacobi+DIIS iterations on the correction equation
 * (D + A) delta = -r, T += delta.  Unless the plan has DLPNO_FLAG_GENERAL_T,
 * the same-spin blocks of T are replaced by their antisymmetric part on entry
 * and after every step (removing the rounding of the low-precision
 * corrections).  T in/out (device).  Synchronous. */
dlpno_status dlpno_solve_mixed(dlpno_plan* plan, int32_t n_outer, int32_t n_inner, double* T,
                               double* R, double* e_pair, double* e_total, double* max_abs_R,
                               void* stream);

/* Algorithmic FLOPs of one residual evaluation (ladder: 4 m n^3 per block;
 * projection: 2 n_p n_q (n_p + n_q) per applied term, occupied-Fock and
 * hole-hole ladder terms alike). */
dlpno_status dlpno_flop_count(const dlpno_plan* plan, double* ladder, double* projection);

/* Time every variant of the grouped kernel's tile schedule on the plan's
 * workload and keep the fastest (T: a device amplitude buffer to run on,
 * R: scratch of n_T doubles).  Synchronous.  The choice is reported through
 * dlpno_plan_info. */
dlpno_status dlpno_autotune(dlpno_plan* plan, const double* T, double* R, void* stream);

/* dlpno_autotune with a persistent cache: when the JSON file `path` holds
 * choices for this device's architecture and the plan's precision, they are
 * applied without timing (*hit = 1); otherwise dlpno_autotune runs and its
 * choices are written to the file under that key, keeping its other entries
 * (*hit = 0).  The choices: the ladder and projection tile variants per tile
 * class of 16 PNOs, items per wave, the two-wave launches and the persistent
 * workgroup count.  Synchronous. */
dlpno_status dlpno_autotune_cached(dlpno_plan* plan, const double* T, double* R, const char* path, int32_t* hit,
                                   void* stream);

/* Kernel timing: when enabled, residual/iterate record HIP events around the
 * phases on the call's stream (graphs are bypassed) and dlpno_phase_times
 * returns the accumulated milliseconds and launch counts of:
 *   0 grouped kernel over the ladder items, 1 finish/update, 2 energy
 *   reduction, 3 DIIS, 4 precision conversion, 5 grouped kernel over the
 *   projection items, 6 grouped kernel over the ladder items run at two
 *   waves per SIMD (FP64 plans: pairs of at most 48 PNOs), 7 cooperative
 *   ladder launch (FP64 plans: pairs of 49 to 64 PNOs, one workgroup per
 *   item), 8 projection items run at two waves per SIMD (FP64 plans: target
 *   and source pairs of at most 48 PNOs), 9 weights of the quadratic terms
 *   (DLPNO_FLAG_QUADRATIC, DLPNO_FLAG_QUADRATIC_OCC), 10 ring/exchange term
 *   (n_ring > 0). */
dlpno_status dlpno_set_profiling(dlpno_plan* plan, int32_t enable);
/* Useful FP64 flops of the ring/exchange term per residual evaluation
 * (2 n_p n_q (n_q + n_p) per contraction S_{p,q} op(T_q) X) and the number
 * of such contractions; both 0 without ring couplings. */
dlpno_status dlpno_ring_flop_count(const dlpno_plan* plan, double* flops, int64_t* contractions);
dlpno_status dlpno_phase_times(const dlpno_plan* plan, double* ms, int64_t* launches, int32_t n);

/* ---- PNO construction (Sec. II.B.2) ----
 *
 * For every pair p, from the pair's first-order amplitude blocks X^{ss'}
 * (N_p x N_p each, in an orthonormal basis of the pair's domain of N_p
 * virtual functions) and the domain's virtual Fock matrix F_p:
 *   D_p = 1 / (2 (1 + delta_ij)) sum_{ss'} w_{ss'} (X X^T + X^T X),
 *         w = 1/2 for same spin, 1 for opposite spin (all four spin blocks;
 *         a diagonal pair's beta-alpha block, when not stored, is the
 *         transpose of its alpha-beta block).  With no SOMOs this is the
 *         closed-shell MP1 pair density, to which the paper's single set of
 *         PNOs per pair reduces;
 *   occupations = eigenvalues of D_p in descending order; the PNOs are the
 *         eigenvectors whose occupation is >= t_cut (T_CutPNO), n_p of them;
 *   semicanonical PNOs: the kept natural orbitals V_k rotated by the
 *         eigenvectors U of V_k^T F_p V_k, C_p = V_k U, orbital energies eps
 *         ascending; each column of C_p is signed so that its
 *         largest-magnitude element (the first on ties) is positive.
 * Domains of 1..64 functions.  Eigenproblems are solved by parallel cyclic
 * Jacobi in FP64. */
typedef struct {
  int32_t dim;       /* N_p, 1..64 */
  int32_t blocks;    /* stored amplitude blocks: bit 0 AA, 1 BB, 2 AB, 3 BA */
  int32_t diagonal;  /* 1 when the pair is (i, i), else 0 */
  int32_t first;     /* the domain is the window first .. first + dim - 1 of an orthonormal global
                      * virtual space (used by dlpno_pno_overlap), >= 0 */
  int64_t off_X;     /* first stored block; blocks back to back in the order AA, BB, AB, BA,
                      * each N_p x N_p row-major [a][b] */
  int64_t off_F;     /* N_p x N_p row-major, symmetric */
  int64_t off_C;     /* output, N_p x N_p row-major [domain function][PNO]: columns 0..n_p-1
                      * hold C_p, the others are zero */
  int64_t off_v;     /* outputs, N_p each: occupations (all N_p) and eps (first n_p, rest zero) */
} dlpno_pno_pair;

typedef struct dlpno_pno_plan dlpno_pno_plan;   /* opaque, owned by the library */

/* Validates the descriptors against the buffer sizes (in doubles) and
 * uploads them.  pairs: host array, read during the call.  Synchronous. */
dlpno_status dlpno_pno_plan_create(const dlpno_pno_pair* pairs, int64_t n_pairs, int64_t n_X, int64_t n_F,
                                   int64_t n_C, int64_t n_v, dlpno_pno_plan** out);

/* Builds the PNOs of every pair.  X, F: inputs; occ, eps (n_v doubles each),
 * C (n_C doubles), n_kept (n_pairs int32): outputs; sweeps: optional
 * (NULL or 2 n_pairs int32: Jacobi sweeps of the density and of the PNO Fock
 * matrix).  All device pointers, caller-owned.  n_kept[p] is n_p >= 0, or
 * -1 (density eigenproblem not converged in 40 sweeps), -2 (PNO Fock
 * eigenproblem not converged) or -3 (non-finite density); occupations, eps
 * and C of such a pair are zero.  Asynchronous on stream. */
dlpno_status dlpno_pno_build(dlpno_pno_plan* plan, const double* X, const double* F, double t_cut, double* occ,
                             double* eps, double* C, int32_t* n_kept, int32_t* sweeps, void* stream);
dlpno_status dlpno_pno_plan_destroy(dlpno_pno_plan* plan);

/* PNO overlaps for a coupling list (the S input of the residual): for every
 * coupling e of target pair p with source pair q = src[e] (CSR by target,
 * rowptr[p] .. rowptr[p+1]-1), the n_q x n_p block at off_S[e], element
 * [c][a] = sum over the global functions x shared by the two domain windows
 * of C_q[x - first_q][c] C_p[x - first_p][a] (zero when the windows do not
 * meet).  n_kept: the host copy of the n_kept that dlpno_pno_build returned
 * (every entry >= 0; a pair's PNO count is max(n_kept, 1), the extra column
 * of a pair that kept none being zero); rowptr, src, off_S: host arrays,
 * validated (CSR monotonic, sources in range, blocks inside n_S doubles)
 * and uploaded by _prepare, which is synchronous and replaces an earlier
 * list.  dlpno_pno_overlap: C as written by dlpno_pno_build, S (n_S
 * doubles): device pointers; asynchronous. */
dlpno_status dlpno_pno_overlap_prepare(dlpno_pno_plan* plan, const int32_t* n_kept, const int64_t* rowptr,
                                       const int32_t* src, const int64_t* off_S, int64_t n_S);
dlpno_status dlpno_pno_overlap(dlpno_pno_plan* plan, const double* C, double* S, void* stream);

/* Human-readable summary of the plan (schedule, variants, workspace). */
const char* dlpno_plan_info(const dlpno_plan* plan);

const char* dlpno_status_string(dlpno_status s);

/* Text of the last failure reported by any call on this thread ("" if none). */
const char* dlpno_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DLPNO_H */
