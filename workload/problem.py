"""Synthetic open-shell DLPNO pair workloads.

Data model (the paper's Sec. II.A high-spin spin cases and Sec. II.B.2/II.B.4
spin-independent PNO sets):
  * occupied orbitals 0..n_occ-1 on a 1-D chain; SOMOs are alpha-occupied and
    beta-virtual, so occ_alpha = all, occ_beta = DOMOs;
  * a retained pair p = (i, j), i <= j, owns n_p PNOs shared by every spin block
    and m_p local density-fitting functions;
  * a spin block s s' (first spin on electron i / virtual a, second on j / b) is
    stored iff i in occ_s, j in occ_s', not (s == s' and i == j), and for i == j
    only the alpha-beta block is kept (beta-alpha is its transpose);
  * stored blocks of a pair are contiguous in the order AA, BB, AB, BA.

Flat layouts (element offsets, 32-element aligned):
  B  : per pair [Q][a][c], m_p x n_p x n_p, symmetric in (a, c)
  T/R: per pair, stored blocks back to back, each n_p x n_p row-major [a][b]
  K  : per pair n_p x n_p, the spatial exchange integrals (i a | j b)
  eps: per pair n_p virtual energies per spin (eps_a / eps_b arrays)
  S  : per directed coupling (target p <- source q): n_q x n_p row-major,
       element [c][a] = overlap of source PNO c with target PNO a
  f_a, f_b: n_occ x n_occ occupied Fock matrices per spin

Couplings (CSR by target pair): target p = (i, j) reads source q when an
occupied k replaces i (side 0, q = {k, j}, Fock weight f[k][i]) or replaces j
(side 1, q = {i, k}, weight f[k][j]); only retained sources with a non-zero
occupied Fock element are listed.
"""
from dataclasses import dataclass, field
import numpy as np

from . import philox

BLOCK_NAMES = ("AA", "BB", "AB", "BA")
BLOCK_BITS = {"AA": 1, "BB": 2, "AB": 4, "BA": 8}
BLOCK_SPINS = {"AA": (0, 0), "BB": (1, 1), "AB": (0, 1), "BA": (1, 0)}

# Philox field ids (fourth counter word)
F_NPNO, F_NAUX, F_B, F_T, F_K, F_EPS, F_FDIAG, F_FOFF, F_S, F_QR, F_W, F_F12, F_FOFFB, F_HH = range(1, 15)
# PNO-construction inputs (workload.pno)
F_DOM, F_TAU, F_PX, F_PF = range(15, 19)
# ring/exchange-term integrals (stream 2 e for X, 2 e + 1 for J of ring coupling e)
F_RING = 19

# F12 inputs (synthetic): W = V + C per stored block, in the amplitude layout,
# and six scalars per block (V, V', B1..B4, see Problem.f12_scalars)
SIGMA_W = 0.05

# segment generation modes (see segment_values)
MODE_PLAIN, MODE_SYM, MODE_ANTI, MODE_TRANS, MODE_EYE, MODE_DECAY, MODE_FOCK = 0, 1, 2, 3, 4, 5, 6
MODE_AUG_PLAIN, MODE_AUG_TRANS = 7, 8

SEG_DTYPE = np.dtype([("off", np.int64), ("stream", np.int64), ("field", np.int32),
                      ("mode", np.int32), ("layers", np.int32), ("rows", np.int32),
                      ("cols", np.int32), ("pad", np.int32), ("scale", np.float64)])

ALIGN = 32

# name -> recipe.  Sizes and distributions follow the workload shapes of the
# paper's tests (a small radical, a 1-D chain, a C160H322-like triplet alkane).
CONFIGS = {
    # 16 doubly + 2 singly occupied, all 171 pairs, n=12, m=80
    "tiny": dict(n_occ=18, somos=(16, 17), band=None, npno=("fixed", 12),
                 naux=("fixed", 80), sigma_B=0.05, S="qr60", seed=1, kappa=0.01,
                 sigma_T=1e-2),
    # 160 occupied (2 SOMOs), |i-j| <= 20, n ~ lognormal(mean 28), m ~ U{300..900}
    "chain": dict(n_occ=160, somos=(53, 106), band=20, npno=("lognormal", 28.0, 0.4, 8, 64),
                  naux=("uniform", 300, 900), sigma_B="scaled", S="random", seed=2,
                  kappa=0.01, sigma_T=1e-2),
    # C160H322-shaped: 481 occupied (2 SOMOs), |i-j| <= 40, n ~ lognormal(mean 30), m ~ U{400..1200}
    # kappa sets the driver scale so that the converged correlation energy of this
    # model is about the CCSD energy the paper reports for C160H322 (-28.78 Eh)
    "c160": dict(n_occ=481, somos=(160, 320), band=40, npno=("lognormal", 30.0, 0.4, 8, 64),
                 naux=("uniform", 400, 1200), sigma_B="scaled", S="random", seed=3,
                 kappa=0.015451, sigma_T=1e-2),
}


def _align(x):
    return (x + ALIGN - 1) // ALIGN * ALIGN


def stored_blocks(i, j, is_somo):
    """Names of the stored spin blocks of pair (i, j), i <= j, in storage order."""
    occ = (lambda k: True, lambda k: not is_somo[k])  # alpha, beta occupation
    out = []
    for name in BLOCK_NAMES:
        s1, s2 = BLOCK_SPINS[name]
        if not (occ[s1](i) and occ[s2](j)):
            continue
        if s1 == s2 and i == j:
            continue
        if i == j and name == "BA":
            continue
        out.append(name)
    return out


@dataclass
class Problem:
    name: str
    seed: int
    n_occ: int
    is_somo: np.ndarray            # uint8 [n_occ]
    pi: np.ndarray                 # int32 [P]
    pj: np.ndarray
    npno: np.ndarray
    naux: np.ndarray
    blocks: np.ndarray             # uint32 [P] mask
    off_B: np.ndarray              # int64 [P]
    off_T: np.ndarray
    off_K: np.ndarray
    off_eps: np.ndarray
    cpl_rowptr: np.ndarray         # int64 [P+1]
    cpl_src: np.ndarray            # int32 [C]
    cpl_k: np.ndarray
    cpl_side: np.ndarray
    cpl_off_S: np.ndarray          # int64 [C]
    f_a: np.ndarray
    f_b: np.ndarray
    eps_a: np.ndarray
    eps_b: np.ndarray
    n_B: int
    n_T: int
    n_K: int
    n_S: int
    segs: dict = field(default_factory=dict)   # name -> SEG_DTYPE array
    S_host: np.ndarray = None                  # set when S is built on the host (QR recipe)
    pair_index: dict = field(default_factory=dict)
    # hole-hole ladder couplings (CSR by target pair; empty when the term is off):
    # ordered occupied source (k, l), source pair {k, l}, weight (k i | l j), overlap block
    hh_rowptr: np.ndarray = None
    hh_src: np.ndarray = None
    hh_k: np.ndarray = None
    hh_l: np.ndarray = None
    hh_w: np.ndarray = None
    hh_off_S: np.ndarray = None
    hole_scale: float = 0.0
    hole_range: int = 2
    # SOMO virtual functions appended to every pair's PNOs (None: none)
    n_sv: np.ndarray = None
    # the quadratic CCSD term over the hole-hole couplings (needs hole_ladder)
    quadratic: bool = False
    # the quadratic part of the occupied Fock intermediate on the Fock couplings
    quadratic_occ: bool = False
    # ring/exchange-term couplings (CSR by target pair; empty when the term is
    # off): role (0: the target's i is shared, 1: its j), replacing occupied m,
    # source pair {x, m}, overlap block, and the integral blocks X = (m e|b y),
    # J = (m y|b e) (n_src x n_target, [e][b]) in the ring buffer of n_Rg
    ring_rowptr: np.ndarray = None
    ring_src: np.ndarray = None
    ring_role: np.ndarray = None
    ring_m: np.ndarray = None
    ring_off_S: np.ndarray = None
    ring_off_X: np.ndarray = None
    ring_off_J: np.ndarray = None
    n_Rg: int = 0
    ring_scale: float = 0.0
    ring_range: int = 2

    def t_mask(self):
        """Flat boolean array over the amplitude layout: True inside the
        virtual spaces of each block's spins (everything, without SOMO
        virtual functions)."""
        mask = np.ones(self.n_T, dtype=bool)
        if self.n_sv is None:
            return mask
        for p in range(self.n_pairs):
            n, ns, o = int(self.npno[p]), int(self.n_sv[p]), int(self.off_T[p])
            for name in BLOCK_NAMES:
                if not self.blocks[p] & BLOCK_BITS[name]:
                    continue
                s1, s2 = BLOCK_SPINS[name]
                m = np.ones((n, n), dtype=bool)
                if s1 == 0 and ns:
                    m[n - ns:, :] = False
                if s2 == 0 and ns:
                    m[:, n - ns:] = False
                mask[o:o + n * n] = m.ravel()
                o += n * n
        return mask

    @property
    def n_hh(self):
        return 0 if self.hh_src is None else len(self.hh_src)

    @property
    def n_ring(self):
        return 0 if self.ring_src is None else len(self.ring_src)

    def ring_matrix(self, e, which):
        """X (which = 0) or J (which = 1) of ring coupling e, n_src x n_target."""
        seg = self.segs["Rg"][2 * e + which]
        return segment_values(self.seed, seg).reshape(seg["rows"], seg["cols"])

    def eri_occ(self, k, i, l, j):
        """The synthetic occupied integral (k i | l j) of this workload (0 when
        the hole-hole term is off)."""
        if self.hole_scale == 0.0:
            return 0.0
        return float(occ_eri(self.seed, self.n_occ, self.hole_scale, self.hole_range, [k], [i], [l], [j])[0])

    @property
    def n_pairs(self):
        return len(self.pi)

    @property
    def n_couplings(self):
        return len(self.cpl_src)

    def n_blocks(self):
        return np.array([bin(int(b)).count("1") for b in self.blocks])

    def block_list(self, p):
        return [n for n in BLOCK_NAMES if self.blocks[p] & BLOCK_BITS[n]]

    # ---------------- materialisation of the large fields ----------------
    def materialize(self, what):
        """Full flat array of 'B', 'T', 'K', 'S', 'W' or 'Rg' (host memory; small problems)."""
        size = {"B": self.n_B, "T": self.n_T, "K": self.n_K, "S": self.n_S, "W": self.n_T, "Rg": self.n_Rg}[what]
        if what == "S" and self.S_host is not None:
            return self.S_host.copy()
        out = np.zeros(size, dtype=np.float64)
        for seg in self.segs[what]:
            v = segment_values(self.seed, seg)
            out[seg["off"]:seg["off"] + v.size] = v.ravel()
        return out

    def pair_B(self, p):
        """B_p as an (m, n, n) array regenerated from its counters."""
        seg = self.segs["B"][p]
        return segment_values(self.seed, seg).reshape(seg["layers"], seg["rows"], seg["cols"])

    def f12_scalars(self):
        """Six synthetic F12 scalars per stored block, in block order (pairs in
        order, blocks AA, BB, AB, BA within a pair): the geminal diagonal
        V (negative, about -0.02), its exchange counterpart V' (opposite spin),
        and four B-tilde values (positive, about 0.02).  float64 [n_blocks, 6]."""
        nb = int(self.n_blocks().sum())
        idx = (np.arange(nb, dtype=np.uint64)[:, None] * np.uint64(8) + np.arange(6, dtype=np.uint64)[None, :])
        z = philox.normals(self.seed, F_F12, 0, idx)
        out = np.empty((nb, 6))
        out[:, 0] = -0.02 * (1.0 + 0.25 * z[:, 0])
        out[:, 1] = 0.005 * z[:, 1]
        out[:, 2:] = 0.02 * (1.0 + 0.25 * z[:, 2:])
        return out

    def segment(self, what, idx):
        seg = self.segs[what][idx]
        return segment_values(self.seed, seg).reshape(seg["layers"], seg["rows"], seg["cols"])


def segment_values(seed, seg):
    """Values of one generated segment: layers x rows x cols (rows, cols <= 64)."""
    L, R, C = int(seg["layers"]), int(seg["rows"]), int(seg["cols"])
    mode, fld, stream, scale = int(seg["mode"]), int(seg["field"]), int(seg["stream"]), float(seg["scale"])
    lay = np.arange(L, dtype=np.uint64)[:, None, None] * np.uint64(4096)
    x = np.arange(R, dtype=np.uint64)[None, :, None]
    y = np.arange(C, dtype=np.uint64)[None, None, :]
    if mode == MODE_PLAIN:
        idx = lay + x * np.uint64(64) + y
    elif mode == MODE_TRANS:
        idx = lay + y * np.uint64(64) + x
    elif mode == MODE_SYM:
        idx = lay + np.minimum(x, y) * np.uint64(64) + np.maximum(x, y)
    elif mode == MODE_DECAY:
        # plain normals times 2^-floor((x + y) / pad): a staircase decay of
        # exact powers of two (bit-identical on both generators)
        z = philox.normals(seed, fld, stream, lay + x * np.uint64(64) + y)
        tau = int(seg["pad"])
        e = -((x.astype(np.int64) + y.astype(np.int64)) // tau)
        return z * np.ldexp(1.0, e) * scale
    elif mode == MODE_FOCK:
        # symmetric normals times scale off the diagonal, 0.2 + 2.8 u on it
        # (u: the first Philox word of the diagonal element's counter / 2^32)
        idx = lay + np.minimum(x, y) * np.uint64(64) + np.maximum(x, y)
        z = philox.normals(seed, fld, stream, idx) * scale
        u = philox.uniforms(seed, fld, stream, idx)
        return np.where(x == y, 0.2 + 2.8 * u, z) + np.zeros((L, 1, 1))
    elif mode in (MODE_AUG_PLAIN, MODE_AUG_TRANS):
        # overlap block of two SOMO-augmented PNO sets: the PNO part as
        # MODE_PLAIN / MODE_TRANS, the last pad rows and columns the identity
        ns = int(seg["pad"])
        idx = lay + (x * np.uint64(64) + y if mode == MODE_AUG_PLAIN else y * np.uint64(64) + x)
        z = philox.normals(seed, fld, stream, idx) * scale
        xs, ys = x.astype(np.int64) - (R - ns), y.astype(np.int64) - (C - ns)
        return np.where((xs < 0) & (ys < 0), z, np.where((xs >= 0) & (xs == ys), 1.0, 0.0)) + np.zeros((L, 1, 1))
    elif mode == MODE_EYE:
        # identity blocks (the overlap of a pair's PNOs with themselves)
        return np.broadcast_to((x == y).astype(np.float64), (L, R, C)).copy()
    elif mode == MODE_ANTI:
        z1 = philox.normals(seed, fld, stream, lay + x * np.uint64(64) + y)
        z2 = philox.normals(seed, fld, stream, lay + y * np.uint64(64) + x)
        return (z1 - z2) * scale
    else:
        raise ValueError(mode)
    return philox.normals(seed, fld, stream, idx) * scale


def _dims(rule, seed, fld, P):
    kind = rule[0]
    if kind == "fixed":
        return np.full(P, rule[1], dtype=np.int32)
    if kind == "given":          # one value per pair, e.g. PNO counts from a PNO build
        v = np.asarray(rule[1], dtype=np.int32)
        if v.shape != (P,):
            raise ValueError("given dimensions: %d values for %d pairs" % (v.size, P))
        return v.copy()
    streams = np.arange(P, dtype=np.uint64)
    if kind == "uniform":
        lo, hi = rule[1], rule[2]
        u = philox.uniforms(seed, fld, streams, 0)
        return (lo + np.floor(u * (hi - lo + 1))).astype(np.int32)
    if kind == "lognormal":
        mean, s, lo, hi = rule[1:]
        u1 = philox.uniforms(seed, fld, streams, 0)
        u2 = philox.uniforms(seed, fld, streams, 1)
        z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)   # Box-Muller
        mu = np.log(mean) - 0.5 * s * s                                 # arithmetic mean = `mean`
        return np.clip(np.rint(np.exp(mu + s * z)), lo, hi).astype(np.int32)
    raise ValueError(kind)


def occ_eri(seed, n_occ, scale, rng, k, i, l, j):
    """Synthetic occupied four-index integrals (k i | l j) (chemists' notation)
    for arrays of indices: scale exp(-(|k - i| + |l - j|)) z with one normal z
    per orbit of the eightfold permutational symmetry of real integrals
    ((ki|lj) = (ik|lj) = (ki|jl) = (lj|ki) ...), zero unless |k - i| <= rng
    and |l - j| <= rng.  A random draw of the inputs, not a computed integral."""
    k, i, l, j = (np.asarray(x, dtype=np.int64) for x in (k, i, l, j))
    a, b = np.minimum(k, i), np.maximum(k, i)
    c, d = np.minimum(l, j), np.maximum(l, j)
    swap = (a > c) | ((a == c) & (b > d))
    a2, b2 = np.where(swap, c, a), np.where(swap, d, b)
    c2, d2 = np.where(swap, a, c), np.where(swap, b, d)
    n = np.int64(n_occ)
    idx = (((a2 * n + b2) * n + c2) * n + d2).astype(np.uint64)
    z = philox.normals(seed, F_HH, 0, idx)
    dk, dl = np.abs(k - i), np.abs(l - j)
    v = scale * np.exp(-(dk + dl).astype(np.float64)) * z
    return np.where((dk <= rng) & (dl <= rng), v, 0.0)


def build_problem(name="tiny", **override):
    """Build the descriptors and small inputs of a named (or customised) workload.

    Overrides: any CONFIGS key, e.g. n_occ=24, band=6, somos=(8, 16), and
    fock_spin=x: beta off-diagonal occupied Fock elements f_b[i,k] = f_a[i,k] +
    x 0.02 exp(-|i-k|/3) z' with z' from a field of their own (default 0: the
    off-diagonal elements are the same for both spins);
    hole_ladder=c, hole_range=d: the hole-hole ladder's occupied integrals
    (k i | l j) drawn by occ_eri with scale c and range d (default 0: no
    hole-hole term), with one coupling per target pair (i, j) and ordered
    occupied pair (k, l) whose integral is non-zero and whose pair {k, l} is
    retained (the pair itself included: its overlap block is the identity);
    quadratic=True (with hole_ladder): the quadratic CCSD term over the
    hole-hole couplings is part of the residual (Problem.quadratic);
    quadratic_occ=True: the quadratic part of the occupied Fock intermediate,
    over the occupied-Fock couplings, is part of the residual
    (Problem.quadratic_occ; no further inputs);
    ring=c, ring_range=d: the ring/exchange term, with one coupling per target
    pair (i, j), role (x = i, y = j or, for i < j, x = j, y = i) and occupied
    m with |m - x| <= d whose pair {x, m} is retained (the pair itself
    included when m = y: identity overlap); its integral blocks X and J are
    normals times c exp(-(|m - x| + |m - y|) / 2) / sqrt(n_target) (default
    c = 0: no ring term);
    somo_virt=True: every pair's PNOs are followed by the SOMOs as virtual
    functions for beta electrons (Sec. II.B.4): n_p = min(n_p, 64 - N_SOMO) +
    N_SOMO, B and K cover all of them, the SOMO part of every overlap block
    is the identity, the SOMOs' beta virtual energies are 0.1 + 0.2 u (the
    alpha entries there are the same numbers and never used), and
    Problem.t_mask() gives the amplitude elements that exist."""
    cfg = dict(CONFIGS[name]) if name in CONFIGS else {}
    cfg.update(override)
    seed = int(cfg["seed"])
    n_occ = int(cfg["n_occ"])
    is_somo = np.zeros(n_occ, dtype=np.uint8)
    for s in cfg["somos"]:
        is_somo[s] = 1
    band = cfg["band"]
    band = n_occ if band is None else int(band)

    # ---- retained pairs, chain order (i ascending, then j) ----
    ii, jj = [], []
    for i in range(n_occ):
        for j in range(i, min(n_occ, i + band + 1)):
            ii.append(i)
            jj.append(j)
    pi = np.array(ii, dtype=np.int32)
    pj = np.array(jj, dtype=np.int32)
    P = len(pi)
    pair_index = {(int(a), int(b)): p for p, (a, b) in enumerate(zip(pi, pj))}

    npno = _dims(cfg["npno"], seed, F_NPNO, P)
    naux = _dims(cfg["naux"], seed, F_NAUX, P)
    n_sv = None
    if cfg.get("somo_virt", False):
        ns = len(cfg["somos"])
        npno = (np.minimum(npno, 64 - ns) + ns).astype(np.int32)
        n_sv = np.full(P, ns, dtype=np.int32)

    blocks = np.zeros(P, dtype=np.uint32)
    nblk = np.zeros(P, dtype=np.int64)
    for p in range(P):
        names = stored_blocks(int(pi[p]), int(pj[p]), is_somo)
        blocks[p] = sum(BLOCK_BITS[n] for n in names)
        nblk[p] = len(names)

    n2 = npno.astype(np.int64) ** 2
    szB = np.array([_align(int(a) * int(b)) for a, b in zip(naux, n2)], dtype=np.int64)
    szT = np.array([_align(int(k) * int(b)) for k, b in zip(nblk, n2)], dtype=np.int64)
    szK = np.array([_align(int(b)) for b in n2], dtype=np.int64)
    szE = np.array([_align(int(n)) for n in npno], dtype=np.int64)
    off_B = np.concatenate([[0], np.cumsum(szB)[:-1]]).astype(np.int64)
    off_T = np.concatenate([[0], np.cumsum(szT)[:-1]]).astype(np.int64)
    off_K = np.concatenate([[0], np.cumsum(szK)[:-1]]).astype(np.int64)
    off_eps = np.concatenate([[0], np.cumsum(szE)[:-1]]).astype(np.int64)
    n_B, n_T, n_K, n_E = int(szB.sum()), int(szT.sum()), int(szK.sum()), int(szE.sum())

    # ---- occupied Fock: diagonal U[-1.2,-0.3]; off-diagonal for retained (i,k) ----
    somos = [int(s) for s in cfg["somos"]]
    occ_idx = np.arange(n_occ)
    fdiag = -1.2 + 0.9 * philox.uniforms(seed, F_FDIAG, 0, np.arange(n_occ, dtype=np.uint64))
    f_a = np.diag(fdiag)
    for d in range(1, min(band, n_occ - 1) + 1):
        i = np.arange(n_occ - d)
        z = philox.normals(seed, F_FOFF, d, i.astype(np.uint64))
        v = 0.02 * np.exp(-d / 3.0) * z
        f_a[i, i + d] = v
        f_a[i + d, i] = v
    f_b = f_a.copy()
    # optional spin dependence of the off-diagonal occupied Fock elements: the
    # beta elements get an independent draw of relative size fock_spin on the
    # same support (so the coupling list is unchanged)
    fock_spin = float(cfg.get("fock_spin", 0.0))
    if fock_spin != 0.0:
        for d in range(1, min(band, n_occ - 1) + 1):
            i = np.arange(n_occ - d)
            z = philox.normals(seed, F_FOFFB, d, i.astype(np.uint64))
            v = fock_spin * 0.02 * np.exp(-d / 3.0) * z
            f_b[i, i + d] += v
            f_b[i + d, i] += v
    pol_occ = np.zeros(n_occ)
    for s in somos:
        pol_occ += 0.05 * np.exp(-np.abs(occ_idx - s) / 2.0)
    f_b[occ_idx, occ_idx] += pol_occ

    # ---- virtual energies per pair and spin ----
    eps_a = np.zeros(n_E)
    eps_b = np.zeros(n_E)
    for p in range(P):
        n = int(npno[p])
        u = philox.uniforms(seed, F_EPS, p, np.arange(n, dtype=np.uint64))
        ea = 0.2 + 2.8 * u
        d = np.minimum(np.abs(pi[p] - np.array(somos)), np.abs(pj[p] - np.array(somos))) if somos else np.zeros(0)
        shift = float(np.sum(0.05 * np.exp(-d / 2.0)))
        eb = ea + shift
        if n_sv is not None and n_sv[p]:
            ns = int(n_sv[p])
            ea[n - ns:] = 0.1 + 0.2 * u[n - ns:]
            eb[n - ns:] = ea[n - ns:]
        eps_a[off_eps[p]:off_eps[p] + n] = ea
        eps_b[off_eps[p]:off_eps[p] + n] = eb

    # ---- couplings (CSR by target) ----
    src, kk, side = [], [], []
    rowptr = np.zeros(P + 1, dtype=np.int64)
    for p in range(P):
        i, j = int(pi[p]), int(pj[p])
        for sd, (rep, keep) in enumerate(((i, j), (j, i))):
            for k in range(max(0, rep - band), min(n_occ, rep + band + 1)):
                if k == rep or f_a[k, rep] == 0.0:
                    continue
                q = pair_index.get((min(k, keep), max(k, keep)))
                if q is None:
                    continue
                src.append(q)
                kk.append(k)
                side.append(sd)
        rowptr[p + 1] = len(src)
    cpl_src = np.array(src, dtype=np.int32)
    cpl_k = np.array(kk, dtype=np.int32)
    cpl_side = np.array(side, dtype=np.int32)
    C = len(cpl_src)
    tgt = np.repeat(np.arange(P, dtype=np.int64), np.diff(rowptr))

    # ---- hole-hole ladder couplings (CSR by target): ordered (k, l) near (i, j) ----
    hh_scale = float(cfg.get("hole_ladder", 0.0))
    hh_range = int(cfg.get("hole_range", 2))
    hh_rowptr = np.zeros(P + 1, dtype=np.int64)
    hh_src = np.zeros(0, dtype=np.int32)
    hh_k = np.zeros(0, dtype=np.int32)
    hh_l = np.zeros(0, dtype=np.int32)
    hh_w = np.zeros(0)
    if hh_scale != 0.0:
        offs = np.arange(-hh_range, hh_range + 1)
        dk = np.repeat(offs, len(offs))
        dl = np.tile(offs, len(offs))
        pp = np.repeat(np.arange(P, dtype=np.int64), len(dk))
        ci, cj = pi[pp].astype(np.int64), pj[pp].astype(np.int64)
        ck, cl = ci + np.tile(dk, P), cj + np.tile(dl, P)
        ok = (ck >= 0) & (ck < n_occ) & (cl >= 0) & (cl < n_occ)
        pp, ci, cj, ck, cl = pp[ok], ci[ok], cj[ok], ck[ok], cl[ok]
        w = occ_eri(seed, n_occ, hh_scale, hh_range, ck, ci, cl, cj)
        pidx = np.full((n_occ, n_occ), -1, dtype=np.int64)
        pidx[pi, pj] = np.arange(P)
        q = pidx[np.minimum(ck, cl), np.maximum(ck, cl)]
        ok = (w != 0.0) & (q >= 0)
        pp, ck, cl, q, w = pp[ok], ck[ok], cl[ok], q[ok], w[ok]
        hh_rowptr[1:] = np.cumsum(np.bincount(pp, minlength=P))
        hh_src, hh_k, hh_l, hh_w = q.astype(np.int32), ck.astype(np.int32), cl.astype(np.int32), w
    hh_tgt = np.repeat(np.arange(P, dtype=np.int64), np.diff(hh_rowptr))

    # ---- ring/exchange-term couplings (CSR by target): (role, m) near x ----
    ring_scale = float(cfg.get("ring", 0.0))
    ring_range = int(cfg.get("ring_range", 2))
    ring_rowptr = np.zeros(P + 1, dtype=np.int64)
    r_src, r_role, r_m = [], [], []
    if ring_scale != 0.0:
        for p in range(P):
            i, j = int(pi[p]), int(pj[p])
            for role, x in enumerate((i, j)):
                if role == 1 and i == j:
                    continue
                for m in range(max(0, x - ring_range), min(n_occ, x + ring_range + 1)):
                    q = pair_index.get((min(x, m), max(x, m)))
                    if q is None:
                        continue
                    r_src.append(q)
                    r_role.append(role)
                    r_m.append(m)
            ring_rowptr[p + 1] = len(r_src)
    ring_src = np.array(r_src, dtype=np.int32)
    ring_role = np.array(r_role, dtype=np.int32)
    ring_m = np.array(r_m, dtype=np.int32)
    ring_tgt = np.repeat(np.arange(P, dtype=np.int64), np.diff(ring_rowptr))

    # one S block per (target, source) pair of pairs, shared by every coupling
    # (Fock or hole-hole) between them; the two sides of a diagonal target that
    # reach the same source share it
    key = np.concatenate([tgt * P + cpl_src, hh_tgt * P + hh_src.astype(np.int64),
                          ring_tgt * P + ring_src.astype(np.int64)])
    ukey, first, inv = np.unique(key, return_index=True, return_inverse=True)
    sz_dir = np.array([_align(int(npno[int(k // P)]) * int(npno[int(k % P)])) for k in ukey], dtype=np.int64)
    off_dir = np.concatenate([[0], np.cumsum(sz_dir)[:-1]]).astype(np.int64)
    H = len(hh_src)
    cpl_off_S = off_dir[inv[:C]]
    hh_off_S = off_dir[inv[C:C + H]]
    ring_off_S = off_dir[inv[C + H:]].astype(np.int64)
    n_S = int(sz_dir.sum())

    # ---- generated segments ----
    sigma_B = cfg["sigma_B"]
    if sigma_B == "scaled":
        sB = np.sqrt(1.0 / (naux.astype(np.float64) * (npno.astype(np.float64) + 1.0)))
    else:
        sB = np.full(P, float(sigma_B))
    segB = np.zeros(P, dtype=SEG_DTYPE)
    segB["off"], segB["stream"], segB["field"], segB["mode"] = off_B, np.arange(P), F_B, MODE_SYM
    segB["layers"], segB["rows"], segB["cols"], segB["scale"] = naux, npno, npno, sB

    kappa = float(cfg["kappa"])
    segK = np.zeros(P, dtype=SEG_DTYPE)
    segK["off"], segK["stream"], segK["field"] = off_K, np.arange(P), F_K
    segK["mode"] = np.where(pi == pj, MODE_SYM, MODE_PLAIN)
    segK["layers"], segK["rows"], segK["cols"] = 1, npno, npno
    segK["scale"] = kappa * (1.0 + np.abs(pi - pj).astype(np.float64)) ** -3

    sT = float(cfg["sigma_T"])
    tl = []
    for p in range(P):
        o = int(off_T[p])
        for name in BLOCK_NAMES:
            if not blocks[p] & BLOCK_BITS[name]:
                continue
            same = name in ("AA", "BB")
            tl.append((o, p * 4 + BLOCK_NAMES.index(name), F_T, MODE_ANTI if same else MODE_PLAIN,
                       1, int(npno[p]), int(npno[p]), 0, sT / np.sqrt(2.0) if same else sT))
            o += int(npno[p]) ** 2
    segT = np.array(tl, dtype=SEG_DTYPE)
    # F12 input W = V + C: general (no symmetry), same layout as the amplitudes
    segW = segT.copy()
    segW["field"], segW["mode"], segW["scale"] = F_W, MODE_PLAIN, SIGMA_W

    segs = {"B": segB, "K": segK, "T": segT, "W": segW}

    # ring integral blocks: X then J per coupling, n_src x n_target each
    NR = len(ring_src)
    r_rows = npno[ring_src].astype(np.int64) if NR else np.zeros(0, dtype=np.int64)
    r_cols = npno[ring_tgt].astype(np.int64) if NR else np.zeros(0, dtype=np.int64)
    r_sz = np.repeat(np.array([_align(int(a) * int(b)) for a, b in zip(r_rows, r_cols)], dtype=np.int64), 2)
    r_off = np.concatenate([[0], np.cumsum(r_sz)[:-1]]).astype(np.int64) if NR else np.zeros(0, dtype=np.int64)
    n_Rg = int(r_sz.sum())
    segR = np.zeros(2 * NR, dtype=SEG_DTYPE)
    if NR:
        x_r = np.where(ring_role == 0, pi[ring_tgt], pj[ring_tgt]).astype(np.int64)
        y_r = np.where(ring_role == 0, pj[ring_tgt], pi[ring_tgt]).astype(np.int64)
        dec = ring_scale * np.exp(-(np.abs(ring_m - x_r) + np.abs(ring_m - y_r)) / 2.0) / np.sqrt(r_cols)
        segR["off"] = r_off
        segR["stream"] = np.arange(2 * NR)
        segR["field"] = F_RING
        segR["mode"] = MODE_PLAIN
        segR["layers"] = 1
        segR["rows"] = np.repeat(r_rows, 2)
        segR["cols"] = np.repeat(r_cols, 2)
        segR["scale"] = np.repeat(dec, 2)
    segs["Rg"] = segR
    S_host = None
    if cfg["S"] == "qr60":
        # orthonormal PNO bases over a shared 60-dimensional virtual space
        Qs = []
        nsv = np.zeros(P, dtype=np.int64) if n_sv is None else n_sv
        for p in range(P):
            n = int(npno[p] - nsv[p])
            G = philox.normals(seed, F_QR, p, (np.arange(60)[:, None] * 64 + np.arange(n)[None, :]).astype(np.uint64))
            Qm, Rm = np.linalg.qr(G)
            Qs.append(Qm * np.sign(np.diag(Rm))[None, :])
        S_host = np.zeros(n_S)
        for u, k in enumerate(ukey):
            p, q = int(k // P), int(k % P)
            W = np.eye(int(npno[p])) if p == q else Qs[q].T @ Qs[p]     # [c][a] = <c_q | a_p>
            if p != q and nsv[p]:        # SOMO functions: identity block
                Wa = np.zeros((int(npno[q]), int(npno[p])))
                Wa[:W.shape[0], :W.shape[1]] = W
                Wa[W.shape[0]:, W.shape[1]:] = np.eye(int(nsv[p]))
                W = Wa
            S_host[off_dir[u]:off_dir[u] + W.size] = W.ravel()
    else:
        # random overlaps: S_{lo,hi} = sigma * Z (n_lo x n_hi), S_{hi,lo} = its transpose
        lo = np.minimum(ukey // P, ukey % P)
        hi = np.maximum(ukey // P, ukey % P)
        und, und_inv = np.unique(lo * P + hi, return_inverse=True)
        segS = np.zeros(len(ukey), dtype=SEG_DTYPE)
        p_t, q_s = ukey // P, ukey % P
        segS["off"] = off_dir
        segS["stream"] = und_inv
        segS["field"] = F_S
        # stored W[c][a] (c on source q, a on target p) = S_{q,p}[c][a]:
        #   q == lo: Z[c][a] (plain); q == hi: Z[a][c] (transposed)
        segS["mode"] = np.where(q_s == p_t, MODE_EYE, np.where(q_s < p_t, MODE_PLAIN, MODE_TRANS))
        if n_sv is not None:
            segS["mode"] = np.where(q_s == p_t, MODE_EYE, np.where(q_s < p_t, MODE_AUG_PLAIN, MODE_AUG_TRANS))
            segS["pad"] = n_sv[p_t]
        segS["layers"] = 1
        segS["rows"] = npno[q_s]
        segS["cols"] = npno[p_t]
        # decay with the distance between the replaced and the replacing orbital
        dist = np.zeros(len(ukey))
        a_i, a_j, b_i, b_j = pi[p_t], pj[p_t], pi[q_s], pj[q_s]
        dist = np.abs((a_i + a_j) - (b_i + b_j)).astype(np.float64)
        segS["scale"] = np.exp(-dist / 4.0) / (np.sqrt(npno[p_t].astype(np.float64)) + np.sqrt(npno[q_s].astype(np.float64)))
        segs["S"] = segS

    return Problem(name=name, seed=seed, n_occ=n_occ, is_somo=is_somo, pi=pi, pj=pj,
                   npno=npno, naux=naux, blocks=blocks, off_B=off_B, off_T=off_T, off_K=off_K,
                   off_eps=off_eps, cpl_rowptr=rowptr, cpl_src=cpl_src, cpl_k=cpl_k,
                   cpl_side=cpl_side, cpl_off_S=cpl_off_S, f_a=f_a, f_b=f_b, eps_a=eps_a,
                   eps_b=eps_b, n_B=n_B, n_T=n_T, n_K=n_K, n_S=n_S, segs=segs, S_host=S_host,
                   pair_index=pair_index, hh_rowptr=hh_rowptr, hh_src=hh_src, hh_k=hh_k, hh_l=hh_l,
                   hh_w=hh_w, hh_off_S=hh_off_S.astype(np.int64), hole_scale=hh_scale, hole_range=hh_range,
                   n_sv=n_sv, quadratic=bool(cfg.get("quadratic", False)) and hh_scale != 0.0,
                   ring_rowptr=ring_rowptr, ring_src=ring_src, ring_role=ring_role, ring_m=ring_m,
                   ring_off_S=ring_off_S, ring_off_X=r_off[0::2].copy(), ring_off_J=r_off[1::2].copy(),
                   n_Rg=n_Rg, ring_scale=ring_scale, ring_range=ring_range,
                   quadratic_occ=bool(cfg.get("quadratic_occ", False)))
