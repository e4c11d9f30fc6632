"""FP64 oracle: open-shell pair residual, closed-shell residual, Jacobi, energies.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

SPIN = {"AA": (0, 0), "BB": (1, 1), "AB": (0, 1), "BA": (1, 0)}
ORDER = ("AA", "BB", "AB", "BA")


def stored_blocks(i, j, is_somo):
    """Spin blocks kept for pair (i, j), i <= j (Sec. II.A, high-spin cases).

    SOMOs are occupied for alpha only.  A block s s' needs i in occ_s and
    j in occ_s'; same-spin blocks vanish for i == j (Pauli); for i == j the
    beta-alpha block is the transpose of the alpha-beta block and is not kept.
    DOMO-DOMO pairs thus have 4 blocks, DOMO-SOMO pairs 2 (AA and the one with
    the SOMO as alpha electron), SOMO-SOMO pairs 1 (AA), diagonal DOMO pairs 1.
    """
    out = []
    for name in ORDER:
        s1, s2 = SPIN[name]
        in1 = s1 == 0 or not is_somo[i]
        in2 = s2 == 0 or not is_somo[j]
        if not (in1 and in2):
            continue
        if s1 == s2 and i == j:
            continue
        if i == j and name == "BA":
            continue
        out.append(name)
    return out


def name_of(s1, s2):
    for k, v in SPIN.items():
        if v == (s1, s2):
            return k
    raise KeyError((s1, s2))


class OccInts:
    """Occupied four-index integrals (k i | l j) (chemists' notation) from a dense
    array g[k, i, l, j]; neighbors(i) lists the k for which (k i | . .) may be
    non-zero (here every orbital)."""

    def __init__(self, g):
        self.g = np.asarray(g, dtype=np.float64)

    def value(self, k, i, l, j):
        return float(self.g[k, i, l, j])

    def neighbors(self, i):
        return range(self.g.shape[0])


class Inputs:
    """Everything the residual reads, held per pair in plain numpy arrays.

    pairs      list of (i, j) with i <= j (retained pairs)
    B[p]       (m_p, n_p, n_p) density-fitting three-index integrals (Q|ac)
    K[p]       (n_p, n_p) spatial exchange integrals (i a | j b)
    eps_a[p], eps_b[p]   (n_p,) virtual PNO energies per spin
    f_a, f_b   (n_occ, n_occ) occupied Fock matrices per spin
    S(p, q)    overlap S_{p,q} (n_p x n_q) between the PNOs of two pairs
    occ_ints   optional occupied integrals (k i | l j) of the hole-hole ladder:
               an object with value(k, i, l, j) and neighbors(i) (the k that
               can give a non-zero (k i | . .)); None: no hole-hole term
    n_sv[p]    optional: the last n_sv[p] of the pair's n_p virtual functions
               are SOMOs (Sec. II.B.4: every PNO set is augmented by the
               SOMOs, which are virtual for beta electrons only); they belong
               to the beta virtual space, not to the alpha one.  B, K, S and
               eps cover all n_p functions (the SOMO part of S between two
               pairs is the identity); residual blocks vanish outside the
               virtual spaces of their spins.  None: no SOMO functions.
    ring       optional integrals of the ring/exchange term (RingInts or an
               object with the same couplings(p)); None: no such term
    B and S may be callables (lazy regeneration for large workloads).
    """

    def __init__(self, n_occ, is_somo, pairs, B, K, eps_a, eps_b, f_a, f_b, S, occ_ints=None, n_sv=None,
                 ring=None):
        self.n_occ = int(n_occ)
        self.is_somo = np.asarray(is_somo).astype(bool)
        self.pairs = [(int(i), int(j)) for i, j in pairs]
        self.index = {pq: p for p, pq in enumerate(self.pairs)}
        self._B, self.K, self.eps_a, self.eps_b = B, K, eps_a, eps_b
        self.f_a, self.f_b = np.asarray(f_a, dtype=np.float64), np.asarray(f_b, dtype=np.float64)
        self._S = S
        self.occ_ints = occ_ints
        self.n_sv = None if n_sv is None else [int(x) for x in n_sv]
        self.quadratic = False   # add the quadratic term over the hole-hole couplings
        self.quadratic_occ = False   # add the quadratic part of the occupied Fock intermediate
        self.ring = ring

    def B(self, p):
        return self._B(p) if callable(self._B) else self._B[p]

    def S(self, p, q):
        return self._S(p, q) if callable(self._S) else self._S[(p, q)]

    def fock_listed(self, p, q):
        """Whether the problem lists an occupied-Fock coupling of target p and
        source q (always, for overlaps given as a function)."""
        if getattr(self, "_fock_listed", None) is not None:
            return (p, q) in self._fock_listed
        return callable(self._S) or (p, q) in self._S

    def npno(self, p):
        return len(self.eps_a[p])

    def occ(self, s):
        return [k for k in range(self.n_occ) if s == 0 or not self.is_somo[k]]

    def fock(self, s):
        return self.f_a if s == 0 else self.f_b

    def eps(self, s, p):
        return self.eps_a[p] if s == 0 else self.eps_b[p]

    def vmask(self, s, p):
        """Which of pair p's virtual functions belong to spin s's virtual space."""
        n = self.npno(p)
        m = np.ones(n, dtype=bool)
        if s == 0 and self.n_sv is not None and self.n_sv[p] > 0:
            m[n - self.n_sv[p]:] = False
        return m

    def blocks(self, p):
        i, j = self.pairs[p]
        return stored_blocks(i, j, self.is_somo)

    @classmethod
    def from_problem(cls, prob, B=None, K=None, S=None, eps_a=None, eps_b=None):
        """Unpack flat arrays laid out by the workload descriptors.

        B, K, S: flat arrays; when B or S is None they are regenerated per pair
        or per coupling from the seeded counters when first needed."""
        P = prob.n_pairs
        pairs = list(zip(prob.pi.tolist(), prob.pj.tolist()))
        n = prob.npno.astype(int)
        m = prob.naux.astype(int)
        eps_a = prob.eps_a if eps_a is None else eps_a
        eps_b = prob.eps_b if eps_b is None else eps_b
        ea = [eps_a[prob.off_eps[p]:prob.off_eps[p] + n[p]].copy() for p in range(P)]
        eb = [eps_b[prob.off_eps[p]:prob.off_eps[p] + n[p]].copy() for p in range(P)]
        if K is None:
            K = prob.materialize("K")
        Kd = [K[prob.off_K[p]:prob.off_K[p] + n[p] ** 2].reshape(n[p], n[p]).copy() for p in range(P)]
        if B is None:
            cache = {}

            def Bf(p):
                if p not in cache:
                    cache[p] = prob.pair_B(p)
                return cache[p]
        else:
            def Bf(p):
                o = prob.off_B[p]
                return B[o:o + m[p] * n[p] ** 2].reshape(m[p], n[p], n[p])
        # overlap lookup (target, source) -> offset of its block (Fock and
        # hole-hole couplings share the blocks)
        where = {}
        for p in range(P):
            for e in range(prob.cpl_rowptr[p], prob.cpl_rowptr[p + 1]):
                where.setdefault((p, int(prob.cpl_src[e])), int(prob.cpl_off_S[e]))
            if prob.n_hh > 0:
                for e in range(prob.hh_rowptr[p], prob.hh_rowptr[p + 1]):
                    where.setdefault((p, int(prob.hh_src[e])), int(prob.hh_off_S[e]))
            if getattr(prob, "n_ring", 0) > 0:
                for e in range(prob.ring_rowptr[p], prob.ring_rowptr[p + 1]):
                    where.setdefault((p, int(prob.ring_src[e])), int(prob.ring_off_S[e]))
        S_full = S if S is not None else (prob.S_host if prob.S_host is not None else None)
        s_cache = {}

        def Sf(p, q):
            o = where[(p, q)]
            if S_full is not None:
                W = S_full[o:o + n[q] * n[p]].reshape(n[q], n[p])
            else:
                if o not in s_cache:
                    segs = prob.segs["S"]
                    u = int(np.searchsorted(segs["off"], o))
                    s_cache[o] = prob.segment("S", u)[0]
                W = s_cache[o]
            return W.T          # stored [c][a] = <c_q|a_p>  ->  S_{p,q}[a][c]
        occ = None
        if prob.hole_scale != 0.0:
            occ = _WorkloadOccInts(prob)
        n_sv = getattr(prob, "n_sv", None)
        ring = _WorkloadRing(prob) if getattr(prob, "n_ring", 0) > 0 else None
        inp = cls(prob.n_occ, prob.is_somo, pairs, Bf, Kd, ea, eb, prob.f_a, prob.f_b, Sf, occ, n_sv, ring)
        inp._fock_listed = {(p, int(prob.cpl_src[e])) for p in range(P)
                            for e in range(prob.cpl_rowptr[p], prob.cpl_rowptr[p + 1])}
        inp.quadratic = bool(getattr(prob, "quadratic", False))
        inp.quadratic_occ = bool(getattr(prob, "quadratic_occ", False))
        return inp


class _WorkloadRing:
    """The workload's ring couplings, integrals regenerated per target pair."""

    def __init__(self, prob):
        self.prob = prob
        self.cache = {}

    def couplings(self, p):
        if p not in self.cache:
            pr = self.prob
            self.cache[p] = [(int(pr.ring_role[e]), int(pr.ring_m[e]), int(pr.ring_src[e]), pr.ring_matrix(e, 0),
                              pr.ring_matrix(e, 1)) for e in range(pr.ring_rowptr[p], pr.ring_rowptr[p + 1])]
        return self.cache[p]


class _WorkloadOccInts:
    """The workload's synthetic occupied integrals, zero beyond |k - i| > range."""

    def __init__(self, prob):
        self.prob = prob

    def value(self, k, i, l, j):
        return self.prob.eri_occ(k, i, l, j)

    def neighbors(self, i):
        d = self.prob.hole_range
        return range(max(0, i - d), min(self.prob.n_occ, i + d + 1))


def unpack_T(prob, flat):
    """Flat T/R array -> {(p, block): n x n} following the workload layout."""
    out = {}
    for p in range(prob.n_pairs):
        n = int(prob.npno[p])
        o = int(prob.off_T[p])
        for name in stored_blocks(int(prob.pi[p]), int(prob.pj[p]), prob.is_somo.astype(bool)):
            out[(p, name)] = flat[o:o + n * n].reshape(n, n).copy()
            o += n * n
    return out


def pack_T(prob, blocks, out=None):
    flat = np.zeros(prob.n_T) if out is None else out
    for p in range(prob.n_pairs):
        n = int(prob.npno[p])
        o = int(prob.off_T[p])
        for name in stored_blocks(int(prob.pi[p]), int(prob.pj[p]), prob.is_somo.astype(bool)):
            if (p, name) in blocks:
                flat[o:o + n * n] = blocks[(p, name)].ravel()
            o += n * n
    return flat


def t_lookup(inp, T, k, l, s1, s2):
    """Amplitude block T^{s1 s2} of the ordered pair (k, l) in the PNOs of {k, l}.

    Returns (pair, block, transposed, matrix) or None when the pair is not
    retained or the block vanishes.  Exchanging both electrons (occupied and
    virtual labels together) leaves a doubles amplitude unchanged, so for
    k > l the block is the transposed s2 s1 block of (l, k)."""
    if k == l and s1 == s2:
        return None
    if k <= l:
        q = inp.index.get((k, l))
        if q is None:
            return None
        if k == l:
            mat = T[(q, "AB")]
            return (q, "AB", s1 == 1, mat.T if s1 == 1 else mat)
        name = name_of(s1, s2)
        if (q, name) not in T:
            return None
        return (q, name, False, T[(q, name)])
    q = inp.index.get((l, k))
    if q is None:
        return None
    name = name_of(s2, s1)
    if (q, name) not in T:
        return None
    return (q, name, True, T[(q, name)].T)


def denominators(inp, p, name):
    i, j = inp.pairs[p]
    s1, s2 = SPIN[name]
    return (inp.eps(s1, p)[:, None] + inp.eps(s2, p)[None, :]
            - inp.fock(s1)[i, i] - inp.fock(s2)[j, j])


def driver(inp, p, name):
    s1, s2 = SPIN[name]
    Kp = inp.K[p]
    return Kp - Kp.T if s1 == s2 else Kp.copy()


def ladder(Bp, Tb):
    """sum_Q B^Q T (B^Q)^T: R_ab = sum_Q sum_cd B^Q_ac T_cd B^Q_bd, as two matmuls
    over the combined (Q, d) index."""
    m, n, _ = Bp.shape
    X = (Bp.reshape(m * n, n) @ Tb).reshape(m, n, n)            # X[Q,a,d] = sum_c B[Q,a,c] T[c,d]
    return X.transpose(1, 0, 2).reshape(n, m * n) @ Bp.transpose(0, 2, 1).reshape(m * n, n)


def projection_terms(inp, T, p, name):
    """The occupied-Fock terms of block `name` of pair p: list of
    (weight, q, S_pq, source tuple from t_lookup)."""
    i, j = inp.pairs[p]
    s1, s2 = SPIN[name]
    out = []
    for k in inp.occ(s1):                      # k replaces i
        if k == i:
            continue
        w = inp.fock(s1)[k, i]
        if w == 0.0:
            continue
        src = t_lookup(inp, T, k, j, s1, s2)
        if src is None:
            continue
        out.append((w, src[0], inp.S(p, src[0]), src))
    for k in inp.occ(s2):                      # k replaces j
        if k == j:
            continue
        w = inp.fock(s2)[k, j]
        if w == 0.0:
            continue
        src = t_lookup(inp, T, i, k, s1, s2)
        if src is None:
            continue
        out.append((w, src[0], inp.S(p, src[0]), src))
    return out


def quadratic_weight(inp, T, p, name, k, l, q, Spq):
    """Weight that the quadratic CCSD term adds to the hole-hole coupling
    (k, l) of block `name` of pair p (source pair q = {k, l}, S_pq = S(p, q)).

    In spin orbitals the term is 1/4 sum_KLCD <KL||CD> t_IJ^CD t_KL^AB, i.e.
    the hole-hole ladder 1/2 sum_KL W_KLIJ t_KL^AB with <KL||IJ> replaced by
    W_KLIJ = 1/2 sum_CD <KL||CD> t_IJ^CD.  Reduced to spin blocks like the
    hole-hole term, W adds c_ss' <(k c | l d), T^{ss'}_p> to (k i | l j), with
    c = 1/2 for same spin and 1 for opposite spin, c and d in pair p's PNOs.
    Reading: (k c | l d) in pair p's PNOs is the projection S_pq K_(k,l) S_pq^T
    of pair q's exchange integrals K_q = (min a | max b) (K_q^T when k > l):
    exact when the two pairs share their PNOs (the canonical limit, where a
    brute-force pin checks it)."""
    s1, s2 = SPIN[name]
    Kq = inp.K[q] if k <= l else inp.K[q].T
    c = 0.5 if s1 == s2 else 1.0
    return c * float(np.sum((Spq @ Kq @ Spq.T) * T[(p, name)]))


def hole_terms(inp, T, p, name, quadratic=False):
    """The hole-hole ladder terms of block `name` of pair p = (i, j): list of
    (weight, q, S_pq, source tuple from t_lookup).

    In spin orbitals the term is 1/2 sum_KL <KL||IJ> t_KL^AB.  With I, J of
    spins s, s' it keeps K = k_s, L = l_s' from <KL|IJ> = (k i | l j) and
    K = k_s', L = l_s from <KL|JI>; relabelling the second and using
    t_KL = -t_LK turns it into the first, so the term is
      sum_{k in occ_s, l in occ_s'} (k i | l j) S_{p,kl} T^{ss'}_{(k,l)} S_{kl,p}
    over ordered (k, l), with the amplitude lookup of t_lookup (zero for pairs
    that are not retained).  Its spin-orbital form is checked by brute force."""
    if inp.occ_ints is None:
        return []
    i, j = inp.pairs[p]
    s1, s2 = SPIN[name]
    occ1, occ2 = set(inp.occ(s1)), set(inp.occ(s2))
    out = []
    for k in inp.occ_ints.neighbors(i):
        if k not in occ1:
            continue
        for l in inp.occ_ints.neighbors(j):
            if l not in occ2:
                continue
            w = inp.occ_ints.value(k, i, l, j)
            if w == 0.0 and not quadratic:
                continue
            src = t_lookup(inp, T, k, l, s1, s2)
            if src is None:
                continue
            Spq = inp.S(p, src[0])
            if quadratic:
                w += quadratic_weight(inp, T, p, name, k, l, src[0], Spq)
            out.append((w, src[0], Spq, src))
    return out


def occ_intermediate(inp, T, m, j, s):
    """Quadratic part of the occupied Fock intermediate, F^s_{mj} =
    1/2 sum_{N,E,F} t_{(j s) N}^{EF} <(m s) N||EF>.  Reduced to spin blocks,
    the two spin assignments of (E, F) make each block count once with
    factor 1:  F^s_{mj} = sum_{n, s_n} <G_(m,n), T^{s s_n}_{(j,n)}>, over
    occupied n of either spin (n in occ_{s_n}), with G[e][f] = (m e | n f)
    over the PNOs of pair {j, n}.  Reading (as in quadratic_weight): those
    integrals are the projection S_{jn,mn} K_(m,n) S_{mn,jn} of pair {m, n}'s
    exchange integrals (K of {m, n}, transposed for m > n); for m = j they
    are K_(j,n) itself.  Terms whose pairs are not retained, or whose pairs
    the problem does not couple by an occupied-Fock coupling (local
    truncation), vanish."""
    total = 0.0
    for n in range(inp.n_occ):
        r = inp.index.get((min(m, n), max(m, n)))
        if r is None:
            continue
        Kmn = inp.K[r] if m <= n else inp.K[r].T
        for sn in (0, 1):
            if sn == 1 and inp.is_somo[n]:
                continue
            src = t_lookup(inp, T, j, n, s, sn)
            if src is None:
                continue
            q = src[0]
            if q == r:
                G = Kmn
            else:
                if not inp.fock_listed(q, r):  # coupling not listed: local truncation
                    continue
                Sqr = inp.S(q, r)
                G = Sqr @ Kmn @ Sqr.T
            total += float(np.sum(G * src[3]))
    return total


class OccIntermediate:
    """F^s_{mj} of amplitudes T, computed when first asked for (occ_intermediate)."""

    def __init__(self, inp, T):
        self.inp, self.T, self.cache = inp, T, {}

    def get(self, key):
        if key not in self.cache:
            m, j, s = key
            self.cache[key] = occ_intermediate(self.inp, self.T, m, j, s)
        return self.cache[key]


def occ_quadratic_block(inp, T, p, name, F):
    """-P(IJ) sum_M t_IM^AB F_MJ for block `name` of pair p = (i, j), F an
    OccIntermediate (get((m, j, s)) -> F^s_{mj}).  t_JM^AB = -t_MJ^AB turns the exchanged half into
    the same form as the first, like the occupied-Fock projections:
      - sum_{m in occ_s} F^s_{mi} S T^{ss'}_{(m,j)} S^T
      - sum_{m in occ_s'} F^{s'}_{mj} S T^{ss'}_{(i,m)} S^T,
    m = i and m = j included (the pair itself, identity overlap); sources
    without a listed occupied-Fock coupling to p are left out."""
    i, j = inp.pairs[p]
    s1, s2 = SPIN[name]
    out = np.zeros_like(T[(p, name)])
    for side, (s, rep_, keep) in enumerate(((s1, i, j), (s2, j, i))):
        for m in inp.occ(s):
            src = t_lookup(inp, T, m, j, s1, s2) if side == 0 else t_lookup(inp, T, i, m, s1, s2)
            if src is None:
                continue
            if src[0] != p and not inp.fock_listed(p, src[0]):
                continue
            f = F.get((m, rep_, s))
            if src[0] == p:
                out -= f * src[3]
            else:
                Spq = inp.S(p, src[0])
                out -= f * (Spq @ src[3] @ Spq.T)
    return out


class RingInts:
    """Integrals of the ring/exchange term, listed per target pair.

    couplings(p) gives (role, m, q, X, J) tuples for target pair p = (i, j):
    role 0 keeps the target's first occupied index x = i (other index y = j),
    role 1 its second, x = j (y = i); m is the replacing occupied orbital and
    q the retained source pair {x, m};
        X[e][b] = (m e | b y),   J[e][b] = (m y | b e)   (chemists' notation)
    with e over the source's PNOs (rows) and b over the target's (columns).
    A diagonal target (i == j) lists role 0 only: it serves both index orders.
    """

    def __init__(self, table):
        self.table = table          # {p: [(role, m, q, X, J), ...]}

    def couplings(self, p):
        return self.table.get(p, [])


def ring_amplitude(inp, T, x, sx, m, sm, ra, se):
    """The doubles amplitude t_{(x sx)(m sm)}^{(r ra)(e se)} as a matrix [r][e]
    over the PNOs of pair {x, m}, with the pair index: (q, matrix) or None.
    It vanishes unless the virtual spins are those of the occupied ones in
    some order; exchanging the two virtual labels alone changes its sign."""
    if sx == ra and sm == se:
        src = t_lookup(inp, T, x, m, sx, sm)
        return None if src is None else (src[0], src[3])
    if sx == se and sm == ra:
        src = t_lookup(inp, T, x, m, sx, sm)
        return None if src is None else (src[0], -src[3].T)
    return None


def ring_part(inp, T, p, role, ra, cb, s1, s2):
    """F[r][c] = sum_{M, E} t_{X M}^{R E} <M C||E Y> for target pair p, where
    (X, Y) are the target's occupied spin orbitals (i s1, j s2) for role 0 and
    (j s2, i s1) for role 1, R and C virtuals of spins ra and cb in the
    target's PNOs.  <M C||E Y> = (m e | c y) when e has the spin of m and
    c that of y, minus (m y | c e) when m has the spin of y and e that of c;
    the amplitude's virtual index r is carried into the target's PNOs by
    S_{p,q}."""
    i, j = inp.pairs[p]
    (x, sx), (y, sy) = ((i, s1), (j, s2)) if role == 0 else ((j, s2), (i, s1))
    n = inp.npno(p)
    out = np.zeros((n, n))
    for crole, m, q, X, J in inp.ring.couplings(p):
        if i != j and crole != role:
            continue
        Spq = inp.S(p, q)
        for sm in (0, 1):
            if sm == 1 and inp.is_somo[m]:      # M must be occupied: SOMOs are alpha only
                continue
            if cb == sy:                        # (m e | c y), e of spin sm
                a = ring_amplitude(inp, T, x, sx, m, sm, ra, sm)
                if a is not None:
                    assert a[0] == q
                    out += Spq @ a[1] @ X
            if sm == sy:                        # (m y | c e), e of spin cb
                a = ring_amplitude(inp, T, x, sx, m, sm, ra, cb)
                if a is not None:
                    assert a[0] == q
                    out -= Spq @ a[1] @ J
    return out


def ring_block(inp, T, p, name):
    """Ring/exchange term of block `name` of pair p.  In spin orbitals it is
    P(ij) P(ab) sum_ME t_IM^AE <MB||EJ>, the part of the CCSD doubles residual
    that is linear in the doubles and couples pairs through one shared
    occupied index: with F(XY, ab) = sum_ME t_XM^aE <Mb||EY>,
        R_IJ^AB += F(IJ, AB) - F(JI, AB) - F(IJ, BA) + F(JI, BA),
    which for block s s' (A of spin s, B of spin s') is ring_part with role
    0 / 1 and virtual spins (s, s') / (s', s), the latter transposed.  Its
    spin-orbital form is checked by brute force in the canonical limit."""
    s1, s2 = SPIN[name]
    return (ring_part(inp, T, p, 0, s1, s2, s1, s2) - ring_part(inp, T, p, 1, s1, s2, s1, s2)
            - ring_part(inp, T, p, 0, s2, s1, s1, s2).T + ring_part(inp, T, p, 1, s2, s1, s1, s2).T)


def residual_os(inp, T, pairs=None, terms=("driver", "fock", "projection", "ladder", "hole", "quadratic", "ring",
                                           "quadratic_occ")):
    """Open-shell residual blocks {(p, name): R} for the given target pairs.
    The hole-hole term is present only when inp.occ_ints is given; with
    inp.quadratic set, its couplings carry the quadratic CCSD term too
    (quadratic_weight); the ring/exchange term only when inp.ring is given
    (ring_block); with inp.quadratic_occ the quadratic part of the occupied
    Fock intermediate (occ_intermediate, occ_quadratic_block).  With SOMO
    virtual functions (inp.n_sv) each block is the model residual restricted
    to its spins' virtual spaces (the rows of an alpha virtual index and the
    columns of an alpha virtual index vanish at SOMO functions); amplitudes
    must vanish there too."""
    R = {}
    Focc = None
    if "quadratic_occ" in terms and getattr(inp, "quadratic_occ", False):
        Focc = OccIntermediate(inp, T)
    for p in (range(len(inp.pairs)) if pairs is None else pairs):
        Bp = inp.B(p) if "ladder" in terms else None
        for name in inp.blocks(p):
            Tb = T[(p, name)]
            r = np.zeros_like(Tb)
            if "driver" in terms:
                r += driver(inp, p, name)
            if "fock" in terms:
                r += denominators(inp, p, name) * Tb
            if "projection" in terms:
                for w, q, Spq, src in projection_terms(inp, T, p, name):
                    r -= w * (Spq @ src[3] @ Spq.T)
            if "ladder" in terms:
                r += ladder(Bp, Tb)
            if "hole" in terms:
                quad = "quadratic" in terms and getattr(inp, "quadratic", False)
                for w, q, Spq, src in hole_terms(inp, T, p, name, quadratic=quad):
                    r += w * (Spq @ src[3] @ Spq.T)
            if "ring" in terms and getattr(inp, "ring", None) is not None:
                r += ring_block(inp, T, p, name)
            if Focc is not None:
                r += occ_quadratic_block(inp, T, p, name, Focc)
            if inp.n_sv is not None:
                s1, s2 = SPIN[name]
                r = r * (inp.vmask(s1, p)[:, None] & inp.vmask(s2, p)[None, :])
            R[(p, name)] = r
    return R


def jacobi(inp, T, R):
    """T' = T - R / D for every stored block (all pairs at once)."""
    return {key: T[key] - R[key] / denominators(inp, *key) for key in R}


def pair_energies(inp, T):
    """e[(p, name)] = w <K^{ss'}_p, T^{ss'}_p>, w = 1/2 same spin, 1 opposite."""
    e = {}
    for (p, name), Tb in T.items():
        s1, s2 = SPIN[name]
        w = 0.5 if s1 == s2 else 1.0
        e[(p, name)] = w * float(np.sum(driver(inp, p, name) * Tb))
    return e


# ---------------------------------------------------------------------------
# closed-shell reference (separate code path: spatial amplitudes only)
# ---------------------------------------------------------------------------

def residual_cs(pairs, B, K, eps, f, S, Tcs, occ_ints=None):
    """Closed-shell residual of the same model on spatial amplitudes T_p (i <= j).

    R_p = K_p + (eps + eps - f_ii - f_jj) o T_p - sum_{k != i} f_ki S T_kj S^T
          - sum_{k != j} f_kj S T_ik S^T + sum_Q B^Q T_p B^Q^T
          + sum_{k,l} (k i | l j) S T_kl S^T       (with occ_ints),
    with T_(k,l) = T_(l,k)^T for k > l."""
    index = {pq: p for p, pq in enumerate(pairs)}

    def amp(k, l):
        if k <= l:
            q = index.get((k, l))
            return None if q is None else (q, Tcs[q])
        q = index.get((l, k))
        return None if q is None else (q, Tcs[q].T)

    n_occ = f.shape[0]
    R = []
    for p, (i, j) in enumerate(pairs):
        Tp = Tcs[p]
        r = K[p] + (eps[p][:, None] + eps[p][None, :] - f[i, i] - f[j, j]) * Tp
        for k in range(n_occ):
            if k != i and f[k, i] != 0.0:
                a = amp(k, j)
                if a is not None:
                    Spq = S(p, a[0])
                    r = r - f[k, i] * (Spq @ a[1] @ Spq.T)
            if k != j and f[k, j] != 0.0:
                a = amp(i, k)
                if a is not None:
                    Spq = S(p, a[0])
                    r = r - f[k, j] * (Spq @ a[1] @ Spq.T)
        Bp = B(p)
        for Q in range(Bp.shape[0]):
            r = r + Bp[Q] @ Tp @ Bp[Q].T
        if occ_ints is not None:
            for k in occ_ints.neighbors(i):
                for l in occ_ints.neighbors(j):
                    w = occ_ints.value(k, i, l, j)
                    a = amp(k, l) if w != 0.0 else None
                    if a is not None:
                        Spq = S(p, a[0])
                        r = r + w * (Spq @ a[1] @ Spq.T)
        R.append(r)
    return R


def pair_energies_cs(pairs, K, Tcs):
    """Closed-shell pair energy (2 - delta_ij) <K, 2T - T^T>."""
    return [(2.0 - (i == j)) * float(np.sum(K[p] * (2.0 * Tcs[p] - Tcs[p].T)))
            for p, (i, j) in enumerate(pairs)]
