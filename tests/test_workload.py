"""Seeded generator: published Philox vectors and per-element regeneration."""
import os

import numpy as np

from workload import build_problem, philox
from workload.problem import segment_values

HERE = os.path.dirname(__file__)


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*[np.array([c]) for c in v[:4]], v[4], v[5])
        assert [int(o[0]) for o in out] == v[6:]


def test_irwin_hall_normals_moments_and_bounds():
    z = philox.normals(7, 3, 5, np.arange(200000, dtype=np.uint64))
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert np.max(np.abs(z)) <= 2 * np.sqrt(3.0)


def test_segments_symmetric_antisymmetric_and_regenerable():
    prob = build_problem("tiny")
    B = prob.pair_B(5)
    assert np.array_equal(B, B.transpose(0, 2, 1))
    flat = prob.materialize("B")
    o = prob.off_B[5]
    assert np.array_equal(flat[o:o + B.size], B.ravel())
    T = prob.materialize("T")
    seg = prob.segs["T"][0]
    t = segment_values(prob.seed, seg).reshape(seg["rows"], seg["cols"])
    if seg["mode"] == 2:
        assert np.array_equal(t, -t.T)


def test_random_overlaps_of_reverse_couplings_are_transposes():
    prob = build_problem("chain", n_occ=20, band=4, somos=(6, 13))
    S = prob.materialize("S")
    where = {}
    for p in range(prob.n_pairs):
        for e in range(prob.cpl_rowptr[p], prob.cpl_rowptr[p + 1]):
            where[(p, int(prob.cpl_src[e]))] = int(prob.cpl_off_S[e])
    n = prob.npno
    checked = 0
    for (p, q), o in where.items():
        o2 = where[(q, p)]
        W = S[o:o + n[q] * n[p]].reshape(n[q], n[p])        # S_{q,p}
        W2 = S[o2:o2 + n[p] * n[q]].reshape(n[p], n[q])     # S_{p,q}
        assert np.array_equal(W, W2.T)
        checked += 1
    assert checked == len(where)


def test_spin_dependent_offdiagonal_fock_option():
    """fock_spin draws the beta off-diagonal occupied Fock from a field of its
    own on the alpha support: symmetric, different from alpha, same coupling
    list, and the default recipe unchanged."""
    base = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16), fock_spin=0.3)
    assert np.array_equal(base.f_a, prob.f_a) and np.array_equal(base.f_b, build_problem(
        "chain", n_occ=24, band=6, somos=(7, 16)).f_b)
    d = prob.f_b - prob.f_a - np.diag(np.diag(prob.f_b - prob.f_a))
    assert np.array_equal(prob.f_b, prob.f_b.T)
    assert np.count_nonzero(d) == np.count_nonzero(prob.f_a - np.diag(np.diag(prob.f_a)))
    assert np.array_equal(prob.cpl_src, base.cpl_src) and np.array_equal(prob.cpl_k, base.cpl_k)


def test_spin_dependent_fock_makes_a_spin_swap_visible():
    """With fock_spin, taking the alpha Fock matrix for a beta electron (or the
    reverse) in the projection weights changes the residual far beyond the
    1e-12 parity tolerance, in every spin-block class that has a beta
    electron; without it only the diagonal differs, which the projection never
    reads."""
    import oracle
    from oracle.model import unpack_T
    for spin, expect_visible in ((0.3, True), (0.0, False)):
        prob = build_problem("chain", n_occ=12, band=3, somos=(4, 8), npno=("fixed", 6), naux=("fixed", 10),
                             fock_spin=spin)
        inp = oracle.Inputs.from_problem(prob, B=prob.materialize("B"), K=prob.materialize("K"),
                                         S=prob.materialize("S"))
        T = unpack_T(prob, prob.materialize("T"))
        R = oracle.residual_os(inp, T, terms=("projection",))
        fb_swapped = prob.f_a.copy()
        np.fill_diagonal(fb_swapped, np.diag(prob.f_b))     # keep the diagonal (it never enters)
        bad = oracle.Inputs(inp.n_occ, inp.is_somo, inp.pairs, inp._B, inp.K, inp.eps_a, inp.eps_b,
                            inp.f_a, fb_swapped, inp._S)
        Rb = oracle.residual_os(bad, T, terms=("projection",))
        scale = max(float(np.max(np.abs(v))) for v in R.values())
        for name in ("BB", "AB", "BA"):
            diff = max(float(np.max(np.abs(R[k] - Rb[k]))) for k in R if k[1] == name)
            if expect_visible:
                assert diff > 1e-6 * scale, (name, diff, scale)
            else:
                assert diff == 0.0, (name, diff)
        assert max(float(np.max(np.abs(R[k] - Rb[k]))) for k in R if k[1] == "AA") == 0.0


def test_hole_hole_couplings_follow_the_integral_rule():
    """Hole-hole couplings of target (i, j): every ordered (k, l) with a
    non-zero synthetic integral (k i | l j) whose pair {k, l} is retained,
    weight = that integral; the integrals have the eightfold symmetry of real
    two-electron integrals; self-couplings point at identity overlap blocks;
    without the option the workload is unchanged."""
    base = build_problem("chain", n_occ=16, band=4, somos=(5, 11))
    prob = build_problem("chain", n_occ=16, band=4, somos=(5, 11), hole_ladder=0.02, hole_range=2)
    assert base.n_hh == 0 and prob.n_hh > 0
    assert np.array_equal(base.cpl_src, prob.cpl_src)
    rng = np.random.default_rng(3)
    for _ in range(50):
        k, i, l, j = (int(x) for x in rng.integers(0, 16, 4))
        v = prob.eri_occ(k, i, l, j)
        for perm in ((i, k, l, j), (k, i, j, l), (l, j, k, i), (j, l, i, k)):
            assert prob.eri_occ(*perm) == v
        if abs(k - i) > 2 or abs(l - j) > 2:
            assert v == 0.0
    S = prob.materialize("S")
    for p in range(prob.n_pairs):
        i, j = int(prob.pi[p]), int(prob.pj[p])
        want = {}
        for k in range(16):
            for l in range(16):
                w = prob.eri_occ(k, i, l, j)
                q = prob.pair_index.get((min(k, l), max(k, l)))
                if w != 0.0 and q is not None:
                    want[(k, l)] = (q, w)
        got = {(int(prob.hh_k[e]), int(prob.hh_l[e])): (int(prob.hh_src[e]), float(prob.hh_w[e]))
               for e in range(prob.hh_rowptr[p], prob.hh_rowptr[p + 1])}
        assert got == want, p
        for e in range(prob.hh_rowptr[p], prob.hh_rowptr[p + 1]):
            if prob.hh_src[e] == p:
                n = int(prob.npno[p])
                o = int(prob.hh_off_S[e])
                assert np.array_equal(S[o:o + n * n].reshape(n, n), np.eye(n))


def test_ring_couplings_follow_their_rule():
    """Ring couplings of target (i, j): role 0 (x = i, y = j) and, for i < j,
    role 1 (x = j, y = i), every m with |m - x| <= range whose pair {x, m} is
    retained; self-couplings point at identity overlap blocks; the integral
    blocks are regenerable and sized n_src x n_target; without the option
    the workload is unchanged."""
    base = build_problem("chain", n_occ=16, band=4, somos=(5, 11))
    prob = build_problem("chain", n_occ=16, band=4, somos=(5, 11), ring=0.05, ring_range=2)
    assert base.n_ring == 0 and prob.n_ring > 0
    assert np.array_equal(base.cpl_src, prob.cpl_src) and np.array_equal(base.off_T, prob.off_T)
    S = prob.materialize("S")
    Rg = prob.materialize("Rg")
    for p in range(prob.n_pairs):
        i, j = int(prob.pi[p]), int(prob.pj[p])
        want = []
        for role, x in enumerate((i, j)):
            if role == 1 and i == j:
                continue
            for m in range(max(0, x - 2), min(16, x + 3)):
                q = prob.pair_index.get((min(x, m), max(x, m)))
                if q is not None:
                    want.append((role, m, q))
        rows = range(prob.ring_rowptr[p], prob.ring_rowptr[p + 1])
        assert [(int(prob.ring_role[e]), int(prob.ring_m[e]), int(prob.ring_src[e])) for e in rows] == want, p
        n = int(prob.npno[p])
        for e in rows:
            q = int(prob.ring_src[e])
            nq = int(prob.npno[q])
            if q == p:
                o = int(prob.ring_off_S[e])
                assert np.array_equal(S[o:o + n * n].reshape(n, n), np.eye(n))
            for which, off in ((0, prob.ring_off_X[e]), (1, prob.ring_off_J[e])):
                M = prob.ring_matrix(e, which)
                assert M.shape == (nq, n)
                assert np.array_equal(Rg[int(off):int(off) + nq * n].reshape(nq, n), M)
    assert not np.array_equal(prob.ring_matrix(0, 0), prob.ring_matrix(0, 1))
