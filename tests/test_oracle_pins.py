"""Pins of the FP64 oracle against what the paper and the mathematics fix."""
import numpy as np
import pytest

import oracle
from oracle.model import stored_blocks, residual_cs, pair_energies_cs, ladder, t_lookup
from oracle.solver import keys_of, flatten, unflatten, apply_operator
from tests.oracle_helpers import make_inputs, random_T, inner
from workload import build_problem


# ---------------------------------------------------------------- block rule
def test_spin_case_counts_per_pair_class():
    # Sec. II.A: DOMO-DOMO pairs carry aa, ab, bb; SOMO-DOMO two (aa, ab); SOMO-SOMO one (aa)
    somo = np.array([0, 0, 1, 1], dtype=bool)
    assert stored_blocks(0, 1, somo) == ["AA", "BB", "AB", "BA"]     # ab and ba both kept for i < j
    assert stored_blocks(0, 0, somo) == ["AB"]                       # diagonal DOMO pair
    assert stored_blocks(0, 2, somo) == ["AA", "BA"]                 # DOMO-SOMO: the SOMO (j) is the alpha electron
    assert stored_blocks(2, 3, somo) == ["AA"]                       # SOMO-SOMO
    assert stored_blocks(2, 2, somo) == []                           # SOMO diagonal: nothing
    somo2 = np.array([1, 0, 0], dtype=bool)
    assert stored_blocks(0, 1, somo2) == ["AA", "AB"]                # SOMO (i) first: alpha-beta


@pytest.mark.parametrize("name,blocks,pairs", [("tiny", 561, 171), ("chain", 11958, 3150)])
def test_generator_masks_follow_oracle_rule(name, blocks, pairs):
    prob = build_problem(name)
    assert prob.n_pairs == pairs
    bits = {"AA": 1, "BB": 2, "AB": 4, "BA": 8}
    total = 0
    for p in range(prob.n_pairs):
        names = stored_blocks(int(prob.pi[p]), int(prob.pj[p]), prob.is_somo.astype(bool))
        assert int(prob.blocks[p]) == sum(bits[n] for n in names)
        total += len(names)
    assert total == blocks


def test_generator_lists_every_nonzero_projection_term():
    prob = build_problem("chain", n_occ=30, band=5, somos=(9, 20))
    inp = oracle.Inputs.from_problem(prob)
    listed = {(p, int(prob.cpl_src[e]), int(prob.cpl_k[e]), int(prob.cpl_side[e]))
              for p in range(prob.n_pairs) for e in range(prob.cpl_rowptr[p], prob.cpl_rowptr[p + 1])}
    want = set()
    for p, (i, j) in enumerate(inp.pairs):
        for side, (rep, keep) in enumerate(((i, j), (j, i))):
            for k in range(inp.n_occ):
                if k != rep and inp.f_a[k, rep] != 0.0:
                    q = inp.index.get((min(k, keep), max(k, keep)))
                    if q is not None:
                        want.add((p, q, k, side))
    assert listed == want


# ------------------------------------------------- P1 closed-shell reduction
def test_closed_shell_reduction_exact():
    # Abstract and Sec. II.B.2: with no SOMOs the open-shell formalism must reproduce
    # the closed-shell one (one PNO set for all spins).
    rng = np.random.default_rng(11)
    inp = make_inputs(rng, n_occ=6, somos=(), npno=5, naux=7, hole=0.05)
    Tcs = []
    for p, (i, j) in enumerate(inp.pairs):
        g = 1e-2 * rng.standard_normal((5, 5))
        Tcs.append((g + g.T) / 2 if i == j else g)
    T = {}
    for p, (i, j) in enumerate(inp.pairs):
        for name in inp.blocks(p):
            T[(p, name)] = Tcs[p] - Tcs[p].T if name in ("AA", "BB") else Tcs[p].copy()
    R = oracle.residual_os(inp, T)
    Rcs = residual_cs(inp.pairs, inp.B, inp.K, inp.eps_a, inp.f_a, inp.S, Tcs, occ_ints=inp.occ_ints)
    for p, (i, j) in enumerate(inp.pairs):
        for name in inp.blocks(p):
            want = Rcs[p] - Rcs[p].T if name in ("AA", "BB") else Rcs[p]
            np.testing.assert_allclose(R[(p, name)], want, rtol=0, atol=1e-14)
    # energies after a Jacobi step
    Tn = oracle.jacobi(inp, T, R)
    e_os = sum(oracle.pair_energies(inp, Tn).values())
    Tcs_n = [Tcs[p] - Rcs[p] / (inp.eps_a[p][:, None] + inp.eps_a[p][None, :]
                                - inp.f_a[i, i] - inp.f_a[j, j]) for p, (i, j) in enumerate(inp.pairs)]
    e_cs = sum(pair_energies_cs(inp.pairs, inp.K, Tcs_n))
    assert abs(e_os - e_cs) <= 1e-15 * max(1.0, abs(e_cs)) * 10


def test_closed_shell_energy_identity_worked():
    # same-spin + opposite-spin energies of a closed-shell i<j pair: 2<K, 2T - T^T>
    rng = np.random.default_rng(3)
    K = rng.standard_normal((4, 4))
    T = rng.standard_normal((4, 4))
    same = 0.5 * np.sum((K - K.T) * (T - T.T))
    opp = np.sum(K * T)
    assert np.isclose(2 * same + 2 * opp, 2 * np.sum(K * (2 * T - T.T)), rtol=1e-14)


# ------------------------------------ P2 canonical limit vs brute force
@pytest.mark.parametrize("somos,hole", [((1,), 0.0), ((1, 3), 0.0), ((1,), 0.05), ((1, 3), 0.05), ((), 0.05)])
def test_canonical_limit_matches_spin_orbital_bruteforce(somos, hole):
    # Sec. IV.A: with no truncation the method equals its canonical counterpart;
    # hole > 0 adds the hole-hole ladder 1/2 sum_KL <KL||IJ> t_KL from explicit
    # antisymmetrised occupied integrals
    rng = np.random.default_rng(5 + len(somos) + int(100 * hole))
    inp = make_inputs(rng, n_occ=5, somos=somos, npno=5, naux=6, shared_space=True, hole=hole)
    T = random_T(rng, inp, scale=0.05)
    R = oracle.residual_os(inp, T)
    Tb = {(inp.pairs[p], name): v for (p, name), v in T.items()}
    Kp = {inp.pairs[p]: inp.K[p] for p in range(len(inp.pairs))}
    Rbf, Ebf = oracle.residual_spinorbital(inp.n_occ, inp.is_somo, inp.B(0), Kp, inp.eps_a[0],
                                           inp.eps_b[0], inp.f_a, inp.f_b, Tb, inp.pairs, g_occ=inp.g_occ)
    n_checked = 0
    for (p, name), r in R.items():
        np.testing.assert_allclose(r, Rbf[(inp.pairs[p], name)], rtol=0, atol=1e-13)
        n_checked += 1
    assert n_checked == len(keys_of(inp))
    # R_(j,i) = R_(i,j)^T with spins swapped (ordered pairs), e.g. the beta-alpha diagonal block
    for p, (i, j) in enumerate(inp.pairs):
        if i == j and (p, "AB") in R:
            np.testing.assert_allclose(Rbf[((i, i), "BA")], R[(p, "AB")].T, atol=1e-13)
    # energy weights: sum of pair energies = 1/4 sum <IJ||AB> t
    e = sum(oracle.pair_energies(inp, T).values())
    assert abs(e - Ebf) < 1e-14


# ----------------------------- P3/P9 relabelling and PNO permutations
def _reversed_inputs(inp):
    n = inp.n_occ
    rev = lambda k: n - 1 - k
    new_pairs = [(rev(j), rev(i)) for (i, j) in inp.pairs]
    order = sorted(range(len(new_pairs)), key=lambda p: new_pairs[p])
    newp = {old: new for new, old in enumerate(order)}
    pairs = [new_pairs[o] for o in order]
    B = {newp[p]: inp.B(p) for p in range(len(inp.pairs))}
    K = {newp[p]: inp.K[p].T.copy() for p in range(len(inp.pairs))}
    ea = {newp[p]: inp.eps_a[p] for p in range(len(inp.pairs))}
    eb = {newp[p]: inp.eps_b[p] for p in range(len(inp.pairs))}
    perm = np.arange(n)[::-1]
    fa = inp.f_a[np.ix_(perm, perm)]
    fb = inp.f_b[np.ix_(perm, perm)]
    inv = {v: k for k, v in newp.items()}
    S = lambda p, q: inp.S(inv[p], inv[q])
    occ = None
    if inp.occ_ints is not None:
        occ = oracle.OccInts(inp.g_occ[::-1, ::-1, ::-1, ::-1].copy())
    new = oracle.Inputs(n, inp.is_somo[::-1].copy(), pairs, B, K, ea, eb, fa, fb, S, occ)
    return new, newp


def test_orbital_relabelling_transposes_blocks():
    # R_(j,i)^{s's} = (R_(i,j)^{ss'})^T: reversing the chain swaps the electrons of every pair
    rng = np.random.default_rng(21)
    inp = make_inputs(rng, n_occ=7, somos=(2, 5), npno=4, naux=5, band=3, hole=0.05)
    T = random_T(rng, inp)
    new, newp = _reversed_inputs(inp)
    swap = {"AA": "AA", "BB": "BB", "AB": "BA", "BA": "AB"}
    Tn = {}
    for (p, name), v in T.items():
        i, j = inp.pairs[p]
        nn = "AB" if i == j else swap[name]
        Tn[(newp[p], nn)] = v if i == j else v.T
    R = oracle.residual_os(inp, T)
    Rn = oracle.residual_os(new, Tn)
    assert set(Rn) == set(Tn)
    for (p, name), v in R.items():
        i, j = inp.pairs[p]
        if i == j:
            np.testing.assert_allclose(Rn[(newp[p], "AB")], v, atol=1e-15)
        else:
            np.testing.assert_allclose(Rn[(newp[p], swap[name])], v.T, atol=1e-15)


def test_pno_permutation_covariance():
    # Sec. II.B.2: pair energies and pair functions are invariant to unitary rotations
    # within the virtual space; a relabelling of one pair's PNOs permutes its residual
    rng = np.random.default_rng(8)
    inp = make_inputs(rng, n_occ=5, somos=(3,), npno=5, naux=6, hole=0.05)
    T = random_T(rng, inp)
    R = oracle.residual_os(inp, T)
    p0 = 4
    pi = rng.permutation(5)
    B = {p: (inp.B(p)[:, pi][:, :, pi] if p == p0 else inp.B(p)) for p in range(len(inp.pairs))}
    K = {p: (inp.K[p][np.ix_(pi, pi)] if p == p0 else inp.K[p]) for p in range(len(inp.pairs))}
    ea = {p: (inp.eps_a[p][pi] if p == p0 else inp.eps_a[p]) for p in range(len(inp.pairs))}
    eb = {p: (inp.eps_b[p][pi] if p == p0 else inp.eps_b[p]) for p in range(len(inp.pairs))}

    def S(p, q):
        s = inp.S(p, q)
        if p == p0:
            s = s[pi, :]
        if q == p0:
            s = s[:, pi]
        return s
    new = oracle.Inputs(inp.n_occ, inp.is_somo, inp.pairs, B, K, ea, eb, inp.f_a, inp.f_b, S, inp.occ_ints)
    Tp = {k: (v[np.ix_(pi, pi)] if k[0] == p0 else v) for k, v in T.items()}
    Rp = oracle.residual_os(new, Tp)
    for k, v in R.items():
        want = v[np.ix_(pi, pi)] if k[0] == p0 else v
        np.testing.assert_allclose(Rp[k], want, atol=1e-15)


# ------------------------------------------------------- P5 / P6 closed forms
def test_mp2_limit_closed_form():
    rng = np.random.default_rng(2)
    inp = make_inputs(rng, n_occ=5, somos=(4,), npno=4, naux=3, b_scale=0.0, f_off=0.0)
    zero = {k: np.zeros((4, 4)) for k in keys_of(inp)}
    R = oracle.residual_os(inp, zero)
    Tn = oracle.jacobi(inp, zero, R)
    e = oracle.pair_energies(inp, Tn)
    for (p, name), t in Tn.items():
        K = inp.K[p] - inp.K[p].T if name in ("AA", "BB") else inp.K[p]
        D = oracle.denominators(inp, p, name)
        np.testing.assert_allclose(t, -K / D, rtol=1e-15, atol=0)
        w = 0.5 if name in ("AA", "BB") else 1.0
        assert abs(e[(p, name)] + w * np.sum(K * K / D)) < 1e-16


def test_ladder_special_cases():
    rng = np.random.default_rng(4)
    T = rng.standard_normal((6, 6))
    np.testing.assert_allclose(ladder(np.eye(6)[None], T), T, rtol=0, atol=1e-15)
    u = rng.standard_normal(6)
    Bq = np.outer(u, u)[None]
    np.testing.assert_allclose(ladder(Bq, T), (u @ T @ u) * np.outer(u, u), rtol=1e-13)
    # additivity over Q
    B2 = rng.standard_normal((3, 6, 6))
    want = sum(B2[q] @ T @ B2[q].T for q in range(3))
    np.testing.assert_allclose(ladder(B2, T), want, rtol=1e-13)


# ----------------------------------------------------- P7 dense linear solve
def test_jacobi_diis_converges_to_dense_solution():
    rng = np.random.default_rng(7)
    inp = make_inputs(rng, n_occ=4, somos=(3,), npno=4, naux=6, b_scale=0.15, hole=0.05)
    Tstar, A = oracle.dense_solution(inp)
    zero = {k: np.zeros_like(v) for k, v in Tstar.items()}
    T, hist = oracle.solve(inp, zero, 60, use_diis=True, tol_r=1e-13, tol_e=1e-15)
    for k in Tstar:
        np.testing.assert_allclose(T[k], Tstar[k], atol=1e-12)
    # converged residual vanishes
    R = oracle.residual_os(inp, Tstar)
    assert max(np.max(np.abs(r)) for r in R.values()) < 1e-13
    # DIIS needs fewer iterations than plain Jacobi to reach 1e-10
    _, h_j = oracle.solve(inp, zero, 60, use_diis=False)
    it_j = next((k for k, (_, r) in enumerate(h_j) if r < 1e-10), 99)
    it_d = next((k for k, (_, r) in enumerate(hist) if r < 1e-10), 99)
    assert it_d <= it_j


# -------------------------------------------- P8 self-adjointness, Lambda = w T
def test_operator_self_adjoint():
    rng = np.random.default_rng(9)
    inp = make_inputs(rng, n_occ=6, somos=(2, 4), npno=5, naux=6, band=3, hole=0.05)
    keys = keys_of(inp)
    G = {k: rng.standard_normal((5, 5)) for k in keys}
    T = {k: rng.standard_normal((5, 5)) for k in keys}
    a = inner(G, apply_operator(inp, T))
    b = inner(apply_operator(inp, G), T)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_lambda_equals_weighted_amplitudes():
    # the paper approximates Lambda by T^dagger (Sec. II.A); for this model the Lambda
    # equations (D + A)^T Lambda = -dE/dT give Lambda = w T exactly
    rng = np.random.default_rng(10)
    inp = make_inputs(rng, n_occ=4, somos=(1,), npno=3, naux=4, hole=0.05)
    Tstar, A = oracle.dense_solution(inp)
    keys = keys_of(inp)
    dE = {}
    for (p, name) in keys:
        K = inp.K[p] - inp.K[p].T if name in ("AA", "BB") else inp.K[p]
        dE[(p, name)] = (0.5 if name in ("AA", "BB") else 1.0) * K
    lam = np.linalg.solve(A.T, -flatten(dE, keys))
    lam = unflatten(lam, keys, inp)
    for (p, name) in keys:
        w = 0.5 if name in ("AA", "BB") else 1.0
        np.testing.assert_allclose(lam[(p, name)], w * Tstar[(p, name)], atol=1e-13)


# ---------------------------------------------------- P10 VJP by finite differences
def test_vjp_matches_central_differences_and_adjoint_identity():
    rng = np.random.default_rng(12)
    inp = make_inputs(rng, n_occ=5, somos=(2,), npno=4, naux=5, band=2, hole=0.05)
    keys = keys_of(inp)
    T = random_T(rng, inp, scale=0.1)
    Lam = {k: rng.standard_normal(v.shape) for k, v in T.items()}
    dT, dB = oracle.vjp(inp, T, Lam)

    def L(Tx, Bx=None):
        src = inp if Bx is None else oracle.Inputs(inp.n_occ, inp.is_somo, inp.pairs, Bx, inp.K,
                                                   inp.eps_a, inp.eps_b, inp.f_a, inp.f_b, inp.S, inp.occ_ints)
        R = oracle.residual_os(src, Tx)
        return inner(Lam, R)

    h = 1e-5
    dir_T = {k: rng.standard_normal(v.shape) for k, v in T.items()}
    Tp = {k: T[k] + h * dir_T[k] for k in T}
    Tm = {k: T[k] - h * dir_T[k] for k in T}
    fd = (L(Tp) - L(Tm)) / (2 * h)
    an = inner(dT, dir_T)
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))
    # B direction (general, unsymmetrised)
    Bd = {p: rng.standard_normal(inp.B(p).shape) for p in range(len(inp.pairs))}
    Bp = {p: inp.B(p) + h * Bd[p] for p in Bd}
    Bm = {p: inp.B(p) - h * Bd[p] for p in Bd}
    fd = (L(T, Bp) - L(T, Bm)) / (2 * h)
    an = sum(float(np.sum(dB[p] * Bd[p])) for p in dB)
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


# ------------------------------------------------------------- DIIS pins
def test_diis_two_vector_closed_form():
    # Pulay extrapolation minimises |sum c_k e_k| subject to sum c_k = 1; for two
    # error vectors that is c1 = <e2, e2 - e1> / |e1 - e2|^2, c2 = 1 - c1
    rng = np.random.default_rng(41)
    d = oracle.DIIS(max_vec=8, start=2)
    e1, e2 = rng.standard_normal(50), rng.standard_normal(50)
    v1, v2 = rng.standard_normal(50), rng.standard_normal(50)
    d.push(v1, e1)
    d.push(v2, e2)
    c = d.coefficients()
    c1 = float(np.dot(e2, e2 - e1) / np.dot(e1 - e2, e1 - e2))
    np.testing.assert_allclose(c, [c1, 1.0 - c1], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(d.extrapolate(), c1 * v1 + (1 - c1) * v2, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("k", [3, 5, 8])
def test_diis_extrapolated_error_orthogonal_to_affine_hull(k):
    # optimality of the constrained minimum: the extrapolated error e* is
    # orthogonal to every difference e_a - e_b, and the coefficients sum to 1
    rng = np.random.default_rng(100 + k)
    d = oracle.DIIS(max_vec=8, start=3)
    E = rng.standard_normal((k, 40))
    for a in range(k):
        d.push(rng.standard_normal(40), E[a])
    c = d.coefficients()
    assert abs(float(np.sum(c)) - 1.0) < 1e-13
    es = c @ E
    for a in range(k):
        for b in range(a + 1, k):
            assert abs(float(np.dot(es, E[a] - E[b]))) < 1e-12 * float(np.dot(E[a] - E[b], E[a] - E[b]))
    # and it is the minimum: moving inside the hull never lowers |e*|
    for _ in range(20):
        z = rng.standard_normal(k)
        z -= z.mean()
        assert np.linalg.norm((c + 1e-3 * z) @ E) >= np.linalg.norm(es)


def test_diis_drops_the_oldest_of_a_near_dependent_history():
    # e3 = e1 + 1e-9 w: the bordered matrix's condition number is ~1e18 > 1e14,
    # so the oldest vector (e1) is dropped and the remaining two give the
    # two-vector closed form
    rng = np.random.default_rng(43)
    e1, e2, w = rng.standard_normal(30), rng.standard_normal(30), rng.standard_normal(30)
    e3 = e1 + 1e-9 * w
    vs = [rng.standard_normal(30) for _ in range(3)]
    d = oracle.DIIS(max_vec=8, start=3)
    for v, e in zip(vs, (e1, e2, e3)):
        d.push(v, e)
    c = d.coefficients()
    assert d.drops == 1 and len(d.errs) == 2
    assert np.array_equal(d.errs[0], e2) and np.array_equal(d.errs[1], e3)
    c1 = float(np.dot(e3, e3 - e2) / np.dot(e2 - e3, e2 - e3))
    np.testing.assert_allclose(c, [c1, 1.0 - c1], rtol=1e-12)
    # a well-conditioned history of three is kept whole
    d2 = oracle.DIIS(max_vec=8, start=3)
    for v, e in zip(vs, (e1, e2, w)):
        d2.push(v, e)
    d2.coefficients()
    assert d2.drops == 0 and len(d2.errs) == 3


def test_diis_ring_keeps_newest_eight_and_starts_at_three():
    rng = np.random.default_rng(44)
    d = oracle.DIIS(max_vec=8, start=3)
    vs = [rng.standard_normal(12) for _ in range(10)]
    d.push(vs[0], rng.standard_normal(12))
    d.push(vs[1], rng.standard_normal(12))
    # fewer than `start` stored: no extrapolation, the newest vector is taken
    assert np.array_equal(d.extrapolate(), vs[1])
    for v in vs[2:]:
        d.push(v, rng.standard_normal(12))
    assert len(d.vecs) == 8
    assert all(np.array_equal(a, b) for a, b in zip(d.vecs, vs[2:]))


def test_diis_drop_rule_is_scale_invariant():
    # the drop test measures near linear dependence, not the size of the
    # errors: the same history scaled by 1e-10 (a converging iteration) keeps
    # every vector and gives the same coefficients; the near-dependent one
    # still drops its oldest vector
    rng = np.random.default_rng(45)
    E = rng.standard_normal((6, 40))
    for scale in (1.0, 1e-10):
        d = oracle.DIIS(max_vec=8, start=3)
        for e in E:
            d.push(rng.standard_normal(40), scale * e)
        c = d.coefficients()
        assert d.drops == 0 and len(d.errs) == 6
        if scale == 1.0:
            c_ref = c
        else:
            np.testing.assert_allclose(c, c_ref, rtol=1e-10, atol=1e-12)
    e1, e2, w = E[0], E[1], E[2]
    d = oracle.DIIS(max_vec=8, start=3)
    for e in (e1, e2, e1 + 1e-9 * w):
        d.push(rng.standard_normal(40), 1e-10 * e)
    d.coefficients()
    assert d.drops == 1 and len(d.errs) == 2


# ------------------------- SOMO-augmented virtual spaces (Sec. II.B.4)
def _mask_T(inp, T):
    for (p, name), Tb in T.items():
        s1, s2 = oracle.model.SPIN[name]
        Tb *= inp.vmask(s1, p)[:, None] & inp.vmask(s2, p)[None, :]
    return T


@pytest.mark.parametrize("somos,hole", [((1,), 0.0), ((1, 3), 0.0), ((1, 3), 0.05)])
def test_somo_augmented_canonical_limit_matches_bruteforce(somos, hole):
    # every PNO set augmented by the SOMOs, which are beta virtuals only: the
    # pair residual on the augmented space, restricted to each block's virtual
    # spaces, equals the spin-orbital residual whose beta virtual space holds
    # the SOMOs and whose alpha virtual space does not
    rng = np.random.default_rng(41 + len(somos) + int(100 * hole))
    ns = len(somos)
    inp = make_inputs(rng, n_occ=5, somos=somos, npno=4 + ns, naux=6, shared_space=True, hole=hole)
    inp.n_sv = [ns] * len(inp.pairs)
    T = _mask_T(inp, random_T(rng, inp, scale=0.05))
    R = oracle.residual_os(inp, T)
    Tb = {(inp.pairs[p], name): v for (p, name), v in T.items()}
    Kp = {inp.pairs[p]: inp.K[p] for p in range(len(inp.pairs))}
    Rbf, Ebf = oracle.residual_spinorbital(inp.n_occ, inp.is_somo, inp.B(0), Kp, inp.eps_a[0], inp.eps_b[0],
                                           inp.f_a, inp.f_b, Tb, inp.pairs, g_occ=inp.g_occ, n_sv=ns)
    for (p, name), r in R.items():
        np.testing.assert_allclose(r, Rbf[(inp.pairs[p], name)], rtol=0, atol=1e-13)
    # the masks matter: the alpha rows of an AB block vanish at the SOMOs, its
    # beta columns do not
    p = next(p for p, (i, j) in enumerate(inp.pairs) if (p, "AB") in R and i != j)
    assert np.all(R[(p, "AB")][-ns:, :] == 0.0) and np.any(R[(p, "AB")][:, -ns:] != 0.0)
    assert abs(sum(oracle.pair_energies(inp, T).values()) - Ebf) < 1e-14


def test_somo_augmentation_leaves_alpha_alpha_blocks_alone():
    # alpha-alpha amplitudes and residuals live in the PNOs only: augmenting
    # every space by SOMO functions (identity overlap block, arbitrary
    # integrals with them) changes no alpha-alpha residual element; with
    # amplitudes that vanish on the SOMOs the PNO part of every block is
    # unchanged, while beta blocks extend into the SOMO rows and columns
    rng = np.random.default_rng(47)
    inp = make_inputs(rng, n_occ=6, somos=(2, 4), npno=[5] * 21, naux=7, band=5)
    T = random_T(rng, inp, scale=0.05)
    R0 = oracle.residual_os(inp, T)
    ns, P = 2, len(inp.pairs)
    n = 5 + ns

    def grow(M):
        out = rng.standard_normal(M.shape[:-2] + (n, n)) * 0.05
        out[..., :5, :5] = M
        return out
    B = {}
    for p in range(P):
        b = grow(inp.B(p))
        B[p] = (b + b.transpose(0, 2, 1)) / 2.0
        B[p][:, :5, :5] = inp.B(p)
    K = {p: grow(inp.K[p]) for p in range(P)}
    ea = {p: np.concatenate([inp.eps_a[p], [9.0, 9.0]]) for p in range(P)}
    eb = {p: np.concatenate([inp.eps_b[p], rng.uniform(0.1, 0.3, ns)]) for p in range(P)}

    def S(p, q):
        M = np.zeros((n, n))
        M[:5, :5] = inp.S(p, q)
        M[5:, 5:] = np.eye(ns)
        return M
    aug = oracle.Inputs(inp.n_occ, inp.is_somo, inp.pairs, B, K, ea, eb, inp.f_a, inp.f_b, S, n_sv=[ns] * P)
    Ta = {}
    for key, Tb in T.items():
        X = np.zeros((n, n))
        X[:5, :5] = Tb
        Ta[key] = X
    Ta = _mask_T(aug, Ta)
    Ra = oracle.residual_os(aug, Ta)
    for (p, name), r in R0.items():
        if name == "AA":
            np.testing.assert_allclose(Ra[(p, name)][:5, :5], r, rtol=0, atol=1e-15)
            assert np.all(Ra[(p, name)][5:, :] == 0.0) and np.all(Ra[(p, name)][:, 5:] == 0.0)
        elif name == "BB":   # beta virtuals include the SOMOs: the block grows into them
            np.testing.assert_allclose(Ra[(p, name)][:5, :5], r, rtol=0, atol=1e-15)
            assert np.any(Ra[(p, name)][5:, :] != 0.0)


# ------------------- quadratic CCSD term over the hole-hole couplings
@pytest.mark.parametrize("somos", [(), (1,), (1, 3)])
def test_quadratic_term_canonical_limit_matches_bruteforce(somos):
    # 1/4 sum_KLCD <KL||CD> t_IJ^CD t_KL^AB from explicit antisymmetrised
    # integrals, against the pair form: the hole-hole couplings with the
    # weights (k i | l j) + c <K_(k,l), T_ij> (c = 1/2 same spin, 1 opposite)
    rng = np.random.default_rng(61 + len(somos))
    inp = make_inputs(rng, n_occ=5, somos=somos, npno=5, naux=6, shared_space=True, hole=0.05)
    inp.quadratic = True
    T = random_T(rng, inp, scale=0.2)
    R = oracle.residual_os(inp, T)
    Tb = {(inp.pairs[p], name): v for (p, name), v in T.items()}
    Kp = {inp.pairs[p]: inp.K[p] for p in range(len(inp.pairs))}
    Rbf, _ = oracle.residual_spinorbital(inp.n_occ, inp.is_somo, inp.B(0), Kp, inp.eps_a[0], inp.eps_b[0],
                                         inp.f_a, inp.f_b, Tb, inp.pairs, g_occ=inp.g_occ, quadratic=True)
    Rlin, _ = oracle.residual_spinorbital(inp.n_occ, inp.is_somo, inp.B(0), Kp, inp.eps_a[0], inp.eps_b[0],
                                          inp.f_a, inp.f_b, Tb, inp.pairs, g_occ=inp.g_occ)
    big = 0.0
    for (p, name), r in R.items():
        np.testing.assert_allclose(r, Rbf[(inp.pairs[p], name)], rtol=0, atol=1e-13)
        big = max(big, np.abs(Rbf[(inp.pairs[p], name)] - Rlin[(inp.pairs[p], name)]).max())
    assert big > 1e-4            # the quadratic term is not negligible at these amplitudes


def test_quadratic_term_is_quadratic():
    # R(T) - R_linear(T) scales as the square of T and vanishes with T
    rng = np.random.default_rng(67)
    inp = make_inputs(rng, n_occ=6, somos=(2,), npno=[6] * 21, naux=5, hole=0.05)
    T = random_T(rng, inp, scale=0.1)
    lin = ("driver", "fock", "projection", "ladder", "hole")

    def quad(x):
        Tx = {k: x * v for k, v in T.items()}
        inp.quadratic = True
        Rq = oracle.residual_os(inp, Tx)
        inp.quadratic = False
        Rl = oracle.residual_os(inp, Tx, terms=lin)
        return {k: Rq[k] - Rl[k] for k in Rq}
    d1, d2 = quad(1.0), quad(2.0)
    for k in d1:
        np.testing.assert_allclose(d2[k], 4.0 * d1[k], rtol=1e-9, atol=1e-13)
    assert max(np.abs(v).max() for v in d1.values()) > 1e-6


# ---------------------------------- ring/exchange term (linear in T2)
@pytest.mark.parametrize("somos,n_sv", [((), 0), ((1,), 0), ((1, 3), 0), ((1, 3), 2)])
def test_ring_term_canonical_limit_matches_bruteforce(somos, n_sv):
    # P(IJ) P(AB) sum_KC <KB||CJ> t_IK^AC from explicit antisymmetrised
    # integrals, against the pair form: per target block four oriented
    # contractions S_pq op(T_q) X / J over the couplings that share an index
    rng = np.random.default_rng(71 + len(somos) + 10 * n_sv)
    inp = make_inputs(rng, n_occ=5, somos=somos, npno=4 + n_sv, naux=6, shared_space=True, hole=0.05,
                      ring=0.05)
    if n_sv:
        inp.n_sv = [n_sv] * len(inp.pairs)
    T = random_T(rng, inp, scale=0.05)
    if n_sv:
        T = _mask_T(inp, T)
    R = oracle.residual_os(inp, T)
    Tb = {(inp.pairs[p], name): v for (p, name), v in T.items()}
    Kp = {inp.pairs[p]: inp.K[p] for p in range(len(inp.pairs))}
    args = (inp.n_occ, inp.is_somo, inp.B(0), Kp, inp.eps_a[0], inp.eps_b[0], inp.f_a, inp.f_b, Tb, inp.pairs)
    Rbf, _ = oracle.residual_spinorbital(*args, g_occ=inp.g_occ, n_sv=n_sv, g_ovvo=inp.g_ovvo, g_oovv=inp.g_oovv)
    Rno, _ = oracle.residual_spinorbital(*args, g_occ=inp.g_occ, n_sv=n_sv)
    big = 0.0
    for (p, name), r in R.items():
        np.testing.assert_allclose(r, Rbf[(inp.pairs[p], name)], rtol=0, atol=1e-13)
        big = max(big, np.abs(Rbf[(inp.pairs[p], name)] - Rno[(inp.pairs[p], name)]).max())
    assert big > 1e-3            # the ring term is far above the tolerance
    # every spin case of the ring term is exercised: opposite-spin blocks
    # read same-spin sources and the reverse
    names = {name for (_, name) in R}
    assert {"AA", "AB"} <= names


def test_ring_term_is_linear_and_separate():
    # truncated PNO spaces: the ring term is linear in T, vanishes with its
    # integrals, and adds to the rest of the residual
    rng = np.random.default_rng(73)
    inp = make_inputs(rng, n_occ=6, somos=(2,), npno=[5, 6, 4, 5, 6, 4, 5, 6, 4, 5, 6, 4, 5, 6, 4, 5, 6, 4, 5,
                                                      6, 4], naux=5, ring=0.05)
    T = random_T(rng, inp, scale=0.1)
    base = ("driver", "fock", "projection", "ladder", "hole")
    Rf = oracle.residual_os(inp, T)
    Rb = oracle.residual_os(inp, T, terms=base)
    T2 = {k: 2.0 * v for k, v in T.items()}
    Rf2 = oracle.residual_os(inp, T2)
    Rb2 = oracle.residual_os(inp, T2, terms=base)
    for k in Rf:
        d1, d2 = Rf[k] - Rb[k], Rf2[k] - Rb2[k]
        np.testing.assert_allclose(d2, 2.0 * d1, rtol=1e-12, atol=1e-15)
    assert max(np.abs(Rf[k] - Rb[k]).max() for k in Rf) > 1e-4


# --------------- quadratic part of the occupied Fock intermediate F_MJ
@pytest.mark.parametrize("somos,n_sv", [((), 0), ((1,), 0), ((1, 3), 0), ((1, 3), 2)])
def test_occupied_intermediate_canonical_limit_matches_bruteforce(somos, n_sv):
    # -P(IJ) sum_M t_IM^AB F_MJ with F_MJ = 1/2 sum_NEF t_JN^EF <MN||EF> from
    # explicit antisymmetrised integrals, against the pair form: the occupied
    # Fock weights f_kj dressed by F^s_kj, the pair itself included (m = i, j)
    rng = np.random.default_rng(81 + len(somos) + 10 * n_sv)
    inp = make_inputs(rng, n_occ=5, somos=somos, npno=4 + n_sv, naux=6, shared_space=True)
    if n_sv:
        inp.n_sv = [n_sv] * len(inp.pairs)
    inp.quadratic_occ = True
    T = random_T(rng, inp, scale=0.2)
    if n_sv:
        T = _mask_T(inp, T)
    R = oracle.residual_os(inp, T)
    Tb = {(inp.pairs[p], name): v for (p, name), v in T.items()}
    Kp = {inp.pairs[p]: inp.K[p] for p in range(len(inp.pairs))}
    args = (inp.n_occ, inp.is_somo, inp.B(0), Kp, inp.eps_a[0], inp.eps_b[0], inp.f_a, inp.f_b, Tb, inp.pairs)
    Rbf, _ = oracle.residual_spinorbital(*args, n_sv=n_sv, quadratic_occ=True)
    Rlin, _ = oracle.residual_spinorbital(*args, n_sv=n_sv)
    big = 0.0
    for (p, name), r in R.items():
        np.testing.assert_allclose(r, Rbf[(inp.pairs[p], name)], rtol=0, atol=1e-13)
        big = max(big, np.abs(Rbf[(inp.pairs[p], name)] - Rlin[(inp.pairs[p], name)]).max())
    assert big > 1e-4


def test_occupied_intermediate_is_quadratic_and_uses_the_diagonal():
    # the term scales as T^2; F^s_jj (m = j) contributes
    rng = np.random.default_rng(83)
    inp = make_inputs(rng, n_occ=6, somos=(2,), npno=[6] * 21, naux=5)
    T = random_T(rng, inp, scale=0.1)
    lin = ("driver", "fock", "projection", "ladder")

    def quad(x):
        Tx = {k: x * v for k, v in T.items()}
        inp.quadratic_occ = True
        Rq = oracle.residual_os(inp, Tx)
        inp.quadratic_occ = False
        Rl = oracle.residual_os(inp, Tx, terms=lin)
        return {k: Rq[k] - Rl[k] for k in Rq}
    d1, d2 = quad(1.0), quad(2.0)
    for k in d1:
        np.testing.assert_allclose(d2[k], 4.0 * d1[k], rtol=1e-9, atol=1e-13)
    assert max(np.abs(v).max() for v in d1.values()) > 1e-6
    assert abs(oracle.occ_intermediate(inp, T, 0, 0, 0)) > 0.0


@pytest.mark.parametrize("somos", [(), (1, 3)])
def test_all_further_terms_together_match_bruteforce(somos):
    # hole-hole ladder, its quadratic term, ring/exchange term and the
    # occupied intermediate at once: the pair form and the spin-orbital brute
    # force agree, so no term double-counts another
    rng = np.random.default_rng(91 + len(somos))
    inp = make_inputs(rng, n_occ=5, somos=somos, npno=4, naux=6, shared_space=True, hole=0.05, ring=0.05)
    inp.quadratic = True
    inp.quadratic_occ = True
    T = random_T(rng, inp, scale=0.1)
    R = oracle.residual_os(inp, T)
    Tb = {(inp.pairs[p], name): v for (p, name), v in T.items()}
    Kp = {inp.pairs[p]: inp.K[p] for p in range(len(inp.pairs))}
    Rbf, _ = oracle.residual_spinorbital(inp.n_occ, inp.is_somo, inp.B(0), Kp, inp.eps_a[0], inp.eps_b[0],
                                         inp.f_a, inp.f_b, Tb, inp.pairs, g_occ=inp.g_occ, quadratic=True,
                                         g_ovvo=inp.g_ovvo, g_oovv=inp.g_oovv, quadratic_occ=True)
    for (p, name), r in R.items():
        np.testing.assert_allclose(r, Rbf[(inp.pairs[p], name)], rtol=0, atol=1e-13)
