"""Pins of the F12-correction oracle (CPU).

The spin-adapted prefactors are re-derived here from the geminal's cusp
amplitudes, 1/2 on the singlet and 1/4 on the triplet projector (Sec. II.A,
Eq. "ExpCorrWfnRspin"), applied to explicit two-electron spin functions; the
two contractions of Eq. "Vtilde" are checked on rank-one inputs with closed
forms; and the block sum against an enumeration of the spin-orbital pairs.
"""
import numpy as np
import pytest

from oracle import f12
from oracle.model import SPIN, stored_blocks
from workload import build_problem

# two-electron spin space, basis a(1)a(2), a(1)b(2), b(1)a(2), b(1)b(2)
AA, AB, BA, BB = np.eye(4)


def cusp_operator():
    singlet = (AB - BA) / np.sqrt(2.0)
    triplet0 = (AB + BA) / np.sqrt(2.0)
    P0 = np.outer(singlet, singlet)
    P1 = np.outer(AA, AA) + np.outer(triplet0, triplet0) + np.outer(BB, BB)
    return 0.5 * P0 + 0.25 * P1


def amplitudes(name):
    """Geminal amplitudes of the direct and exchanged spatial geminal for a
    block whose electrons carry spins SPIN[name].  The operator maps the spin
    function s1(1) s2(2) onto c_d s1(1) s2(2) + c' s2(1) s1(2); the second term
    belongs to the exchanged spatial geminal with the sign of the swap."""
    e = {(0, 0): AA, (0, 1): AB, (1, 0): BA, (1, 1): BB}
    s1, s2 = SPIN[name]
    G = cusp_operator()
    direct = e[(s1, s2)]
    c_d = float(direct @ G @ direct)
    if s1 == s2:
        # the swapped spin function is the direct one: the antisymmetrised
        # same-spin geminal has the single amplitude c_d
        assert float(np.abs(G @ direct - c_d * direct).max()) < 1e-15
        return c_d, None
    swapped = e[(s2, s1)]
    c_x = -float(swapped @ G @ direct)
    return c_d, c_x


def energy_from_amplitudes(name, vt, vtx, b):
    """2 sum_g c_g V~_g + sum_{g,g'} c_g c_g' B~_{g,g'} (Eq. "F12 energy")."""
    c_d, c_x = amplitudes(name)
    if c_x is None:
        return 2.0 * c_d * vt + c_d * c_d * b[0]
    return (2.0 * (c_d * vt + c_x * vtx)
            + c_d * c_d * b[0] + c_d * c_x * b[1] + c_x * c_d * b[2] + c_x * c_x * b[3])


@pytest.mark.parametrize("name", ["AA", "BB", "AB", "BA"])
def test_prefactors_follow_from_the_cusp_amplitudes(name):
    rng = np.random.default_rng(7)
    n = 5
    W = np.zeros((n, n))                     # V~ = V: only the prefactors act
    T = rng.standard_normal((n, n))
    scal = rng.standard_normal(6)
    got = f12.block_energy(name, W, T, scal)
    want = energy_from_amplitudes(name, scal[0], scal[1], scal[2:])
    assert abs(got - want) <= 1e-15 * max(1.0, abs(want))


def test_cusp_amplitudes_are_the_known_ones():
    assert amplitudes("AA")[0] == pytest.approx(0.25) and amplitudes("AA")[1] is None
    assert amplitudes("BB")[0] == pytest.approx(0.25)
    assert amplitudes("AB") == pytest.approx((0.375, 0.125))
    assert amplitudes("BA") == pytest.approx((0.375, 0.125))


def test_contractions_rank_one_closed_forms():
    rng = np.random.default_rng(3)
    n = 7
    u, v, x, y = (rng.standard_normal(n) for _ in range(4))
    W = np.outer(u, v)
    T = np.outer(x, y)
    vt, vtx = f12.vtilde(W, T, 0.3, -0.2)
    assert vt == pytest.approx(0.3 + 0.5 * (u @ x) * (v @ y), rel=1e-13)
    assert vtx == pytest.approx(-0.2 + 0.5 * (v @ x) * (u @ y), rel=1e-13)


@pytest.mark.parametrize("cfg", ["tiny", "chain_small"])
def test_block_sum_covers_every_spin_orbital_pair_once(cfg):
    prob = (build_problem("tiny") if cfg == "tiny" else
            build_problem("chain", n_occ=12, band=3, somos=(4, 9)))
    somo = prob.is_somo.astype(bool)
    T = prob.materialize("T")
    W = prob.materialize("W")
    scal = prob.f12_scalars()
    eps, e_pair, total = f12.f12_energy(prob, T, W, scal)
    # spin orbitals: alpha for every occupied orbital, beta for the DOMOs
    occ_a = list(range(prob.n_occ))
    occ_b = [i for i in range(prob.n_occ) if not somo[i]]
    retained = {(int(i), int(j)): p for p, (i, j) in enumerate(zip(prob.pi, prob.pj))}
    seen = {}

    def block_of(k, l, s1, s2):
        # spin-orbital pair (k s1, l s2) -> the stored block that holds it
        if k <= l:
            return retained.get((k, l)), {(0, 0): "AA", (1, 1): "BB", (0, 1): "AB", (1, 0): "BA"}[(s1, s2)]
        return retained.get((l, k)), {(0, 0): "AA", (1, 1): "BB", (0, 1): "BA", (1, 0): "AB"}[(s1, s2)]

    terms = ([(i, j, 0, 0) for i in occ_a for j in occ_a if i < j]
             + [(i, j, 1, 1) for i in occ_b for j in occ_b if i < j]
             + [(i, j, 0, 1) for i in occ_a for j in occ_b])
    enum_total = 0.0
    for (k, l, s1, s2) in terms:
        p, name = block_of(k, l, s1, s2)
        if p is None:
            continue                                  # pair not retained
        key = (p, name)
        assert key in eps, (k, l, s1, s2)
        assert key not in seen, (key, seen.get(key), (k, l, s1, s2))
        seen[key] = (k, l, s1, s2)
        enum_total += eps[key]
    assert set(seen) == set(eps)
    assert enum_total == pytest.approx(total, rel=1e-13)
    assert e_pair.sum() == pytest.approx(total, rel=1e-13)
    # the blocks exist exactly where the spin-case rule puts them
    for p in range(prob.n_pairs):
        assert [n for n in ("AA", "BB", "AB", "BA") if (p, n) in eps] == \
            stored_blocks(int(prob.pi[p]), int(prob.pj[p]), somo)
