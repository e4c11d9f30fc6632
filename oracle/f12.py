"""Second-order F12 correction evaluated with the converged doubles amplitudes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper writes the correction as a sum over occupied pairs of 2 V~ + B~
(Sec. II.A, Eq. "F12 energy"), with V~ the geminal diagonal dressed by the
amplitudes (Eq. "Vtilde"):

    V~^{ij}_{ij} = V^{ij}_{ij} + 1/2 (V + C)^{ij}_{ab} t^{ab}_{ij}   (+ singles)

and then spin-adapts it (the equations that follow Eq. "F12 energy"):

    same spin        eps = 1/2 V~ + 1/16 B~
    opposite spin    eps = 3/4 V~ + 1/4 V~x + 9/64 B~1 + 3/64 B~2 + 3/64 B~3 + 1/64 B~4

where V~x is the element with the geminal's two orbitals exchanged.  Here, per
stored spin block of a pair (its own electron order):
  W      = (V + C)^{ij}_{ab} over the pair's PNOs, an n x n matrix;
  V, V'  = V^{ij}_{ij} and the exchanged V^{ji}_{ij} (opposite spin only);
  B1..B4 = B~ with direct/exchanged geminals on each side (same spin: B1).
V and C are unchanged when both electrons are relabelled, so the exchanged
geminal contracts W^T:  V~x = V' + 1/2 sum_ab W_ba T_ab.  The singles terms of
Eq. "Vtilde" are absent: the model has no T1.  Every stored block is one term
of the spin-adapted sums (AA: I<J, BB: I~<J~, AB and BA: the (I, J~) terms).

Parity status: the spin-adapted prefactors are pinned against the cusp
amplitudes 1/2 (singlet) and 1/4 (triplet) of the geminal (Eq.
"ExpCorrWfnRspin") applied to explicit two-electron spin functions; the two
contractions against rank-one closed forms; the block sum against an
enumeration of the spin-orbital pairs.
"""
import numpy as np

from .model import SPIN, stored_blocks, unpack_T

SAME_SPIN = (1.0 / 2.0, 1.0 / 16.0)
OPPOSITE_SPIN = (3.0 / 4.0, 1.0 / 4.0, 9.0 / 64.0, 3.0 / 64.0, 3.0 / 64.0, 1.0 / 64.0)


def vtilde(Wb, Tb, v, vx):
    """Direct and exchanged V~ of one block (Eq. "Vtilde" without singles)."""
    direct = v + 0.5 * float(np.sum(Wb * Tb))
    exchanged = vx + 0.5 * float(np.sum(Wb.T * Tb))
    return direct, exchanged


def block_energy(name, Wb, Tb, scal):
    """Spin-adapted F12 pair energy of one stored block; scal = (V, V', B1..B4)."""
    v, vx, b1, b2, b3, b4 = (float(x) for x in scal)
    vt, vtx = vtilde(Wb, Tb, v, vx)
    s1, s2 = SPIN[name]
    if s1 == s2:
        a, b = SAME_SPIN
        return a * vt + b * b1
    c = OPPOSITE_SPIN
    return c[0] * vt + c[1] * vtx + c[2] * b1 + c[3] * b2 + c[4] * b3 + c[5] * b4


def f12_energy(prob, T_flat, W_flat, scalars):
    """Per-block energies {(p, name): eps}, pair energies [P, 4] (AA, BB, AB,
    BA) and the total.  scalars: [n_blocks, 6] in block order."""
    T = unpack_T(prob, T_flat)
    W = unpack_T(prob, W_flat)
    somo = prob.is_somo.astype(bool)
    eps = {}
    e_pair = np.zeros((prob.n_pairs, 4))
    g = 0
    for p in range(prob.n_pairs):
        for name in stored_blocks(int(prob.pi[p]), int(prob.pj[p]), somo):
            e = block_energy(name, W[(p, name)], T[(p, name)], scalars[g])
            eps[(p, name)] = e
            e_pair[p, ("AA", "BB", "AB", "BA").index(name)] = e
            g += 1
    total = float(sum(eps[k] for k in sorted(eps)))
    return eps, e_pair, total
