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
