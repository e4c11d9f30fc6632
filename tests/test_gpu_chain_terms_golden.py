"""The chain workload at its stated size (160 occupied, 3,150 pairs) with every
further CCSD term of the library on (hole-hole ladder, its quadratic term,
ring/exchange term, quadratic part of the occupied Fock intermediate): 8 FP64
iterations with DIIS from T = 0 on the GPU against the FP64 oracle's
iterations stored in tests/golden/chain_terms_fp64_iterations.txt (written by
tests/golden/make_chain_terms_golden.py, oracle only): the energy and max|R|
of every iteration and the energy of every pair block after the last."""
import os

import pytest

from tests.gpu_helpers import device_problem
from workload import build_problem

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "chain_terms_fp64_iterations.txt")
OPTIONS = dict(hole_ladder=0.02, quadratic=True, ring=0.05, quadratic_occ=True)
N_ITER = 8


def read_golden():
    its, blks = [], []
    for line in open(GOLDEN):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "it":
            its.append((int(f[1]), float(f[2]), float(f[3])))
        elif f[0] == "blk":
            blks.append((int(f[1]), int(f[2]), float(f[3])))
    return its, blks


def test_golden_file_is_consistent():
    """CPU: the stored block energies cover the workload's stored blocks and
    add up to the last iteration's total."""
    its, blks = read_golden()
    prob = build_problem("chain", **OPTIONS)
    assert len(its) == N_ITER and len(blks) == int(prob.n_blocks().sum())
    assert abs(sum(e for _, _, e in blks) - its[-1][1]) <= 1e-12


@pytest.mark.gpu
def test_chain_with_all_terms_matches_the_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    its, blks = read_golden()
    prob = build_problem("chain", **OPTIONS)
    print("case chain with all terms", prob.n_pairs, "pairs,", prob.n_hh, "hole-hole,", prob.n_ring, "ring couplings,",
          N_ITER, "iterations", flush=True)
    plan, dev = device_problem(prob, T_random=False, quadratic=True, quadratic_occ=True)
    _, e_pair, e_tot, rmax = plan.iterate(N_ITER, dev["T"])
    E, Rm = plan.history()
    assert len(E) == N_ITER
    for (k, e_o, r_o), e_g, r_g in zip(its, E, Rm):
        assert abs(e_g - e_o) <= 1e-10, (k, e_g, e_o)
        assert abs(r_g - r_o) <= 1e-8 * r_o + 1e-13, (k, r_g, r_o)
    ep = e_pair.cpu().numpy().reshape(-1, 4)
    worst = max(abs(ep[p, c] - e) for p, c, e in blks)
    print("worst pair-block energy difference %.3e Eh" % worst, flush=True)
    assert worst <= 1e-10
    plan.close()
