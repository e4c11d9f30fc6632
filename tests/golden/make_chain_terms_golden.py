"""Writes chain_terms_fp64_iterations.txt: the FP64 oracle's 8 Jacobi + DIIS
iterations on the full 160-orbital chain workload (3,150 pairs, |i - j| <= 20,
SOMOs 53 and 106, seed 2) with every further CCSD term of the library on:
the hole-hole ladder (occupied integrals of scale 0.02 within two orbitals),
the quadratic term on its couplings, the ring/exchange term (integral blocks
of scale 0.05, replacing orbitals within two of the shared index) and the
quadratic part of the occupied Fock intermediate; from T = 0, DIIS keeping 8
vectors and extrapolating from 3.

Per iteration it records the total energy of the updated amplitudes T' and
max |R|; after the last iteration, the energy of every stored pair block.
Only the oracle and the seeded input generator are used.

    python tests/golden/make_chain_terms_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle.model import unpack_T  # noqa: E402
from workload import build_problem  # noqa: E402

N_ITER = 8
CODE = {"AA": 0, "BB": 1, "AB": 2, "BA": 3}
OPTIONS = dict(hole_ladder=0.02, quadratic=True, ring=0.05, quadratic_occ=True)


def main(out=os.path.join(HERE, "chain_terms_fp64_iterations.txt")):
    prob = build_problem("chain", **OPTIONS)
    inp = oracle.Inputs.from_problem(prob)
    zero = unpack_T(prob, np.zeros(prob.n_T))
    last = {}
    t0 = time.time()
    _, hist = oracle.solve(inp, zero, N_ITER, use_diis=True, last=last)
    e = last["pair_energies"]
    with open(out, "w") as f:
        f.write("# FP64 oracle, workload 'chain' (160 occupied, SOMOs 53 and 106, |i-j| <= 20, seed 2) with %s:\n"
                % ", ".join("%s=%s" % kv for kv in OPTIONS.items()))
        f.write("# %d Jacobi iterations with DIIS (8 vectors, extrapolation from 3) from T = 0.\n" % N_ITER)
        f.write("# Written by tests/golden/make_chain_terms_golden.py (oracle only) in %.0f s.\n" % (time.time() - t0))
        f.write("# iteration lines: it <k> <total energy of T'> <max |R|>\n")
        f.write("# block lines: blk <pair> <block code 0 AA 1 BB 2 AB 3 BA> <energy of T' after the last iteration>\n")
        for k, (E, rm) in enumerate(hist):
            f.write("it %d %.17e %.17e\n" % (k, E, rm))
        for (p, name) in sorted(e, key=lambda x: (x[0], CODE[x[1]])):
            f.write("blk %d %d %.17e\n" % (p, CODE[name], e[(p, name)]))
    print("wrote", out, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
