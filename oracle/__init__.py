"""Plain FP64 CPU oracle for the open-shell DLPNO-CCSD doubles residual.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP library: it re-derives the spin
block rules, reads the same descriptors and regenerates inputs from the seeded
workload generator.

The paper (Sec. II.B.3) states that the CC residual equations are solved in
the truncated PNO basis of every retained pair, without printing them.  The
residual modelled here is the part of the spin-orbital CCSD doubles residual
that the hot path evaluates, restricted to each pair's PNO space:

  R^{ss'}_p = K^{ss'}_p + (eps^s + eps^s' - f^s_ii - f^s'_jj) o T^{ss'}_p
            - sum_{k in occ_s,  k != i} f^s_ki  S_{p,kj} T^{ss'}_{kj} S_{kj,p}
            - sum_{k in occ_s', k != j} f^s'_kj S_{p,ik} T^{ss'}_{ik} S_{ik,p}
            + sum_Q B^Q_p T^{ss'}_p (B^Q_p)^T

with K^{AA} = K^{BB} = K - K^T (antisymmetrised <ab||ij>), K^{AB} = K^{BA} = K,
T_{(k,l)} for k > l taken as the transposed, spin-swapped block of (l,k), a
Jacobi update T' = T - R / D and pair energies w <K^{ss'}, T'> (w = 1/2 for
same spin, 1 for opposite spin).  Every reading of the paper that this needed
is listed in the design notes of the repository.

Parity status per function (what pins it, see tests/test_oracle_*.py):
  residual_os        closed-shell reduction, brute-force spin-orbital
                     contraction (canonical limit), orbital relabelling,
                     self-adjointness, MP2 and ladder closed forms
  residual_cs        worked closed-shell energy identity and MP2 closed form
  residual_spinorbital  textbook spin-orbital CCSD terms built from explicit
                     <ab||cd> on tiny inputs (itself the pin)
  jacobi/energies    MP2 closed form, dense linear solve (LAPACK)
  diis               converges to the dense-solve fixed point
  vjp                finite differences (exact for this bilinear Lagrangian)
                     and the dot-product (adjoint) identity
  f12.f12_energy     spin-adapted prefactors from the cusp amplitudes on
                     explicit spin functions, rank-one closed forms of the two
                     contractions, enumeration of the spin-orbital pairs
"""
from .model import (Inputs, OccInts, stored_blocks, residual_os, residual_cs, jacobi,  # noqa: F401
                    pair_energies, pair_energies_cs, denominators, t_lookup, hole_terms,
                    quadratic_weight, RingInts, ring_block,
                    occ_intermediate, occ_quadratic_block)
from .spinorbital import residual_spinorbital  # noqa: F401
from .solver import DIIS, solve, dense_solution, apply_operator  # noqa: F401
from .adjoint import vjp  # noqa: F401
from . import f12  # noqa: F401
