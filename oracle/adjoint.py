"""Vector-Jacobian product of the residual (FP64 oracle).

TEST INFRASTRUCTURE ONLY.

For Gbar = dL/dR the residual's transpose map gives
  dT_p   = D o Gbar_p + sum_Q (B^Q)^T Gbar_p B^Q
           + scatter of -w S_pq^T Gbar_p S_pq to every source block read by p
             (projection, w = f) and of +w S_pq^T Gbar_p S_pq (hole-hole
             ladder, w = (k i | l j))
  dB^Q_p = sum_blocks ( Gbar B^Q T^T + Gbar^T B^Q T )
(the last is the gradient for a general, unsymmetrised B, since the ladder is
R = sum_Q B^Q T B^Q^T).  The oracle scatters; no symmetry of the operator is
assumed.
"""
import numpy as np

from .model import denominators, projection_terms, hole_terms


def vjp(inp, T, G):
    if (getattr(inp, "quadratic", False) or getattr(inp, "n_sv", None) is not None
            or getattr(inp, "ring", None) is not None):
        raise NotImplementedError("vjp covers the residual without the quadratic and ring terms on unmasked "
                                  "spaces only")
    dT = {k: np.zeros_like(v) for k, v in T.items()}
    dB = {}
    for p in range(len(inp.pairs)):
        names = inp.blocks(p)
        if not names:
            continue
        Bp = inp.B(p)
        m, n, _ = Bp.shape
        dBp = np.zeros_like(Bp)
        for name in names:
            g = G[(p, name)]
            dT[(p, name)] += denominators(inp, p, name) * g
            # sum_Q B^T g B  via the combined (Q, a) index
            Y = (Bp.transpose(0, 2, 1).reshape(m * n, n) @ g).reshape(m, n, n)   # Y[Q,c,b] = sum_a B[Q,a,c] g[a,b]
            dT[(p, name)] += Y.transpose(1, 0, 2).reshape(n, m * n) @ Bp.reshape(m * n, n)
            Tb = T[(p, name)]
            dBp += np.einsum("ab,qbd,cd->qac", g, Bp, Tb, optimize=True)       # g B T^T
            dBp += np.einsum("ba,qbd,dc->qac", g, Bp, Tb, optimize=True)       # g^T B T
            for w, q, Spq, src in projection_terms(inp, T, p, name):
                contrib = -w * (Spq.T @ g @ Spq)
                dT[(src[0], src[1])] += contrib.T if src[2] else contrib
            for w, q, Spq, src in hole_terms(inp, T, p, name):
                contrib = w * (Spq.T @ g @ Spq)
                dT[(src[0], src[1])] += contrib.T if src[2] else contrib
        dB[p] = dBp
    return dT, dB
