"""Jacobi iterations with DIIS, and the dense linear solution of the model.

TEST INFRASTRUCTURE ONLY.
"""
import numpy as np

from .model import residual_os, jacobi, pair_energies


def keys_of(inp):
    return [(p, name) for p in range(len(inp.pairs)) for name in inp.blocks(p)]


def flatten(T, keys):
    return np.concatenate([T[k].ravel() for k in keys]) if keys else np.zeros(0)


def unflatten(v, keys, inp):
    out, o = {}, 0
    for (p, name) in keys:
        n = inp.npno(p)
        out[(p, name)] = v[o:o + n * n].reshape(n, n).copy()
        o += n * n
    return out


def apply_operator(inp, T):
    """The linear part (D + A)(T) of the residual: everything but the driver."""
    return residual_os(inp, T, terms=("fock", "projection", "ladder", "hole", "ring"))


class DIIS:
    """Pulay extrapolation of amplitude vectors.

    Keeps at most `max_vec` (vector, error) pairs, extrapolates once `start`
    are stored by solving [[G, -1], [-1, 0]] [c; -lambda] = [0; -1] with
    G = <e_i, e_j> / max_k <e_k, e_k> and, if that matrix is ill conditioned
    (cond > 1e14), drops the oldest.  Normalising G leaves c unchanged and
    makes the test one of near linear dependence of the error vectors: without
    it the condition number grows like 1 / |e|^2 as the iteration converges
    and the whole history would be dropped once |e| ~ 1e-7."""

    def __init__(self, max_vec=8, start=3):
        self.max_vec, self.start = max_vec, start
        self.vecs, self.errs = [], []
        self.drops = 0          # vectors dropped for ill conditioning (bookkeeping)

    def push(self, vec, err):
        self.vecs.append(vec.copy())
        self.errs.append(err.copy())
        if len(self.vecs) > self.max_vec:
            self.vecs.pop(0)
            self.errs.pop(0)

    def coefficients(self):
        while True:
            n = len(self.errs)
            M = np.zeros((n + 1, n + 1))
            for a in range(n):
                for b in range(n):
                    M[a, b] = float(np.dot(self.errs[a], self.errs[b]))
            scale = max(M[a, a] for a in range(n)) if n > 0 else 0.0
            if scale > 0.0:
                M[:n, :n] /= scale
            M[n, :n] = M[:n, n] = -1.0
            rhs = np.zeros(n + 1)
            rhs[n] = -1.0
            if n > 1 and np.linalg.cond(M) > 1e14:
                self.vecs.pop(0)
                self.errs.pop(0)
                self.drops += 1
                continue
            return np.linalg.solve(M, rhs)[:n]

    def extrapolate(self):
        if len(self.vecs) < self.start:
            return self.vecs[-1].copy()
        c = self.coefficients()
        return sum(ci * v for ci, v in zip(c, self.vecs))


def solve(inp, T0, n_iter, use_diis=True, tol_r=None, tol_e=None, trace=None, last=None):
    """Iterate R(T), T' = T - R/D, energies of T', then DIIS on (T', T' - T).

    Returns (T, history) with history entries (E, max|R|).  trace: optional
    list that receives, per iteration, (stored vectors, drops so far,
    extrapolation coefficients oldest -> newest or None before the start).
    last: optional dict that receives the pair-block energies of the last
    iteration's T' under "pair_energies"."""
    keys = keys_of(inp)
    T = {k: T0[k].copy() for k in keys}
    diis = DIIS() if use_diis else None
    hist = []
    E_old = None
    for _ in range(n_iter):
        R = residual_os(inp, T)
        Tn = jacobi(inp, T, R)
        e_blocks = pair_energies(inp, Tn)
        E = sum(e_blocks.values())
        if last is not None:
            last["pair_energies"] = e_blocks
        rmax = max(float(np.max(np.abs(r))) for r in R.values()) if R else 0.0
        hist.append((E, rmax))
        if diis is not None:
            vn, v = flatten(Tn, keys), flatten(T, keys)
            diis.push(vn, vn - v)
            T = unflatten(diis.extrapolate(), keys, inp)
            if trace is not None:
                c = diis.coefficients() if len(diis.vecs) >= diis.start else None
                trace.append((len(diis.vecs), diis.drops, c))
        else:
            T = Tn
        if tol_r is not None and rmax < tol_r and E_old is not None and abs(E - E_old) < tol_e:
            break
        E_old = E
    return T, hist


def dense_solution(inp):
    """Solve (D + A) t = -K directly: A assembled column by column from unit
    amplitudes, then a dense LAPACK solve."""
    keys = keys_of(inp)
    sizes = [inp.npno(p) ** 2 for p, _ in keys]
    N = sum(sizes)
    zero = {(p, name): np.zeros((inp.npno(p), inp.npno(p))) for p, name in keys}
    drv = flatten(residual_os(inp, zero, terms=("driver",)), keys)
    A = np.zeros((N, N))
    for col in range(N):
        e = np.zeros(N)
        e[col] = 1.0
        A[:, col] = flatten(apply_operator(inp, unflatten(e, keys, inp)), keys)
    return unflatten(np.linalg.solve(A, -drv), keys, inp), A
