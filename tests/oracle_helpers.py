"""Hand-built oracle inputs for the pin tests (CPU only)."""
import numpy as np

import oracle
from oracle.model import stored_blocks


def orthonormal(rng, dim, n):
    q, r = np.linalg.qr(rng.standard_normal((dim, n)))
    return q * np.sign(np.diag(r))[None, :]


def random_T(rng, inp, scale=1e-2, sym_diag=False):
    T = {}
    for p, (i, j) in enumerate(inp.pairs):
        n = inp.npno(p)
        for name in inp.blocks(p):
            g = scale * rng.standard_normal((n, n))
            if name in ("AA", "BB"):
                g = (g - g.T) / np.sqrt(2.0)
            elif i == j and sym_diag:
                g = (g + g.T) / 2.0
            T[(p, name)] = g
    return T


def occ_integrals(rng, n, scale):
    """Random real occupied integrals g[k, i, l, j] = (k i | l j) with the
    eightfold permutational symmetry of real two-electron integrals."""
    g = rng.standard_normal((n, n, n, n))
    g = g + g.transpose(1, 0, 2, 3)
    g = g + g.transpose(0, 1, 3, 2)
    g = g + g.transpose(2, 3, 0, 1)
    return scale * g / 8.0


def ring_dense(rng, n_occ, V, scale):
    """Random real integrals of the ring term, (k c | b j) as g_ovvo[k, c, b, j]
    and (k j | b c) as g_oovv[k, j, b, c], with the permutational symmetries
    of real two-electron integrals."""
    a = rng.standard_normal((n_occ, V, V, n_occ))
    a = (a + a.transpose(3, 2, 1, 0)) / 2.0            # (kc|bj) = (jb|ck)
    b = rng.standard_normal((n_occ, n_occ, V, V))
    b = (b + b.transpose(1, 0, 2, 3)) / 2.0            # (kj|bc) = (jk|bc)
    b = (b + b.transpose(0, 1, 3, 2)) / 2.0            # (kj|bc) = (kj|cb)
    return scale * a, scale * b


def ring_couplings(inp, make):
    """RingInts over every retained source {x, m}: make(p, role, m, q, x, y)
    returns the (X, J) matrices of one coupling."""
    table = {}
    for p, (i, j) in enumerate(inp.pairs):
        rows = []
        for role, (x, y) in enumerate(((i, j), (j, i))):
            if role == 1 and i == j:
                continue
            for m in range(inp.n_occ):
                q = inp.index.get((min(x, m), max(x, m)))
                if q is None:
                    continue
                X, J = make(p, role, m, q, x, y)
                rows.append((role, m, q, X, J))
        table[p] = rows
    return oracle.RingInts(table)


def make_inputs(rng, n_occ, somos, npno, naux, band=None, dim=None, shared_space=False,
                b_scale=0.1, k_scale=0.05, f_off=0.05, canonical=False, hole=0.0, ring=0.0):
    """Random model instance.  shared_space: all pairs use one untruncated
    virtual space (identity overlaps, one B, one eps): the canonical limit.
    hole: scale of random occupied integrals (k i | l j) of the hole-hole
    ladder (0: no such term); they are kept in inp.g_occ as a dense array.
    ring: scale of the ring term's integrals (0: no such term); in the shared
    space they come from dense arrays inp.g_ovvo, inp.g_oovv, otherwise each
    coupling gets its own random X and J."""
    is_somo = np.zeros(n_occ, dtype=bool)
    is_somo[list(somos)] = True
    band = n_occ if band is None else band
    pairs = [(i, j) for i in range(n_occ) for j in range(i, min(n_occ, i + band + 1))]
    P = len(pairs)
    f = np.diag(rng.uniform(-1.2, -0.3, n_occ))
    for i in range(n_occ):
        for k in range(i + 1, n_occ):
            if k - i <= band:
                f[i, k] = f[k, i] = f_off * rng.standard_normal()
    fb = f.copy()
    # spin-dependent off-diagonal occupied Fock (UHF-like) so that a term taking
    # the wrong spin's Fock matrix is visible
    off = np.triu(rng.standard_normal((n_occ, n_occ)), 1) * f_off * 0.3
    off = off + off.T
    if somos:
        fb = fb + np.where(f != 0.0, off, 0.0) * (1 - np.eye(n_occ))
    for s in somos:
        fb[np.arange(n_occ), np.arange(n_occ)] += 0.05 * np.exp(-np.abs(np.arange(n_occ) - s) / 2.0)
    if shared_space:
        V = npno
        Bg = rng.standard_normal((naux, V, V)) * b_scale
        Bg = (Bg + Bg.transpose(0, 2, 1)) / 2.0
        ea = rng.uniform(0.2, 3.0, V)
        eb = ea + (0.03 if somos else 0.0)
        B = {p: Bg for p in range(P)}
        eps_a = {p: ea.copy() for p in range(P)}
        eps_b = {p: eb.copy() for p in range(P)}
        ident = np.eye(V)
        S = lambda p, q: ident
        ns = [V] * P
    else:
        ns = [npno if np.isscalar(npno) else npno[p] for p in range(P)]
        B, eps_a, eps_b = {}, {}, {}
        for p in range(P):
            b = rng.standard_normal((naux, ns[p], ns[p])) * b_scale
            B[p] = (b + b.transpose(0, 2, 1)) / 2.0
            eps_a[p] = rng.uniform(0.2, 3.0, ns[p])
            eps_b[p] = eps_a[p] + (0.03 if somos else 0.0)
        dim = dim or 3 * max(ns)
        Q = [orthonormal(rng, dim, ns[p]) for p in range(P)]
        S = lambda p, q: Q[p].T @ Q[q]
    K = {}
    for p, (i, j) in enumerate(pairs):
        k = k_scale * rng.standard_normal((ns[p], ns[p]))
        K[p] = (k + k.T) / 2.0 if i == j else k
    g = occ_integrals(rng, n_occ, hole) if hole else None
    inp = oracle.Inputs(n_occ, is_somo, pairs, B, K, eps_a, eps_b, f, fb, S,
                        oracle.OccInts(g) if g is not None else None)
    inp.g_occ = g
    inp.g_ovvo = inp.g_oovv = None
    if ring and shared_space:
        inp.g_ovvo, inp.g_oovv = ring_dense(rng, n_occ, npno, ring)
        inp.ring = ring_couplings(inp, lambda p, role, m, q, x, y: (inp.g_ovvo[m, :, :, y].copy(),
                                                                     inp.g_oovv[m, y].T.copy()))
    elif ring:
        inp.ring = ring_couplings(inp, lambda p, role, m, q, x, y: (
            ring * rng.standard_normal((ns[q], ns[p])), ring * rng.standard_normal((ns[q], ns[p]))))
    return inp


def inner(X, Y):
    return sum(float(np.sum(X[k] * Y[k])) for k in X)
