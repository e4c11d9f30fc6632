"""Brute-force spin-orbital residual for the canonical limit (tiny inputs only).

TEST INFRASTRUCTURE ONLY.

When PNOs are not truncated the pair method must reduce to its canonical
counterpart (Sec. IV.A).  Here every pair shares one V-dimensional virtual
space (all overlaps are identities), and the textbook spin-orbital doubles
terms of the model are formed from explicit antisymmetrised integrals:

  R_IJ^AB = <AB||IJ> + (e_A + e_B) t_IJ^AB - sum_K f_KI t_KJ^AB
            - sum_K f_KJ t_IK^AB + 1/2 sum_CD <AB||CD> t_IJ^CD
            + 1/2 sum_KL <KL||IJ> t_KL^AB
           [+ 1/4 sum_KLCD <KL||CD> t_IJ^CD t_KL^AB]
           [+ P(IJ) P(AB) sum_KC <KB||CJ> t_IK^AC]
           [- P(IJ) sum_M t_IM^AB F_MJ,  F_MJ = 1/2 sum_NEF t_JN^EF <MN||EF>]
  E       = 1/4 sum_IJAB <IJ||AB> t_IJ^AB

with (ac|bd) = sum_Q B^Q_ac B^Q_bd, (ia|jb) given per ordered pair and the
occupied integrals (ki|lj) given as a dense array (the hole-hole term is
absent when they are not given); P(IJ) X_IJ = X_IJ - X_JI.  The ring term
takes <KB||CJ> = (kc|bj) - (kj|bc) from dense arrays g_ovvo[k, c, b, j] =
(k c | b j) and g_oovv[k, j, b, c] = (k j | b c) when they are given.  With n_sv > 0 the last n_sv spatial virtual
functions are SOMOs: beta virtual spin orbitals only (their alpha spin
orbitals are occupied), Sec. II.B.4.
"""
import numpy as np


def _spin_orbitals(n_occ, is_somo, V, n_sv=0):
    occ = [(i, 0) for i in range(n_occ)] + [(i, 1) for i in range(n_occ) if not is_somo[i]]
    vir = [(a, 0) for a in range(V - n_sv)] + [(a, 1) for a in range(V)]
    return occ, vir


def residual_spinorbital(n_occ, is_somo, Bg, Kpair, eps_a, eps_b, f_a, f_b, Tblocks, pairs, g_occ=None, n_sv=0,
                         quadratic=False, g_ovvo=None, g_oovv=None, quadratic_occ=False):
    """Pair blocks of the residual and the total energy of the given amplitudes.

    Bg       (m, V, V) three-index integrals shared by all pairs
    Kpair    {(i, j): V x V} (i a | j b) for i <= j
    Tblocks  {((i, j), name): V x V} stored amplitude blocks (same-spin antisymmetric)
    pairs    list of (i, j) covering every occupied pair (i <= j)
    g_occ    optional (n_occ, n_occ, n_occ, n_occ) array g[k, i, l, j] = (k i | l j)
    n_sv     SOMO functions among the V (the last n_sv; beta virtual only)
    quadratic  add 1/4 sum_KLCD <KL||CD> t_IJ^CD t_KL^AB
    g_ovvo, g_oovv  optional (n_occ, V, V, n_occ) and (n_occ, n_occ, V, V) arrays
             of the ring term (both or neither)
    quadratic_occ  add -P(IJ) sum_M t_IM^AB F_MJ, F_MJ = 1/2 sum_NEF t_JN^EF <MN||EF>
    Returns ({((i, j), name): V x V residual block, zero outside the blocks'
    virtual spaces}, energy of the amplitudes).
    """
    V = Bg.shape[1]
    occ, vir = _spin_orbitals(n_occ, is_somo, V, n_sv)
    no, nv = len(occ), len(vir)
    oidx = {o: x for x, o in enumerate(occ)}
    vidx = {v: x for x, v in enumerate(vir)}
    spins = {"AA": (0, 0), "BB": (1, 1), "AB": (0, 1), "BA": (1, 0)}
    sp_a = np.array([a for a, _ in vir])      # spatial index of each virtual spin orbital
    sp_s = np.array([sa for _, sa in vir])    # its spin

    def Kord(i, j):
        return Kpair[(i, j)] if i <= j else Kpair[(j, i)].T

    # <AB||IJ>
    g_vvoo = np.zeros((nv, nv, no, no))
    for I, (i, si) in enumerate(occ):
        for J, (j, sj) in enumerate(occ):
            for A, (a, sa) in enumerate(vir):
                for B, (b, sb) in enumerate(vir):
                    v = 0.0
                    if sa == si and sb == sj:
                        v += Kord(i, j)[a, b]
                    if sa == sj and sb == si:
                        v -= Kord(j, i)[a, b]
                    g_vvoo[A, B, I, J] = v
    # <AB||CD> = (AC|BD) - (AD|BC), spin orbitals of equal spin in each charge distribution
    acbd = np.einsum("qac,qbd->abcd", Bg, Bg)          # (ac|bd)
    a4 = np.ix_(sp_a, sp_a, sp_a, sp_a)
    s_ = sp_s
    same_ac_bd = (s_[:, None, None, None] == s_[None, None, :, None]) & (s_[None, :, None, None] == s_[None, None, None, :])
    same_ad_bc = (s_[:, None, None, None] == s_[None, None, None, :]) & (s_[None, :, None, None] == s_[None, None, :, None])
    g_vvvv = np.where(same_ac_bd, acbd[a4], 0.0) - np.where(same_ad_bc, acbd.transpose(0, 1, 3, 2)[a4], 0.0)
    # amplitudes as a fully antisymmetric tensor
    t = np.zeros((no, no, nv, nv))
    for ((i, j), name), Tb in Tblocks.items():
        s1, s2 = spins[name]
        I, J = oidx[(i, s1)], oidx[(j, s2)]
        for a in range(V):
            for b in range(V):
                if (a, s1) not in vidx or (b, s2) not in vidx:
                    assert Tb[a, b] == 0.0, "amplitude outside the virtual spaces"
                    continue
                A, B = vidx[(a, s1)], vidx[(b, s2)]
                t[I, J, A, B] = Tb[a, b]
                t[J, I, B, A] = Tb[a, b]
                t[I, J, B, A] = -Tb[a, b]
                t[J, I, A, B] = -Tb[a, b]
    # Fock in spin orbitals
    fo = np.zeros((no, no))
    for K, (k, sk) in enumerate(occ):
        for I, (i, si) in enumerate(occ):
            if sk == si:
                fo[K, I] = (f_a if sk == 0 else f_b)[k, i]
    ev = np.array([(eps_a if sa == 0 else eps_b)[a] for a, sa in vir])
    R = (g_vvoo.transpose(2, 3, 0, 1)
         + (ev[None, None, :, None] + ev[None, None, None, :]) * t
         - np.einsum("ki,kjab->ijab", fo, t)
         - np.einsum("kj,ikab->ijab", fo, t)
         + 0.5 * np.einsum("abcd,ijcd->ijab", g_vvvv, t))
    if g_occ is not None:
        # <KL||IJ> = (KI|LJ) - (KJ|LI), spin orbitals of equal spin in each charge distribution
        g_oooo = np.zeros((no, no, no, no))
        for K, (k, sk) in enumerate(occ):
            for L, (l, sl) in enumerate(occ):
                for I, (i, si) in enumerate(occ):
                    for J, (j, sj) in enumerate(occ):
                        v = 0.0
                        if sk == si and sl == sj:
                            v += g_occ[k, i, l, j]
                        if sk == sj and sl == si:
                            v -= g_occ[k, j, l, i]
                        g_oooo[K, L, I, J] = v
        R = R + 0.5 * np.einsum("klij,klab->ijab", g_oooo, t)
    if quadratic:
        # <KL||CD> = <CD||KL> (real orbitals) = g_vvoo[C, D, K, L]
        R = R + 0.25 * np.einsum("cdkl,ijcd,klab->ijab", g_vvoo, t, t)
    if quadratic_occ:
        # <MN||EF> = <EF||MN> (real orbitals) = g_vvoo[E, F, M, N]
        Fmj = 0.5 * np.einsum("jnef,efmn->mj", t, g_vvoo)
        X = np.einsum("imab,mj->ijab", t, Fmj)
        R = R - (X - X.transpose(1, 0, 2, 3))
    if g_ovvo is not None:
        # <KB||CJ> = <KB|CJ> - <KB|JC> = (KC|BJ) - (KJ|BC), each charge
        # distribution of one spin
        w = np.zeros((no, nv, nv, no))
        for K, (k, sk) in enumerate(occ):
            for B, (b, sb) in enumerate(vir):
                for C, (c, sc) in enumerate(vir):
                    for J, (j, sj) in enumerate(occ):
                        v = 0.0
                        if sk == sc and sb == sj:
                            v += g_ovvo[k, c, b, j]
                        if sk == sj and sb == sc:
                            v -= g_oovv[k, j, b, c]
                        w[K, B, C, J] = v
        X = np.einsum("ikac,kbcj->ijab", t, w)
        R = R + X - X.transpose(1, 0, 2, 3) - X.transpose(0, 1, 3, 2) + X.transpose(1, 0, 3, 2)
    E = 0.25 * float(np.sum(g_vvoo.transpose(2, 3, 0, 1) * t))
    out = {}
    for (i, j) in pairs:
        for name, (s1, s2) in spins.items():
            if (i, s1) in oidx and (j, s2) in oidx:
                I, J = oidx[(i, s1)], oidx[(j, s2)]
                blk = np.zeros((V, V))
                ra = [A for A, (a, sa) in enumerate(vir) if sa == s1]
                rb = [B for B, (b, sb) in enumerate(vir) if sb == s2]
                blk[np.ix_(sp_a[ra], sp_a[rb])] = R[I, J][np.ix_(ra, rb)]
                out[((i, j), name)] = blk
    return out, E
