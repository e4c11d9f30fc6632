"""Synthetic inputs of PNO construction: per retained pair, a domain of N_p
virtual functions (orthonormal within the domain), the first-order amplitude
blocks of the pair in that basis and the domain's virtual Fock matrix.

Pairs and stored spin blocks follow the residual workloads (same chain, band
and SOMOs).  Per pair p = (i, j):
  * N_p (1..64) from a uniform or fixed rule; the domain is the window of N_p
    functions of an orthonormal global virtual space (4 functions per
    occupied orbital along the chain) centred on the pair: first_p =
    max(0, 2 (i + j) - N_p / 2);
  * each stored block X (N_p x N_p, row-major [a][b]) has elements
    sigma_p z 2^-floor((a + b) / tau_p), z unit normal, sigma_p =
    sigma_X exp(-|i - j| / 20), tau_p uniform on a small integer range: a
    graded matrix whose pair density has a geometric-like spectrum, so that
    about 20-50 occupations lie above T_CutPNO = 1e-7 for close pairs and
    fewer for distant ones;
  * F (N_p x N_p, symmetric): diagonal 0.2 + 2.8 u, off-diagonal 0.05 z.

Flat layouts (element offsets, 32-element aligned): X per pair, the stored
blocks back to back in the order AA, BB, AB, BA; F, C per pair N_p x N_p;
occupations and orbital energies per pair N_p.  Holds none of the method's
arithmetic.
"""
from dataclasses import dataclass, field
import numpy as np

from . import philox
from .problem import (CONFIGS, BLOCK_BITS, BLOCK_NAMES, SEG_DTYPE, MODE_DECAY, MODE_FOCK, F_DOM, F_TAU,
                      F_PX, F_PF, _align, _dims, stored_blocks, segment_values)

# matches dlpno_pno_pair in include/dlpno.h (48 bytes)
PNO_PAIR_DTYPE = np.dtype([("dim", np.int32), ("blocks", np.int32), ("diagonal", np.int32),
                           ("first", np.int32), ("off_X", np.int64), ("off_F", np.int64),
                           ("off_C", np.int64), ("off_v", np.int64)])

PNO_CONFIGS = {
    # every pair of the small radical, domains 1..33 (odd, even, tiny)
    "tiny": dict(dom=("uniform", 1, 33), tau=("uniform", 2, 5), sigma_X=0.02, t_cut=1e-7, seed=21),
    # the 1-D chain's 3,150 pairs, domains 24..64
    "chain": dict(dom=("uniform", 24, 64), tau=("uniform", 3, 6), sigma_X=0.02, t_cut=1e-7, seed=22),
    # the C160H322-shaped workload's 18,901 pairs, domains 40..64
    "c160": dict(dom=("uniform", 40, 64), tau=("uniform", 3, 6), sigma_X=0.02, t_cut=1e-7, seed=23),
}

F_OFFDIAG = 0.05


@dataclass
class PnoProblem:
    name: str
    seed: int
    n_occ: int
    pi: np.ndarray
    pj: np.ndarray
    pairs: np.ndarray              # PNO_PAIR_DTYPE [P]
    tau: np.ndarray
    sigma: np.ndarray
    t_cut: float
    n_X: int
    n_F: int
    n_C: int
    n_v: int
    segs: dict = field(default_factory=dict)
    seg_of_X: np.ndarray = None    # pair -> index into segs["X"], -1 when no block is stored

    @property
    def n_pairs(self):
        return len(self.pairs)

    def materialize(self, what):
        """Full flat array of 'X' or 'F' (host memory; small problems)."""
        out = np.zeros({"X": self.n_X, "F": self.n_F}[what])
        for seg in self.segs[what]:
            v = segment_values(self.seed, seg)
            out[seg["off"]:seg["off"] + v.size] = v.ravel()
        return out

    def blocks_of(self, p, X):
        """{name: N x N block} of pair p from the flat X array."""
        d = self.pairs[p]
        N, o = int(d["dim"]), int(d["off_X"])
        out = {}
        for name in BLOCK_NAMES:
            if d["blocks"] & BLOCK_BITS[name]:
                out[name] = X[o:o + N * N].reshape(N, N)
                o += N * N
        return out

    def pair_inputs(self, p):
        """({name: X block}, F) of pair p regenerated from its counters."""
        d = self.pairs[p]
        N = int(d["dim"])
        blocks = {}
        k = int(self.seg_of_X[p])
        if k >= 0:
            v = segment_values(self.seed, self.segs["X"][k]).reshape(-1, N, N)
            names = [nm for nm in BLOCK_NAMES if d["blocks"] & BLOCK_BITS[nm]]
            blocks = {nm: v[i] for i, nm in enumerate(names)}
        F = segment_values(self.seed, self.segs["F"][p]).reshape(N, N)
        return blocks, F

    def fock_of(self, p, F):
        d = self.pairs[p]
        N, o = int(d["dim"]), int(d["off_F"])
        return F[o:o + N * N].reshape(N, N)


def build_pno_problem(name="tiny", **override):
    """Descriptors and generator segments of a named (or customised) PNO
    workload.  Overrides: any PNO_CONFIGS or CONFIGS key (n_occ, band, somos,
    dom, tau, sigma_X, t_cut, seed)."""
    cfg = dict(CONFIGS[name]) if name in CONFIGS else {}
    cfg.update(PNO_CONFIGS.get(name, {}))
    cfg.update(override)
    seed = int(cfg["seed"])
    n_occ = int(cfg["n_occ"])
    is_somo = np.zeros(n_occ, dtype=np.uint8)
    for s in cfg["somos"]:
        is_somo[s] = 1
    band = n_occ if cfg.get("band") is None else int(cfg["band"])
    ii, jj = [], []
    for i in range(n_occ):
        for j in range(i, min(n_occ, i + band + 1)):
            ii.append(i)
            jj.append(j)
    pi, pj = np.array(ii, dtype=np.int32), np.array(jj, dtype=np.int32)
    P = len(pi)
    dim = _dims(cfg["dom"], seed, F_DOM, P)
    tau = _dims(cfg["tau"], seed, F_TAU, P)
    sigma = float(cfg["sigma_X"]) * np.exp(-np.abs(pi - pj).astype(np.float64) / 20.0)

    pairs = np.zeros(P, dtype=PNO_PAIR_DTYPE)
    names = [stored_blocks(int(a), int(b), is_somo) for a, b in zip(pi, pj)]
    nblk = np.array([len(n) for n in names], dtype=np.int64)
    n2 = dim.astype(np.int64) ** 2
    szX = np.array([_align(int(k * b)) for k, b in zip(nblk, n2)], dtype=np.int64)
    szF = np.array([_align(int(b)) for b in n2], dtype=np.int64)
    szv = np.array([_align(int(n)) for n in dim], dtype=np.int64)
    pairs["dim"] = dim
    pairs["blocks"] = [sum(BLOCK_BITS[n] for n in nm) for nm in names]
    pairs["diagonal"] = (pi == pj).astype(np.int32)
    pairs["first"] = np.maximum(0, 2 * (pi.astype(np.int64) + pj) - dim // 2)
    pairs["off_X"] = np.concatenate([[0], np.cumsum(szX)[:-1]])
    pairs["off_F"] = np.concatenate([[0], np.cumsum(szF)[:-1]])
    pairs["off_C"] = pairs["off_F"]
    pairs["off_v"] = np.concatenate([[0], np.cumsum(szv)[:-1]])

    has = nblk > 0
    segX = np.zeros(int(has.sum()), dtype=SEG_DTYPE)
    segX["off"], segX["stream"] = pairs["off_X"][has], np.arange(P)[has]
    segX["field"], segX["mode"] = F_PX, MODE_DECAY
    segX["layers"], segX["rows"], segX["cols"] = nblk[has], dim[has], dim[has]
    segX["pad"], segX["scale"] = tau[has], sigma[has]
    segF = np.zeros(P, dtype=SEG_DTYPE)
    segF["off"], segF["stream"], segF["field"], segF["mode"] = pairs["off_F"], np.arange(P), F_PF, MODE_FOCK
    segF["layers"], segF["rows"], segF["cols"], segF["scale"] = 1, dim, dim, F_OFFDIAG
    return PnoProblem(name=name, seed=seed, n_occ=n_occ, pi=pi, pj=pj, pairs=pairs, tau=tau, sigma=sigma,
                      t_cut=float(cfg["t_cut"]), n_X=int(szX.sum()), n_F=int(szF.sum()), n_C=int(szF.sum()),
                      n_v=int(szv.sum()), segs={"X": segX, "F": segF},
                      seg_of_X=np.where(has, np.cumsum(has) - 1, -1))
