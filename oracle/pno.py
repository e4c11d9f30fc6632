"""PNO construction for one pair (FP64 oracle): pair density, truncation,
semicanonical PNOs.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper obtains one set of PNOs per pair by diagonalising the pair density
in the pair's domain and truncating at T_CutPNO (Sec. II.B.2); with no SOMOs
the set converges to the closed-shell MP1 PNOs.  Its NEVPT2 densities are
not printed; the density used here (a reading) is the spin-summed
first-order density of the pair's amplitude blocks in the domain basis,
    D = 1 / (2 (1 + delta_ij)) sum_{s s'} w_{ss'} (X X^T + X^T X),
with the pair-energy weights w = 1/2 (same spin) and 1 (opposite spin),
summed over all four spin blocks of the pair, the beta-alpha block of a
diagonal pair being the transpose of its alpha-beta block.  With no SOMOs
(X^{ab} = X^{ba} = T, X^{aa} = X^{bb} = T - T^T) it reduces to the
closed-shell MP1 pair density (T~^T T + T~ T^T) / (1 + delta_ij),
T~ = 2T - T^T (these weights are the only ones that do).  The PNOs are the
eigenvectors with occupation >= T_cut, rotated to diagonalise the domain's
virtual Fock matrix (semicanonical).

PNO overlaps between pairs: each domain is a contiguous window of an
orthonormal global virtual space (first function `first`, N functions), so
the overlap of source PNO c of pair q with target PNO a of pair p is the
sum, over the global functions the two windows share, of the products of
their coefficients (the metric between the two domains is the identity on
the shared functions and zero elsewhere).

Parity status: pinned by the closed-shell reduction of the density, the
untruncated limit (an orthogonal C with C^T F C = eig(F)), a spectrum fixed
by construction (truncation count and captured occupation), and the
eigen-equations themselves; the overlaps by the identity for a pair with
itself, the transpose rule, disjoint windows and the global embedding.
"""
import numpy as np


def pair_density(blocks, diagonal):
    """blocks: {name: X} of the stored spin blocks (AA, BB, AB, BA), each N x N
    in the domain basis; diagonal: i == j.  Returns the N x N density."""
    mats = dict(blocks)
    if diagonal and "AB" in mats and "BA" not in mats:
        mats["BA"] = mats["AB"].T
    N = next(iter(mats.values())).shape[0]
    D = np.zeros((N, N))
    for name, X in mats.items():
        w = 0.5 if name in ("AA", "BB") else 1.0
        D += w * (X @ X.T + X.T @ X)
    return D / (2.0 * (2.0 if diagonal else 1.0))


def sign_convention(C):
    """Each column multiplied by the sign of its largest-magnitude element (the
    first such element on ties), so that column is positive there."""
    C = C.copy()
    for k in range(C.shape[1]):
        idx = int(np.argmax(np.abs(C[:, k])))
        if C[idx, k] < 0:
            C[:, k] = -C[:, k]
    return C


def build_pnos(D, F, t_cut):
    """PNOs of one pair from its density D and virtual Fock F (both N x N,
    symmetric) in the domain basis.

    Returns (occupations, n_kept, C, eps): the eigenvalues of D in descending
    order, the number of them >= t_cut, the N x n coefficients of the
    semicanonical PNOs (columns, sign convention applied) and their orbital
    energies in ascending order."""
    occ, V = np.linalg.eigh(D)
    order = np.argsort(-occ, kind="stable")
    occ, V = occ[order], V[:, order]
    n = int(np.count_nonzero(occ >= t_cut))
    Vk = V[:, :n]
    Fp = Vk.T @ F @ Vk
    eps, U = np.linalg.eigh(Fp)
    C = sign_convention(Vk @ U)
    return occ, n, C, eps


def pno_overlap(C_p, first_p, C_q, first_q):
    """Overlap block of a coupling (target p, source q): n_q x n_p, element
    [c][a] = <PNO c of q | PNO a of p>.  C_p: N_p x n_p, C_q: N_q x n_q."""
    lo = max(first_p, first_q)
    hi = min(first_p + C_p.shape[0], first_q + C_q.shape[0])
    if hi <= lo:
        return np.zeros((C_q.shape[1], C_p.shape[1]))
    return C_q[lo - first_q:hi - first_q].T @ C_p[lo - first_p:hi - first_p]
