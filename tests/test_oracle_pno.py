"""Pins of the PNO-construction oracle (pair density, truncation,
semicanonical PNOs) against what the paper and the mathematics fix."""
import numpy as np
import pytest

from oracle.pno import build_pnos, pair_density, pno_overlap, sign_convention


def _sym(rng, n, scale=1.0):
    a = rng.standard_normal((n, n)) * scale
    return (a + a.T) / 2.0


@pytest.mark.parametrize("diagonal", [False, True])
def test_closed_shell_reduction_of_the_pair_density(diagonal):
    # Sec. II.B.2: with no SOMOs the single PNO set converges to the closed-shell
    # MP1 PNOs, whose density is (T~^T T + T~ T^T) / (1 + delta_ij), T~ = 2T - T^T
    rng = np.random.default_rng(3 + diagonal)
    N = 9
    T = rng.standard_normal((N, N))
    if diagonal:
        T = (T + T.T) / 2.0                      # the i = i amplitude is symmetric
        blocks = {"AB": T}
    else:
        blocks = {"AA": T - T.T, "BB": T - T.T, "AB": T, "BA": T}
    Tt = 2.0 * T - T.T
    want = (Tt.T @ T + Tt @ T.T) / (2.0 if diagonal else 1.0)
    np.testing.assert_allclose(pair_density(blocks, diagonal), want, rtol=1e-13, atol=1e-14)


def test_truncation_follows_a_spectrum_fixed_by_construction():
    rng = np.random.default_rng(7)
    N = 12
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    lam = np.array([0.3, 0.1, 3e-2, 1e-2, 4e-3, 1.2e-3, 8e-4, 2e-4, 5e-5, 1e-6, 1e-7, 1e-9])
    D = Q @ np.diag(lam) @ Q.T
    F = _sym(rng, N, 0.1) + np.diag(np.linspace(0.3, 2.8, N))
    occ, n, C, eps = build_pnos(D, F, 1e-3)
    np.testing.assert_allclose(occ, lam, rtol=1e-10, atol=1e-15)
    assert n == 6                                  # occupations 0.3 .. 1.2e-3
    # C spans the six leading natural orbitals, orthonormally
    P = C @ C.T
    Vk = Q[:, :6]
    np.testing.assert_allclose(P, Vk @ Vk.T, atol=1e-12)
    np.testing.assert_allclose(C.T @ C, np.eye(6), atol=1e-13)
    # semicanonical: the Fock matrix is diagonal in the PNOs, eps ascending
    np.testing.assert_allclose(C.T @ F @ C, np.diag(eps), atol=1e-13)
    assert np.all(np.diff(eps) > 0)


def test_untruncated_limit_diagonalises_the_domain_fock_matrix():
    rng = np.random.default_rng(11)
    N = 10
    A = rng.standard_normal((N, N))
    D = A @ A.T + 1e-3 * np.eye(N)                 # positive definite
    F = _sym(rng, N, 0.2) + np.diag(np.linspace(0.2, 3.0, N))
    occ, n, C, eps = build_pnos(D, F, 0.0)
    assert n == N
    np.testing.assert_allclose(C.T @ C, np.eye(N), atol=1e-13)
    np.testing.assert_allclose(eps, np.linalg.eigvalsh(F), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(C.T @ F @ C, np.diag(eps), atol=1e-12)


def test_rotation_of_the_domain_basis():
    # pair energies and PNOs do not depend on the choice of basis of the domain
    # (Sec. II.B.2): occupations and orbital energies are invariant and the
    # PNOs rotate with the basis
    rng = np.random.default_rng(13)
    N = 8
    A = rng.standard_normal((N, N))
    D = A @ A.T
    F = _sym(rng, N, 0.2) + np.diag(np.linspace(0.2, 3.0, N))
    R, _ = np.linalg.qr(rng.standard_normal((N, N)))
    o1, n1, C1, e1 = build_pnos(D, F, 0.05)
    o2, n2, C2, e2 = build_pnos(R.T @ D @ R, R.T @ F @ R, 0.05)
    assert n1 == n2
    np.testing.assert_allclose(o1, o2, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(e1, e2, rtol=1e-12)
    np.testing.assert_allclose(sign_convention(R.T @ C1), C2, atol=1e-11)


def test_density_is_positive_semidefinite_and_sign_convention():
    rng = np.random.default_rng(17)
    N = 7
    blocks = {k: rng.standard_normal((N, N)) for k in ("AA", "AB")}
    blocks["AA"] = blocks["AA"] - blocks["AA"].T
    D = pair_density(blocks, False)
    assert np.min(np.linalg.eigvalsh(D)) > -1e-14 * np.max(np.abs(D))
    C = sign_convention(rng.standard_normal((N, 4)))
    for k in range(4):
        assert C[np.argmax(np.abs(C[:, k])), k] > 0


def _pnos(rng, N, n):
    A = rng.standard_normal((N, N))
    occ, k, C, eps = build_pnos(A @ A.T, _sym(rng, N, 0.2) + np.diag(np.linspace(0.2, 3.0, N)), 0.0)
    return C[:, :n]


def test_overlap_of_a_pair_with_itself_is_the_identity():
    rng = np.random.default_rng(19)
    C = _pnos(rng, 11, 6)
    np.testing.assert_allclose(pno_overlap(C, 5, C, 5), np.eye(6), atol=1e-13)


def test_overlap_against_the_global_embedding():
    # each PNO as a vector of the global space (zero outside its window): the
    # overlap is the plain inner product of those vectors
    rng = np.random.default_rng(23)
    G = 40
    for (Np, fp, n1), (Nq, fq, n2) in [((10, 3, 4), (12, 8, 5)), ((9, 20, 9), (7, 22, 3)),
                                        ((6, 0, 2), (6, 30, 4)), ((13, 10, 7), (13, 10, 7))]:
        Cp, Cq = _pnos(rng, Np, n1), _pnos(rng, Nq, n2)
        Ep, Eq = np.zeros((G, n1)), np.zeros((G, n2))
        Ep[fp:fp + Np], Eq[fq:fq + Nq] = Cp, Cq
        want = np.array([[Eq[:, c] @ Ep[:, a] for a in range(n1)] for c in range(n2)])
        got = pno_overlap(Cp, fp, Cq, fq)
        assert got.shape == (n2, n1)
        np.testing.assert_allclose(got, want, atol=1e-14)
        np.testing.assert_allclose(pno_overlap(Cq, fq, Cp, fp), got.T, atol=1e-14)
    # disjoint windows do not overlap
    assert not np.any(pno_overlap(_pnos(rng, 5, 3), 0, _pnos(rng, 5, 2), 5))
