"""Pins for the SVD-like form of the oracle (Remark 1, oracle/svdlike.py)."""
import numpy as np
import pytest

from oracle.svdlike import svd_small, svd_like, ruqlp_svd
import oracle
import workloads


def _check_conventions(M, Ub, s, Vb, tol=1e-13):
    d = M.shape[0]
    scale = max(1.0, np.abs(M).max())
    assert np.all(np.diff(s) <= 0) and np.all(s >= 0)
    assert np.abs(Ub @ np.diag(s) @ Vb.T - M).max() <= tol * scale * d
    assert np.abs(Vb.T @ Vb - np.eye(d)).max() <= tol * d
    nz = s > 0
    assert np.abs(Ub[:, nz].T @ Ub[:, nz] - np.eye(int(nz.sum()))).max() <= tol * d
    for j in range(d):
        i = int(np.argmax(np.abs(Vb[:, j])))
        assert Vb[i, j] > 0


@pytest.mark.parametrize("M", [[[3.0, 1.0], [-2.0, 0.5]], [[1.0, 0.0], [4.0, 2.0]], [[0.0, 2.0], [1e-3, 0.0]]])
def test_two_by_two_closed_form(M):
    """sigma_1^2 = (||M||_F^2 + sqrt(||M||_F^4 - 4 det(M)^2)) / 2 and
    sigma_1 sigma_2 = |det(M)| (the product form avoids the cancellation of
    the minus root)."""
    M = np.array(M)
    f2 = (M ** 2).sum()
    det = M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]
    disc = np.sqrt(f2 * f2 - 4 * det * det)
    s1 = np.sqrt((f2 + disc) / 2)
    expect = np.array([s1, abs(det) / s1])
    Ub, s, Vb = svd_small(M)
    assert np.allclose(s, expect, rtol=1e-13, atol=1e-15)
    _check_conventions(M, Ub, s, Vb)


def test_diagonal_is_a_signed_permutation():
    dvals = np.array([0.5, -4.0, 2.0, -1.0, 3.0])
    Ub, s, Vb = svd_small(np.diag(dvals))
    order = [1, 4, 2, 3, 0]  # |d| descending
    assert np.array_equal(s, np.abs(dvals)[order])
    P = np.eye(5)[:, order]
    assert np.array_equal(Vb, P)  # largest entry (the only one) positive
    assert np.array_equal(Ub, P * np.sign(dvals)[order][None, :])


def test_zero_singular_value_has_zero_left_vector():
    Ub, s, Vb = svd_small(np.diag([3.0, 0.0, 1.0]))
    assert np.array_equal(s, [3.0, 1.0, 0.0])
    assert np.array_equal(Ub[:, 2], np.zeros(3))
    assert np.array_equal(np.abs(Vb[:, 2]), [0.0, 1.0, 0.0])


@pytest.mark.parametrize("d", [7, 50, 130])
def test_random_lower_triangular(d):
    rng = np.random.default_rng(d)
    M = np.tril(rng.standard_normal((d, d))) + 4 * np.eye(d)
    Ub, s, Vb = svd_small(M)
    _check_conventions(M, Ub, s, Vb, tol=1e-14)
    # singular values against the eigenvalues of M^T M (well conditioned here)
    ev = np.sqrt(np.linalg.eigvalsh(M.T @ M))[::-1]
    assert np.allclose(s, ev, rtol=1e-11)


def test_identity_with_the_qlv_form():
    A, _, _, _ = workloads.dense_from_spectrum(120, 90, workloads.spectrum("geometric", 90, rho=0.85), 4,
                                               trunc=0.0)
    Q, L, V = oracle.ruqlp(A, 12, 5, 1, seed=3)
    U, s, W = svd_like(Q, L, V)
    assert np.abs(U @ np.diag(s) @ W.T - Q @ L @ V.T).max() <= 1e-13 * np.abs(A).max() * 17
    assert np.abs(U.T @ U - np.eye(17)).max() <= 1e-13
    assert np.abs(W.T @ W - np.eye(17)).max() <= 1e-13


def test_known_rank_and_vectors():
    """Rank 8 < d: the form is exact, its singular values and (up to sign)
    singular vectors are A's own."""
    sigma = np.zeros(100)
    sigma[:8] = [5.0, 3.0, 2.0, 1.5, 1.0, 0.7, 0.4, 0.2]
    A, sr, U0, V0 = workloads.dense_from_spectrum(150, 100, sigma, 9, trunc=0.0)
    U0, V0 = U0[:, :8], V0[:, :8]
    U, s, W = ruqlp_svd(A, 10, 5, 1, seed=21)
    assert np.abs(U @ np.diag(s) @ W.T - A).max() <= 1e-12 * 5.0
    assert np.allclose(s[:8], sigma[:8], rtol=0, atol=1e-12 * 5.0)
    assert np.all(s[8:] <= 1e-12 * 5.0)
    assert np.allclose(np.abs(np.sum(U[:, :8] * U0, axis=0)), 1.0, atol=1e-10)
    assert np.allclose(np.abs(np.sum(W[:, :8] * V0, axis=0)), 1.0, atol=1e-10)
    # the left and right vectors of each pair carry the same sign change
    assert np.allclose(np.sum(U[:, :8] * U0, axis=0), np.sum(W[:, :8] * V0, axis=0), atol=1e-10)
