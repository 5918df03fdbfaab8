"""The reading behind one-pass orthonormalization inside the power
iteration, checked on the CPU in float64 against the oracle's Householder
QR: a basis that only feeds the next product may be taken from one
CholeskyQR pass, Q1 = Y R1^-1 with R1 = chol(Y^T Y), instead of the
orthonormal Q.  Q1 = Q R2 for an upper-triangular R2 (the second pass's
factor), so the next orthonormalization, of A^T Q1 = (A^T Q) R2, has the
same Q factor, and the power iteration's final basis and the method's
factors are unchanged up to rounding."""
import numpy as np

import oracle
import workloads


def _chol_pass(Y):
    """One CholeskyQR pass in float64: Q1 = Y R1^-1, R1 = chol(Y^T Y)."""
    R1 = np.linalg.cholesky(Y.T @ Y).T
    return np.linalg.solve(R1.T, Y.T).T, R1


def _qfac(X):
    """The Q factor of the oracle's Householder QR (diag(R) >= 0)."""
    Q, _ = oracle.householder_qr(X)
    return Q


def test_one_pass_basis_is_the_basis_times_an_upper_triangular_factor():
    rng = np.random.default_rng(3)
    sigma = workloads.spectrum("geometric", 300, rho=0.97)
    A, _, _, _ = workloads.dense_from_spectrum(500, 300, sigma, seed=2, trunc=0.0)
    Y = A @ rng.standard_normal((300, 40))
    Q = _qfac(Y)
    Q1, _ = _chol_pass(Y)
    # Q^T Q1 is upper triangular with a positive diagonal (it is R2)
    T = Q.T @ Q1
    assert np.abs(np.tril(T, -1)).max() < 1e-10 * np.abs(T).max()
    assert np.all(np.diag(T) > 0.0)
    # and the next orthonormalization does not see the difference
    Z = _qfac(A.T @ Q)
    Z1 = _qfac(A.T @ Q1)
    assert np.abs(Z - Z1).max() < 1e-10


def test_method_with_one_pass_intermediate_bases_matches_the_oracle():
    """The power iteration with one-pass intermediate bases (orthonormal
    bases only where the method returns them) reproduces oracle.ruqlp's
    factors for q = 1 and q = 2."""
    sigma = workloads.spectrum("geometric", 400, rho=0.95)
    A, _, _, _ = workloads.dense_from_spectrum(600, 400, sigma, seed=5, trunc=0.0)
    k, p, seed = 30, 10, 7
    d = k + p
    Om = oracle.gaussian_matrix(seed, 400, d)
    for q in (1, 2):
        Y = A @ Om
        Qb = _chol_pass(Y)[0]
        for it in range(q):
            W = _chol_pass(A.T @ Qb)[0]
            Y = A @ W
            Qb = _qfac(Y) if it == q - 1 else _chol_pass(Y)[0]
        V, R = oracle.householder_qr(A.T @ Qb)
        L = R.T
        Qo, Lo, Vo = oracle.ruqlp(A, k, p, q, seed)
        assert np.abs(Qb - Qo).max() < 1e-9
        assert np.abs(V - Vo).max() < 1e-9
        assert np.abs(L - Lo).max() < 1e-9 * np.abs(Lo).max()


def test_second_pass_is_needed_for_the_returned_basis():
    """The returned Q must be orthonormal, and one pass leaves an
    orthogonality error that grows with cond(Y)^2 u (here well above the
    float64 rounding), which is why the returned basis and the final QR take
    both passes."""
    rng = np.random.default_rng(1)
    U, _ = np.linalg.qr(rng.standard_normal((800, 30)))
    W, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    Y = U @ np.diag(np.logspace(0, -5, 30)) @ W
    Q1, _ = _chol_pass(Y)
    err1 = np.linalg.norm(Q1.T @ Q1 - np.eye(30))
    Q2, _ = _chol_pass(Q1)
    err2 = np.linalg.norm(Q2.T @ Q2 - np.eye(30))
    assert err1 > 1e-9 and err2 < 1e-14
