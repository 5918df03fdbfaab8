"""Pins for the oracle's Householder QR (oracle/householder.py)."""
import numpy as np
import pytest

from oracle.householder import householder_qr
from tests.pins import check_qr, lapack_qr_positive


def _mat(m, d, cond, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, d)))
    W, _ = np.linalg.qr(rng.standard_normal((d, d)))
    s = np.logspace(0, -np.log10(cond), d)
    return (U * s) @ W.T


@pytest.mark.parametrize("m,d", [(1, 1), (5, 5), (50, 10), (200, 1), (300, 40), (64, 63)])
@pytest.mark.parametrize("cond", [1.0, 1e6])
def test_qr_properties(m, d, cond):
    X = _mat(m, d, cond, m * 31 + d)
    Q, R = householder_qr(X)
    ok, info = check_qr(X, Q, R)
    assert ok, info


@pytest.mark.parametrize("m,d", [(30, 7), (200, 25), (7, 7)])
def test_qr_matches_lapack(m, d):
    X = _mat(m, d, 1e3, 5 + m + d)
    Q, R = householder_qr(X)
    Ql, Rl = lapack_qr_positive(X)
    # unique for full column rank; differences bounded by ~cond * eps
    assert np.linalg.norm(Q - Ql) <= 1e-10
    assert np.linalg.norm(R - Rl) <= 1e-10 * np.linalg.norm(R)


def test_qr_sign_and_zero_columns():
    # column already a negative multiple of e1 (no reflection): sign fixed
    X = np.zeros((4, 2))
    X[0, 0] = -3.0
    X[:, 1] = [1.0, 2.0, 0.0, 0.0]
    Q, R = householder_qr(X)
    assert R[0, 0] == 3.0 and np.allclose(Q @ R, X)
    ok, info = check_qr(X, Q, R)
    assert ok, info
    # a zero column gives a zero diagonal entry and still orthonormal Q
    X = np.random.default_rng(0).standard_normal((10, 4))
    X[:, 2] = 0.0
    Q, R = householder_qr(X)
    assert R[2, 2] == 0.0
    ok, info = check_qr(X, Q, R)
    assert ok, info


def test_qr_rank_deficient():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((40, 3))
    X = np.hstack([B, B @ rng.standard_normal((3, 4))])
    Q, R = householder_qr(X)
    ok, info = check_qr(X, Q, R)
    assert ok, info
    assert np.all(np.abs(np.diag(R)[3:]) < 1e-13 * np.abs(R).max())
