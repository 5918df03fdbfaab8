"""Thin unpivoted Householder QR with a non-negative diagonal in R.

Test infrastructure (see the package docstring).  The paper's qr() and
orth() (Section II-A notation; the unpivoted QR is defined in Section II-B
as an orthonormal Q times an upper triangular R) leave the sign of each
column free.  Reading used here: diag(R) >= 0, which makes (Q, R) unique
whenever X has full column rank.  The reflector construction is the
textbook one (Golub and Van Loan, Matrix Computations, Section 5.1: a
reflector that maps x to a positive multiple of e1, computed without
cancellation), written out plainly with one reflector per column.

Pinned by: tests/test_oracle_qr.py (orthonormal Q, triangular R with
non-negative diagonal, Q R = X to rounding, agreement with LAPACK's QR
after the same sign normalization, exact handling of zero columns).
"""

import numpy as np


def _house(x):
    """Reflector H = I - beta v v^T with v[0] = 1 and H x = mu e1, mu >= 0.

    Returns (v, beta, mu).  When x[1:] is zero no reflection is applied
    (beta = 0) and mu = x[0], whose sign the caller fixes afterwards.
    """
    sigma = float(x[1:] @ x[1:])
    v = x.astype(np.float64).copy()
    x0 = float(x[0])
    if sigma == 0.0:
        v[0] = 1.0
        return v, 0.0, x0
    mu = np.sqrt(x0 * x0 + sigma)
    if x0 <= 0.0:
        v0 = x0 - mu
    else:
        v0 = -sigma / (x0 + mu)
    beta = 2.0 * v0 * v0 / (sigma + v0 * v0)
    v /= v0
    v[0] = 1.0
    return v, beta, mu


def householder_qr(X):
    """Return (Q, R): X = Q R, Q (m x d) orthonormal columns, R (d x d) upper
    triangular with diag(R) >= 0.  Requires m >= d.  float64 throughout."""
    X = np.array(X, dtype=np.float64, copy=True)
    m, d = X.shape
    if m < d:
        raise ValueError("householder_qr needs m >= d")
    vs, betas = [], []
    for j in range(d):
        v, beta, mu = _house(X[j:, j])
        if beta != 0.0:
            sub = X[j:, j:]
            w = v @ sub
            sub -= beta * np.outer(v, w)
        X[j, j] = mu
        X[j + 1:, j] = 0.0
        vs.append(v)
        betas.append(beta)
    R = np.triu(X[:d, :d])
    # Q = H_0 H_1 ... H_{d-1} applied to the first d columns of I (backward).
    Q = np.zeros((m, d))
    Q[:d, :d] = np.eye(d)
    for j in range(d - 1, -1, -1):
        v, beta = vs[j], betas[j]
        if beta != 0.0:
            sub = Q[j:, j:]
            w = v @ sub
            sub -= beta * np.outer(v, w)
    # Sign normalization: columns with negative R_jj (possible only where no
    # reflection was applied) are flipped; sign(0) is taken as +1.
    s = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    Q *= s[None, :]
    R *= s[:, None]
    return Q, R
