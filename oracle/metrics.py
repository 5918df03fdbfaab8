"""Reconstruction differences and errors, computed blockwise in float64.

Test infrastructure (see the package docstring).  The approximation of
Algorithm 1 is A-hat = Q L V^T (Section III-A, its final factors).  The tolerances
compare two approximations by the Frobenius norm of their difference
(Section II-A defines the norm), never forming an m x n matrix at once.

Pinned by: tests/test_oracle_metrics.py (against the dense formula on small
matrices) and tests/test_golden_spectra.py (the optimal-error helper
reproduces the SVD curves printed in the paper's figures).
"""

import numpy as np


def _as64(x):
    return np.asarray(x, dtype=np.float64)


def recon_diff(Qa, La, Va, Qb, Lb, Vb, block_rows=1024):
    """|| Qa La Va^T - Qb Lb Vb^T ||_F, blockwise over rows."""
    QLa = _as64(Qa) @ _as64(La)
    QLb = _as64(Qb) @ _as64(Lb)
    Vta, Vtb = _as64(Va).T, _as64(Vb).T
    total = 0.0
    for r0 in range(0, QLa.shape[0], block_rows):
        r1 = min(QLa.shape[0], r0 + block_rows)
        D = QLa[r0:r1] @ Vta - QLb[r0:r1] @ Vtb
        total += float(np.sum(D * D))
    return np.sqrt(total)


def recon_error(A, Q, L, V, block_rows=1024):
    """|| A - Q L V^T ||_F / || A ||_F, blockwise over rows."""
    A = np.asarray(A)
    QL = _as64(Q) @ _as64(L)
    Vt = _as64(V).T
    num = 0.0
    den = 0.0
    for r0 in range(0, A.shape[0], block_rows):
        r1 = min(A.shape[0], r0 + block_rows)
        Ab = _as64(A[r0:r1])
        D = Ab - QL[r0:r1] @ Vt
        num += float(np.sum(D * D))
        den += float(np.sum(Ab * Ab))
    return np.sqrt(num) / np.sqrt(den) if den > 0 else np.sqrt(num)


def recon_error_csr(rowptr, colidx, vals, m, n, Q, L, V, block_rows=512):
    """recon_error for a CSR matrix, densifying one row block at a time."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    vals = _as64(vals)
    QL = _as64(Q) @ _as64(L)
    Vt = _as64(V).T
    num = 0.0
    for r0 in range(0, m, block_rows):
        r1 = min(m, r0 + block_rows)
        Ab = np.zeros((r1 - r0, n))
        e0, e1 = rowptr[r0], rowptr[r1]
        rows = np.repeat(np.arange(r1 - r0), np.diff(rowptr[r0:r1 + 1]))
        Ab[rows, colidx[e0:e1]] = vals[e0:e1]
        D = Ab - QL[r0:r1] @ Vt
        num += float(np.sum(D * D))
    den = float(np.sum(vals * vals))
    return np.sqrt(num) / np.sqrt(den) if den > 0 else np.sqrt(num)


def orth_error(Q):
    """|| Q^T Q - I ||_F."""
    Q = _as64(Q)
    G = Q.T @ Q
    return float(np.linalg.norm(G - np.eye(G.shape[0])))


def optimal_error(sigma, r, norm):
    """Error of the best rank-r approximation for singular values `sigma`
    (sorted decreasingly): sigma_{r+1} in the 2-norm and the root sum of
    squares of sigma_{r+1..} in the Frobenius norm (Section II-B, the
    optimality of the truncated SVD)."""
    s = np.sort(_as64(sigma))[::-1]
    if norm == 2:
        return float(s[r]) if r < len(s) else 0.0
    if norm == "fro":
        return float(np.sqrt(np.sum(s[r:] ** 2)))
    raise ValueError(norm)
