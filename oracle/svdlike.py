"""The SVD-like form of RU-QLP (Remark 1 of Section III-B), in plain float64.

Test infrastructure (see the package docstring).

Remark 1: an SVD of the small middle factor turns the decomposition into an
SVD-like one.  With A ~ Q L V^T from ruqlp() and the d x d SVD
L = U-bar Sigma-bar V-bar^T:

    A ~ (Q U-bar) Sigma-bar (V V-bar)^T.

The paper states this for the R factor of qr(A P-bar); in the column-sketch
orientation the d x d middle factor is L, and the statement is the same.

svd_small() is the d x d SVD with the conventions this project fixes (the
paper fixes none):
  * singular values in descending order;
  * each right singular vector (column of V-bar) has its entry of largest
    magnitude positive (the first such entry on ties), and the matching left
    vector follows;
  * the left vector of a singular value that is exactly zero is zero.
With distinct singular values these make the factors unique.  The SVD itself
is numpy's (LAPACK) -- a library routine used as one step.

Pinned by tests/test_oracle_svdlike.py: the 2 x 2 closed form, diagonal
input (a permutation with signs), exact identities (U-bar Sigma V-bar^T = L,
orthonormal factors, the sign convention), singular values against the
eigenvalues of the Gram matrix, and the whole form against a matrix of
known rank and singular vectors.
"""

import numpy as np

from .ruqlp import ruqlp


def svd_small(M):
    """SVD of a square float64 matrix with the conventions above.
    Returns (Ub, s, Vb) with M = Ub diag(s) Vb^T."""
    M = np.asarray(M, dtype=np.float64)
    U, s, Vt = np.linalg.svd(M)
    Vb = Vt.T.copy()
    Ub = U.copy()
    for j in range(M.shape[1]):
        i = int(np.argmax(np.abs(Vb[:, j])))
        if Vb[i, j] < 0:
            Vb[:, j] = -Vb[:, j]
            Ub[:, j] = -Ub[:, j]
        if s[j] == 0.0:
            Ub[:, j] = 0.0
    return Ub, s, Vb


def svd_like(Q, L, V):
    """(Q U-bar, Sigma-bar, V V-bar) from the factors of A ~ Q L V^T."""
    Ub, s, Vb = svd_small(L)
    return Q @ Ub, s, V @ Vb


def ruqlp_svd(A, k, p, q, seed, omega_dtype="f64"):
    """RU-QLP followed by Remark 1: A ~ U diag(s) W^T."""
    Q, L, V = ruqlp(A, k, p, q, seed, omega_dtype=omega_dtype)
    return svd_like(Q, L, V)
