"""RU-QLP in plain float64: the reference result the HIP path must match.

Test infrastructure (see the package docstring).

Algorithm 1 (Section III-A) with the power iteration of Algorithm 2
(Section III-B), in the column-sketch orientation: the algorithms applied to
A^T, so that the Gaussian test matrix (n x d; philox.gaussian_matrix, rounded
to the precision the device stores it in and then held in float64)
multiplies A from the right, Q is the orthonormalized sketch after q power
steps (orthonormalized at every half step), and the final unpivoted QR is
taken of A^T Q, whose R gives L = R^T.

Result: A ~ Q L V^T = Q Q^T A, with Q (m x d) and V (n x d) orthonormal.
orth(X) is the Q factor of householder_qr(X).  The products with A are
plain float64 matrix products (numpy matmul for dense A, csr.csr_matmul for
sparse A).

Pinned by: tests/test_oracle_ruqlp.py -- exact invariants (orthonormal
factors, triangular L, L V^T = Q^T A), exact recovery when rank(A) <= d,
sigma_i(L) <= sigma_i(A), the Eckart-Young lower bound, the Theorem 2 and
Theorem 5 upper bounds evaluated with the actual Omega, the q -> infinity
limit (orthogonal iteration, Section III-C: L tends to diag(sigma)), and the
q = 0 case against LAPACK's QR.
"""

import numpy as np

from .householder import householder_qr
from .philox import gaussian_matrix
from .csr import csr_matmul, csr_transpose


def orth(X):
    """Orthonormal basis of range(X): the Q factor of the unpivoted QR."""
    return householder_qr(X)[0]


def round_to(x, dtype):
    """Round float64 values to `dtype` storage ('f64', 'f32' or 'bf16') and
    return them as float64."""
    if dtype in ("f64", np.float64, None):
        return np.asarray(x, dtype=np.float64)
    if dtype in ("f32", np.float32):
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        from .bf16 import round_bf16
        return round_bf16(x)
    raise ValueError(f"unknown dtype {dtype!r}")


def _ruqlp_core(mul_A, mul_At, n, k, p, q, seed, omega_dtype):
    d = k + p
    omega = round_to(gaussian_matrix(seed, n, d), omega_dtype)
    Q = orth(mul_A(omega))
    for _ in range(q):
        W = orth(mul_At(Q))
        Q = orth(mul_A(W))
    Bt = mul_At(Q)
    V, Rt = householder_qr(Bt)
    L = Rt.T.copy()
    return Q, L, V


def ruqlp(A, k, p, q, seed, omega_dtype="f64", operand_dtype="f64"):
    """RU-QLP of dense A (m x n, any float dtype; used in float64).

    Returns (Q, L, V): Q m x d, L d x d lower triangular, V n x d, d = k + p.

    operand_dtype="bf16" models products taken in bfloat16: every product
    with A uses A and its right-hand factor rounded to bfloat16 (round_to)
    and is then formed exactly in float64.  The orthonormalizations are
    unchanged, so Q L V^T = Q round(Q)^T round(A) holds exactly.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    d = k + p
    if not (1 <= k and d <= min(m, n)):
        raise ValueError("need 1 <= k and k + p <= min(m, n)")
    Ar = round_to(A, operand_dtype)
    return _ruqlp_core(lambda X: Ar @ round_to(X, operand_dtype), lambda X: Ar.T @ round_to(X, operand_dtype),
                       n, k, p, q, seed, omega_dtype)


def ruqlp_csr(rowptr, colidx, vals, m, n, k, p, q, seed, omega_dtype="f64"):
    """RU-QLP of a CSR matrix; the same steps with CSR products.

    A^T X uses the CSR of A^T built by csr.csr_transpose.
    """
    d = k + p
    if not (1 <= k and d <= min(m, n)):
        raise ValueError("need 1 <= k and k + p <= min(m, n)")
    rt, ct, vt = csr_transpose(rowptr, colidx, vals, m, n)
    mul_A = lambda X: csr_matmul(rowptr, colidx, vals, m, n, X)  # noqa: E731
    mul_At = lambda X: csr_matmul(rt, ct, vt, n, m, X)  # noqa: E731
    return _ruqlp_core(mul_A, mul_At, n, k, p, q, seed, omega_dtype)


def ruqlp_paper(A, k, p, q, seed, omega_dtype="f64"):
    """RU-QLP in the paper's own orientation (Algorithm 1 as printed, with
    Algorithm 2 computing P-bar): the column-sketch method above applied to
    A^T -- its basis is the paper's P-bar (n x d, from an m x d Gaussian),
    its right-hand factor the paper's Q and its L the transposed R of the
    paper's QR of A P-bar -- followed by the d x d unpivoted QR of that L,
    which gives P-tilde and R-tilde: P = P-bar P-tilde, L = R-tilde^T.

    Returns (Q, L, P): Q m x d, L d x d lower triangular, P n x d; A is
    approximated by Q L P^T = A P-bar P-bar^T.

    Pinned by: tests/test_oracle_ruqlp.py -- invariants (orthonormal Q and
    P, triangular L, Q L P^T = A P-bar P-bar^T), exact recovery when
    rank(A) <= d, sigma_i(L) <= sigma_i(A), and the L-values of the extra QR
    against an independent LAPACK QR of the d x d factor.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    d = k + p
    if not (1 <= k and d <= min(m, n)):
        raise ValueError("need 1 <= k and k + p <= min(m, n)")
    Pbar, Rt, Q = ruqlp(A.T, k, p, q, seed, omega_dtype)
    Pt, Rtt = householder_qr(Rt)
    return Q, Rtt.T.copy(), Pbar @ Pt
