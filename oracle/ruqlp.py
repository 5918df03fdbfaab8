"""RU-QLP in plain float64: the reference result the HIP path must match.

Test infrastructure (see the package docstring).

Algorithm 1 (Section III-A) with Algorithm 2 (Section III-B), run on A^T:
the sketch multiplies A by an n x d Gaussian from the right, so Q spans an
approximation of the range of A, and the final unpivoted QR is taken of
B^T = A^T Q.  Step by step:

  1. Omega = randn(n, d), rounded to the precision the device stores it in
     and then held in float64 (philox.gaussian_matrix).
  2. Q = orth(A Omega)                    (Algorithm 1, sketch and orth)
  3. repeat q times (Algorithm 2, orthonormalizing at every half step):
        W = orth(A^T Q);  Q = orth(A W)
  4. B^T = A^T Q                           (Algorithm 1, the product with A)
  5. [V, Rt] = qr(B^T)                     (Algorithm 1, unpivoted QR)
  6. L = Rt^T (lower triangular)           (Algorithm 1, L = R-tilde^T)

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
    """RU-QLP in the paper's own orientation: Algorithm 1 as printed
    (Section III-A) with Algorithm 2 (Section III-B) computing P-bar.

      1. Phi = randn(m, d)                 (rounded as in ruqlp)
      2. P-bar = orth(A^T Phi); q times: P-bar = orth(A P-bar), then
         P-bar = orth(A^T P-bar)           (Algorithm 2)
      3. [Q, R] = qr(A P-bar)
      4. [P-tilde, R-tilde] = qr(R^T)
      5. Q;  P = P-bar P-tilde;  L = R-tilde^T

    Returns (Q, L, P): Q m x d, L d x d lower triangular, P n x d; A is
    approximated by Q L P^T = A P-bar P-bar^T.

    Pinned by: tests/test_oracle_ruqlp.py -- invariants (orthonormal Q and
    P, triangular L, Q L P^T = A P-bar P-bar^T), exact recovery when
    rank(A) <= d, sigma_i(L) <= sigma_i(A), and its relation to the column
    orientation on A^T (same P-bar and Q, and L-values of the extra QR).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    d = k + p
    if not (1 <= k and d <= min(m, n)):
        raise ValueError("need 1 <= k and k + p <= min(m, n)")
    phi = round_to(gaussian_matrix(seed, m, d), omega_dtype)
    Pbar = orth(A.T @ phi)
    for _ in range(q):
        Pbar = orth(A @ Pbar)
        Pbar = orth(A.T @ Pbar)
    Q, R = householder_qr(A @ Pbar)
    Pt, Rt = householder_qr(R.T)
    return Q, Rt.T.copy(), Pbar @ Pt
