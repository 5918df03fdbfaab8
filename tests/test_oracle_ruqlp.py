"""Pins for the whole method in the oracle (oracle/ruqlp.py)."""
import numpy as np
import pytest

import oracle
from oracle import philox
from oracle.metrics import optimal_error
import workloads
from tests import pins


def _small(spec, m=300, n=200, seed=0, **kw):
    sigma = workloads.spectrum(spec, min(m, n), **kw)
    A, s, U, V = workloads.dense_from_spectrum(m, n, sigma, seed, trunc=0.0)
    full = np.zeros(min(m, n))
    full[:len(s)] = s
    return A, full, U, V


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("spec,kw", [("geometric", dict(rho=0.8)), ("gapped", dict(gap_at=10))])
def test_invariants(q, spec, kw):
    A, s, U, V = _small(spec, seed=q + 3, **kw)
    Q, L, Vf = oracle.ruqlp(A, 10, 5, q, seed=17)
    ok, info = pins.check_ruqlp_invariants(A, Q, L, Vf)
    assert ok, info
    ok, info = pins.check_sv_interlacing(s, L)
    assert ok, info
    # Eckart-Young: no rank-d approximation beats the truncated SVD
    err = np.linalg.norm(A - Q @ L @ Vf.T)
    assert err >= optimal_error(s, 15, "fro") * (1 - 1e-12)


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("spec,kw", [("geometric", dict(rho=0.8)), ("gapped", dict(gap_at=10))])
def test_theorem2_and_theorem5_bounds(q, seed, spec, kw):
    m, n, k, p = 300, 200, 10, 5
    A, s, U, V = _small(spec, m, n, seed=100 + seed, **kw)
    Omega = philox.gaussian_matrix(seed, n, k + p)
    Q, L, Vf = oracle.ruqlp(A, k, p, q, seed=seed)
    ok, info = pins.check_theorem_bounds(A, s, U[:, :k], V[:, :k], Omega, Q, Vf, k, q)
    assert ok, info


@pytest.mark.parametrize("rank,k,p", [(6, 8, 4), (10, 10, 0), (1, 3, 2)])
def test_exact_recovery_when_rank_le_d(rank, k, p):
    sigma = np.zeros(80)
    sigma[:rank] = np.linspace(2.0, 0.5, rank)
    A, _, _, _ = workloads.dense_from_spectrum(120, 80, sigma, seed=rank, trunc=0.0)
    for q in (0, 1):
        Q, L, Vf = oracle.ruqlp(A, k, p, q, seed=5)
        assert oracle.recon_error(A, Q, L, Vf) <= 1e-13
        ok, info = pins.check_ruqlp_invariants(A, Q, L, Vf)
        assert ok, info
        # rank revealed: diag(L) beyond the rank is negligible
        assert np.all(np.abs(np.diag(L)[rank:]) <= 1e-13 * np.abs(np.diag(L)).max())


def test_zero_matrix():
    A = np.zeros((30, 20))
    Q, L, Vf = oracle.ruqlp(A, 3, 2, 1, seed=1)
    assert np.all(L == 0.0)
    assert oracle.orth_error(Q) < 1e-13 and oracle.orth_error(Vf) < 1e-13


def test_orthogonal_iteration_limit():
    # Section III-C: with many power steps the method is orthogonal
    # iteration and L tends to diag(sigma_1..sigma_d) (diag(L) >= 0 here).
    A, s, _, _ = _small("geometric", m=60, n=50, seed=9, rho=0.7)
    Q, L, Vf = oracle.ruqlp(A, 6, 2, 60, seed=4)
    ok, info = pins.check_orth_iteration_limit(L, s)
    assert ok, info


@pytest.mark.parametrize("m,n,k,p", [(90, 60, 5, 3), (40, 40, 10, 0)])
def test_q0_matches_lapack_composition(m, n, k, p):
    # q = 0: Q = qr(A Omega).Q, [V, Rt] = qr(A^T Q), L = Rt^T, each QR unique
    A, s, _, _ = _small("geometric", m=m, n=n, seed=m, rho=0.9)
    Omega = philox.gaussian_matrix(21, n, k + p)
    Ql, _ = pins.lapack_qr_positive(A @ Omega)
    Vl, Rl = pins.lapack_qr_positive(A.T @ Ql)
    Q, L, Vf = oracle.ruqlp(A, k, p, 0, seed=21)
    assert np.linalg.norm(Q - Ql) < 1e-9
    assert np.linalg.norm(Vf - Vl) < 1e-9
    assert np.linalg.norm(L - Rl.T) < 1e-9 * np.linalg.norm(L)


def test_csr_path_equals_dense_path():
    rowptr, colidx, vals = workloads.csr_uniform(400, 150, 3000, seed=8)
    from oracle.csr import csr_to_dense
    D = csr_to_dense(rowptr, colidx, vals, 400, 150)
    Qs, Ls, Vs = oracle.ruqlp_csr(rowptr, colidx, vals, 400, 150, 8, 4, 1, seed=3, omega_dtype="f32")
    Qd, Ld, Vd = oracle.ruqlp(D, 8, 4, 1, seed=3, omega_dtype="f32")
    assert np.linalg.norm(Qs - Qd) < 1e-11 and np.linalg.norm(Vs - Vd) < 1e-11
    assert np.linalg.norm(Ls - Ld) < 1e-11 * np.linalg.norm(Ld)


def test_omega_rounding_modes():
    A, _, _, _ = _small("geometric", m=50, n=40, seed=1, rho=0.8)
    Q64, _, _ = oracle.ruqlp(A, 5, 2, 0, seed=2, omega_dtype="f64")
    Q32, _, _ = oracle.ruqlp(A, 5, 2, 0, seed=2, omega_dtype="f32")
    # float32 rounding of Omega moves Q by ~1e-8, not more
    assert 0 < np.linalg.norm(Q64 - Q32) < 1e-5


@pytest.mark.parametrize("q", [0, 1])
def test_bf16_operand_model(q):
    """operand_dtype='bf16': the products see A and the right-hand factor
    rounded to bfloat16.  Pins: the exact identity Q L V^T = Q round(Q)^T
    round(A) of the projection step; orthonormal Q, V and triangular L still
    hold; and the result moves away from the float64 result by about the
    bfloat16 unit roundoff, no more and no less."""
    from oracle.bf16 import round_bf16
    A, s, _, _ = _small("polynomial", m=300, n=200, seed=3, power=1.5)
    k, p = 10, 5
    Qb, Lb, Vb = oracle.ruqlp(A, k, p, q, seed=4, omega_dtype="bf16", operand_dtype="bf16")
    Qd, Ld, Vd = oracle.ruqlp(A, k, p, q, seed=4, omega_dtype="bf16")
    d = k + p
    assert np.linalg.norm(Qb.T @ Qb - np.eye(d)) < 1e-13
    assert np.linalg.norm(Vb.T @ Vb - np.eye(d)) < 1e-13
    assert np.allclose(np.triu(Lb, 1), 0.0)
    lhs = Qb @ Lb @ Vb.T
    rhs = Qb @ (round_bf16(Qb).T @ round_bf16(A))
    assert np.linalg.norm(lhs - rhs) < 1e-13 * np.linalg.norm(rhs)
    # the unrounded projection would not satisfy it
    assert np.linalg.norm(lhs - Qb @ (Qb.T @ A)) > 1e-6 * np.linalg.norm(rhs)
    diff = np.linalg.norm(Qb @ Lb @ Vb.T - Qd @ Ld @ Vd.T) / np.linalg.norm(A)
    assert 1e-6 < diff < 3e-2


@pytest.mark.parametrize("m,n,seed", [(300, 200, 7), (257, 257, 1), (64, 5, 3)])
def test_fast_orth_generator_has_exact_spectrum(m, n, seed):
    """The structured-orthogonal input generator used for the 20000 x 15000
    case: its singular values are exactly the prescribed ones, and its
    singular vectors are spread (no entry of A dominates)."""
    s = workloads.spectrum("polynomial", n, power=1.5)
    A = workloads.dense_fast_orth(m, n, s, seed, np.float64)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(sv - s) / s) < 1e-12
    assert np.isclose(np.linalg.norm(A) ** 2, np.sum(s ** 2), rtol=1e-13)
    # singular vectors are signed, permuted orthonormal DCT-II columns, whose
    # entries are at most sqrt(2 / N): |A_ij| <= 2 sum(sigma) / sqrt(m n)
    assert np.abs(A).max() <= 2.0 * s.sum() / np.sqrt(m * n) * (1 + 1e-12)
    with pytest.raises(ValueError):
        workloads.dense_fast_orth(n - 1 if n > 1 else 0, n, s, seed)


def test_serving_request_generator():
    """Request shapes follow their ranges; a request's matrix has exactly
    the truncated geometric spectrum, for tall and wide shapes."""
    reqs = workloads.serving_requests(50, 3)
    for r in reqs:
        assert 512 <= r["m"] <= 8192 and 256 <= r["n"] <= 4096 and r["p"] == 10
        assert 8 <= r["k"] <= min(256, min(r["m"], r["n"]) - 10) and 0.8 <= r["rho"] <= 0.99
    for r in workloads.serving_requests(4, 7, m_range=(30, 120), n_range=(30, 120), kmax=12):
        A = workloads.request_matrix(r, np.float64)
        assert A.shape == (r["m"], r["n"])
        i = np.arange(1, min(A.shape) + 1)
        want = np.where(i <= np.ceil(np.log(1e-8) / np.log(r["rho"])), r["rho"] ** i, 0.0)
        assert np.allclose(np.linalg.svd(A, compute_uv=False), want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("m,n,k,p,q", [(120, 90, 10, 4, 0), (90, 120, 8, 3, 1), (200, 150, 20, 5, 2)])
def test_paper_orientation_invariants(m, n, k, p, q):
    """Algorithm 1 as printed: orthonormal Q and P, lower-triangular L,
    Q L P^T = A P-bar P-bar^T (P-bar = P P-tilde^T), and sigma_i(L) <= sigma_i(A)."""
    sigma = workloads.spectrum("geometric", min(m, n), rho=0.85)
    A, s, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed=m + n, trunc=0.0)
    Q, L, P = oracle.ruqlp_paper(A, k, p, q, seed=3)
    d = k + p
    assert np.linalg.norm(Q.T @ Q - np.eye(d)) < 1e-13
    assert np.linalg.norm(P.T @ P - np.eye(d)) < 1e-13
    assert np.all(np.triu(L, 1) == 0)
    # Q L P^T is the projection of A's rows onto span(P)
    assert np.linalg.norm(Q @ L @ P.T - A @ P @ P.T) < 1e-12 * np.linalg.norm(A)
    assert np.all(np.linalg.svd(L, compute_uv=False) <= s[:d] * (1 + 1e-12))


def test_paper_orientation_is_column_orientation_of_transpose():
    """The paper's P-bar, Q and R are the column orientation's Q, V and L^T
    on A^T with the same Gaussian (m x d): the extra d x d QR only rotates
    P and re-triangularizes L (checked with LAPACK's QR of the d x d factor)."""
    m, n, k, p, q = 150, 110, 12, 4, 1
    sigma = workloads.spectrum("geometric", min(m, n), rho=0.9)
    A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed=5, trunc=0.0)
    Q, L, P = oracle.ruqlp_paper(A, k, p, q, seed=8)
    Qc, Lc, Vc = oracle.ruqlp(A.T, k, p, q, seed=8)  # Qc spans A^T's range sketch: P-bar
    # Q (paper) = Vc (column orientation on A^T); R = Lc^T; R^T = Lc = P-tilde R-tilde
    assert np.linalg.norm(Q - Vc) < 1e-11
    Pt, Rt = np.linalg.qr(Lc)
    sgn = np.sign(np.diag(Rt))
    Pt, Rt = Pt * sgn, Rt * sgn[:, None]
    assert np.linalg.norm(L - Rt.T) < 1e-11 * np.linalg.norm(L)
    assert np.linalg.norm(P - Qc @ Pt) < 1e-11


@pytest.mark.parametrize("rank", [3, 9])
def test_paper_orientation_exact_recovery(rank):
    rng = np.random.default_rng(rank)
    A = rng.standard_normal((80, rank)) @ rng.standard_normal((rank, 60))
    Q, L, P = oracle.ruqlp_paper(A, 8, 2, 0, seed=1)
    assert np.linalg.norm(Q @ L @ P.T - A) < 1e-12 * np.linalg.norm(A)


def _lapack_orth(X):
    """Q of LAPACK's QR with diag(R) >= 0 (independent of the oracle's QR)."""
    Qx, Rx = np.linalg.qr(X)
    sgn = np.where(np.diag(Rx) < 0, -1.0, 1.0)
    return Qx * sgn, Rx * sgn[:, None]


@pytest.mark.parametrize("q", [0, 2])
def test_paper_orientation_direct_steps(q):
    """The paper orientation taken directly in its own terms -- an m x d
    Gaussian, P-bar from A^T times it with power steps, QR of A P-bar, QR of
    the transposed R -- with LAPACK's QR in every step, gives the oracle's
    Q, L and P."""
    m, n, k, p = 130, 100, 10, 4
    d = k + p
    sigma = workloads.spectrum("geometric", min(m, n), rho=0.88)
    A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed=17, trunc=0.0)
    phi = oracle.gaussian_matrix(21, m, d)
    Pbar, _ = _lapack_orth(A.T @ phi)
    for _ in range(q):
        Pbar, _ = _lapack_orth(A @ Pbar)
        Pbar, _ = _lapack_orth(A.T @ Pbar)
    Qd, R = _lapack_orth(A @ Pbar)
    Pt, Rt = _lapack_orth(R.T)
    Q, L, P = oracle.ruqlp_paper(A, k, p, q, seed=21)
    assert np.linalg.norm(Q - Qd) < 1e-10
    assert np.linalg.norm(L - Rt.T) < 1e-10 * np.linalg.norm(L)
    assert np.linalg.norm(P - Pbar @ Pt) < 1e-10
