"""Pins for the oracle's error metrics (oracle/metrics.py)."""
import numpy as np

from oracle import metrics
import workloads


def test_recon_diff_and_error_match_dense():
    rng = np.random.default_rng(2)
    m, n, d = 130, 90, 7
    Qa, La, Va = rng.standard_normal((m, d)), np.tril(rng.standard_normal((d, d))), rng.standard_normal((n, d))
    Qb, Lb, Vb = rng.standard_normal((m, d)), np.tril(rng.standard_normal((d, d))), rng.standard_normal((n, d))
    ref = np.linalg.norm(Qa @ La @ Va.T - Qb @ Lb @ Vb.T)
    assert abs(metrics.recon_diff(Qa, La, Va, Qb, Lb, Vb, block_rows=11) - ref) <= 1e-12 * ref
    A = rng.standard_normal((m, n))
    ref = np.linalg.norm(A - Qa @ La @ Va.T) / np.linalg.norm(A)
    assert abs(metrics.recon_error(A, Qa, La, Va, block_rows=13) - ref) <= 1e-12 * ref
    assert abs(metrics.orth_error(Qa) - np.linalg.norm(Qa.T @ Qa - np.eye(d))) < 1e-10


def test_recon_error_csr_matches_dense():
    from oracle.csr import csr_to_dense
    rowptr, colidx, vals = workloads.csr_uniform(70, 50, 400, seed=1)
    rng = np.random.default_rng(0)
    Q, L, V = rng.standard_normal((70, 4)), np.tril(rng.standard_normal((4, 4))), rng.standard_normal((50, 4))
    D = csr_to_dense(rowptr, colidx, vals, 70, 50)
    ref = np.linalg.norm(D - Q @ L @ V.T) / np.linalg.norm(D)
    got = metrics.recon_error_csr(rowptr, colidx, vals, 70, 50, Q, L, V, block_rows=9)
    assert abs(got - ref) <= 1e-12 * ref


def test_optimal_error_matches_svd_of_matrix():
    A = np.random.default_rng(4).standard_normal((40, 30))
    U, s, Vt = np.linalg.svd(A)
    for r in [0, 1, 5, 29]:
        Ar = (U[:, :r] * s[:r]) @ Vt[:r]
        assert abs(metrics.optimal_error(s, r, "fro") - np.linalg.norm(A - Ar)) < 1e-12 * np.linalg.norm(A)
        assert abs(metrics.optimal_error(s, r, 2) - np.linalg.norm(A - Ar, 2)) < 1e-12 * np.linalg.norm(A)
