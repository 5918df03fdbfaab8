"""Checks that pin the oracle to facts other than itself.

Each check returns (ok, detail).  The pin tests assert them on the oracle;
the mutation tests plant a mistake in a copy of an oracle step and assert
that at least one check then fails.
"""

import numpy as np


def check_qr(X, Q, R, tol=1e-13):
    """Q orthonormal, R upper triangular with diag >= 0, Q R = X."""
    d = R.shape[0]
    scale = max(1.0, float(np.linalg.norm(X)))
    e_orth = float(np.linalg.norm(Q.T @ Q - np.eye(d)))
    e_tri = float(np.abs(np.tril(R, -1)).max()) if d > 1 else 0.0
    e_diag = float(-min(0.0, np.diag(R).min()))
    e_rec = float(np.linalg.norm(Q @ R - X)) / scale
    ok = e_orth <= tol * max(10, d) and e_tri == 0.0 and e_diag == 0.0 and e_rec <= tol * max(10, d)
    return ok, dict(orth=e_orth, tri=e_tri, diag=e_diag, rec=e_rec)


def lapack_qr_positive(X):
    """LAPACK QR with the columns flipped so that diag(R) >= 0."""
    Q, R = np.linalg.qr(np.asarray(X, dtype=np.float64))
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def check_ruqlp_invariants(A, Q, L, V, tol=1e-12):
    """Orthonormal Q, V; lower triangular L with diag >= 0; L V^T = Q^T A."""
    A = np.asarray(A, dtype=np.float64)
    d = L.shape[0]
    nA = max(float(np.linalg.norm(A)), 1e-300)
    e_q = float(np.linalg.norm(Q.T @ Q - np.eye(d)))
    e_v = float(np.linalg.norm(V.T @ V - np.eye(d)))
    e_tri = float(np.abs(np.triu(L, 1)).max()) if d > 1 else 0.0
    e_diag = float(-min(0.0, np.diag(L).min()))
    e_proj = float(np.linalg.norm(L @ V.T - Q.T @ A)) / nA
    ok = e_q <= tol * d and e_v <= tol * d and e_tri == 0.0 and e_diag == 0.0 and e_proj <= tol * d
    return ok, dict(q=e_q, v=e_v, tri=e_tri, diag=e_diag, proj=e_proj)


def check_sv_interlacing(A_sigma, L, rel=1e-10):
    """sigma_i(L) <= sigma_i(A) (Corollary 1, first inequality)."""
    sl = np.linalg.svd(L, compute_uv=False)
    sa = np.zeros(len(sl))
    s = np.sort(np.asarray(A_sigma))[::-1]
    sa[:min(len(s), len(sl))] = s[:len(sl)]
    viol = float(np.max(sl - sa * (1 + rel) - rel * (s[0] if len(s) else 0)))
    return viol <= 0.0, dict(max_violation=viol)


def principal_sines(Basis, Sub):
    """Sines of the principal angles between range(Sub) (k columns) and
    range(Basis) (orthonormal, d >= k columns), increasing."""
    R = Sub - Basis @ (Basis.T @ Sub)
    return np.sort(np.linalg.svd(R, compute_uv=False))


def theorem_quantities(Omega, Vfull_k, sigma, k):
    """||Omega2 Omega1^+||_2 with Omega1 = V_k^T Omega, Omega2 = V_perp^T Omega,
    delta_i = sigma_{k+1}/sigma_i, gamma = sigma_min/sigma_1."""
    O1 = Vfull_k.T @ Omega
    O2_full = Omega - Vfull_k @ O1           # V_perp V_perp^T Omega
    pinv = np.linalg.pinv(O1)
    nrm = float(np.linalg.norm(O2_full @ pinv, 2))
    s = np.asarray(sigma, dtype=np.float64)
    delta = s[k] / s[:k]
    gamma = float(s[-1] / s[0])
    return nrm, delta, gamma


def check_theorem_bounds(A, sigma_full, U_k, V_k, Omega, Q, V, k, q, slack=1e-9):
    """Theorem 2 (angle bounds) and Theorem 5 (error bound, the P form), with
    the roles of the singular vectors swapped because the sketch multiplies
    A from the right: range(Q) approximates range(U_k) with the exponent
    2q+1 bound, range(V) approximates range(V_k) with the 2q+2 bound."""
    nrm, delta, gamma = theorem_quantities(Omega, V_k, sigma_full, k)
    res = {}
    # sin of angles between range(Q) and range(U_k): exponent 2q+1
    sq = principal_sines(Q, U_k)
    bq = delta ** (2 * q + 1) * nrm / np.sqrt(1 + delta ** (4 * q + 2) * nrm ** 2)
    res["phi"] = float(np.max(sq - np.sort(bq)))
    sv = principal_sines(V, V_k)
    bv = delta ** (2 * q + 2) * nrm / np.sqrt(1 + delta ** (4 * q + 4) * nrm ** 2)
    res["theta"] = float(np.max(sv - np.sort(bv)))
    A = np.asarray(A, dtype=np.float64)
    E = A - Q @ (Q.T @ A)
    s = np.asarray(sigma_full)
    tail2, tailF = float(s[k]), float(np.sqrt(np.sum(s[k:] ** 2)))
    fac = 1 + delta[-1] ** (2 * q) * nrm / (1 + gamma ** (4 * q + 2) * nrm ** 2)
    res["err2"] = float(np.linalg.norm(E, 2) - fac * tail2)
    res["errF"] = float(np.linalg.norm(E) - fac * tailF)
    ok = all(v <= slack for v in res.values())
    return ok, res


def check_orth_iteration_limit(L, sigma, tol=1e-12):
    """q -> infinity (orthogonal iteration, Section III-C): L -> diag(sigma)."""
    d = L.shape[0]
    s = np.asarray(sigma[:d])
    e_diag = float(np.max(np.abs(np.diag(L) / s - 1.0)))
    off = L - np.diag(np.diag(L))
    e_off = float(np.abs(off).max() / s[0]) if d > 1 else 0.0
    return (e_diag <= tol and e_off <= tol), dict(diag=e_diag, off=e_off)
