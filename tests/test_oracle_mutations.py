"""Plant mistakes in copies of oracle steps (on the CPU) and check that the
pins catch each one.  Nothing here touches the GPU."""
import numpy as np
import pytest

import oracle
from oracle import householder, philox, ruqlp as ruqlp_mod
import workloads
from tests import pins


def _fixture():
    sigma = workloads.spectrum("geometric", 50, rho=0.7)
    A, s, U, V = workloads.dense_from_spectrum(60, 50, sigma, seed=9, trunc=0.0)
    return A, s


def _all_pins_pass(A, s, run):
    """Run the method via `run` and evaluate the whole-method pins."""
    Q, L, Vf = run(A, 6, 2, 0)
    ok1, _ = pins.check_ruqlp_invariants(A, Q, L, Vf)
    ok2, _ = pins.check_sv_interlacing(s, L)
    Ql, _ = pins.lapack_qr_positive(A @ philox.gaussian_matrix(4, A.shape[1], 8))
    ok3 = np.linalg.norm(Q - Ql) < 1e-9
    Q, L, Vf = run(A, 6, 2, 60)
    ok4, _ = pins.check_orth_iteration_limit(L, s)
    return ok1 and ok2 and ok3 and ok4


def _core_with(mutation=None):
    """A copy of the method's steps, optionally with one planted mistake."""
    def orth_(X):
        if mutation == "sign convention dropped":
            return np.linalg.qr(X)[0]
        if mutation == "reflector scaled wrong":
            return householder.householder_qr(X)[0] * 1.001
        return oracle.orth(X)

    def run(A, k, p, q):
        m, n = A.shape
        d = k + p
        omega = philox.gaussian_matrix(4, n, d)
        if mutation == "sketch from the wrong side":
            Y = A.T[:, :n] @ omega if m == n else A[:, ::-1] @ omega
        else:
            Y = A @ omega
        Q = orth_(Y)
        for _ in range(q):
            if mutation == "no orthonormalization in power steps":
                Q = A @ (A.T @ Q)
                Q = Q / np.linalg.norm(Q)
            else:
                W = orth_(A.T @ Q)
                Q = orth_(A @ W)
        Bt = A.T @ (Y if mutation == "projection of the raw sketch" else Q)
        V, Rt = householder.householder_qr(Bt)
        L = Rt if mutation == "L not transposed" else Rt.T.copy()
        return Q, L, V
    return run


def test_unmutated_copy_passes():
    A, s = _fixture()
    assert _all_pins_pass(A, s, _core_with())
    # and the copy agrees with the oracle itself
    Q, L, V = _core_with()(A, 6, 2, 1)
    Qo, Lo, Vo = oracle.ruqlp(A, 6, 2, 1, seed=4)
    assert np.allclose(Q, Qo, atol=1e-12) and np.allclose(L, Lo, atol=1e-12)


MUTANTS = ["sign convention dropped", "reflector scaled wrong", "sketch from the wrong side",
           "no orthonormalization in power steps", "projection of the raw sketch", "L not transposed"]


@pytest.mark.parametrize("name", MUTANTS)
def test_planted_mistake_is_caught(name):
    A, s = _fixture()
    run = _core_with(name)
    try:
        caught = not _all_pins_pass(A, s, run)
    except (ValueError, np.linalg.LinAlgError, FloatingPointError):
        caught = True
    assert caught, name


def test_planted_philox_mistake_is_caught():
    # swap two words in the round: the numpy comparison must fail
    def bad_block(ctr, key):
        out = philox.philox4x64_10(ctr, key)
        return out[..., [0, 3, 2, 1]]
    bg = np.random.Philox(key=np.array([5, 7], np.uint64), counter=np.array([0, 0, 0, 0], np.uint64))
    raw = bg.random_raw(4)
    assert not np.array_equal(bad_block(np.array([[1, 0, 0, 0]], np.uint64), (5, 7))[0], raw)


# ---- the SVD-like form (Remark 1) ----

def _svd_small_with(mutation=None):
    """A copy of oracle.svdlike.svd_small, optionally with one planted mistake."""
    def svd_small(M):
        U, s, Vt = np.linalg.svd(M)
        Vb = Vt.copy() if mutation == "V-bar transposed" else Vt.T.copy()
        Ub = U.copy()
        if mutation == "ascending order":
            Ub, s, Vb = Ub[:, ::-1].copy(), s[::-1].copy(), Vb[:, ::-1].copy()
        for j in range(M.shape[1]):
            i = int(np.argmax(np.abs(Vb[:, j])))
            if Vb[i, j] < 0:
                Vb[:, j] = -Vb[:, j]
                if mutation != "sign flipped on V only":
                    Ub[:, j] = -Ub[:, j]
            if s[j] == 0.0 and mutation != "zero-sigma left vector kept":
                Ub[:, j] = 0.0
        return Ub, s, Vb
    return svd_small


def _svd_pins_pass(svd_small):
    rng = np.random.default_rng(2)
    M = np.tril(rng.standard_normal((30, 30))) + 3 * np.eye(30)
    Ub, s, Vb = svd_small(M)
    ok = np.all(np.diff(s) <= 0) and np.abs(Ub @ np.diag(s) @ Vb.T - M).max() < 1e-12
    ok = ok and all(Vb[int(np.argmax(np.abs(Vb[:, j]))), j] > 0 for j in range(30))
    # the whole form against its Q L V^T
    A, _, _, _ = workloads.dense_from_spectrum(80, 60, workloads.spectrum("geometric", 60, rho=0.8), 3, trunc=0.0)
    Q, L, V = oracle.ruqlp(A, 8, 4, 1, seed=5)
    Ub, s, Vb = svd_small(L)
    ok = ok and np.abs((Q @ Ub) @ np.diag(s) @ (V @ Vb).T - Q @ L @ V.T).max() < 1e-12
    # an exactly zero singular value has a zero left vector
    Ub, s, Vb = svd_small(np.diag([2.0, 0.0, 1.0]))
    ok = ok and s[-1] == 0.0 and np.all(Ub[:, -1] == 0.0)
    return bool(ok)


def test_svdlike_unmutated_copy_passes():
    assert _svd_pins_pass(_svd_small_with())
    M = np.tril(np.random.default_rng(4).standard_normal((12, 12))) + np.eye(12)
    for a, b in zip(_svd_small_with()(M), oracle.svd_small(M)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["V-bar transposed", "ascending order", "sign flipped on V only",
                                  "zero-sigma left vector kept"])
def test_svdlike_planted_mistake_is_caught(name):
    assert not _svd_pins_pass(_svd_small_with(name)), name
