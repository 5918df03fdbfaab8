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
