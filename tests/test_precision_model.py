"""Pins of the accumulation-error model behind the factor-level gates
(tests/fp32_model.py), on the CPU."""
import numpy as np

import oracle
from oracle.metrics import recon_diff
import workloads
from tests.fp32_model import U32, factor_deviation, noisy_product, ruqlp_model


def test_model_noise_bounds_a_real_float32_product():
    """A float32 matrix product (numpy / BLAS sgemm, float32 accumulation)
    stays within the model's noise scale: its RMS error, in units of the
    model's standard deviation, is at most 1 (the model assumes one long
    sequential sum; blocked sums err less)."""
    rng = np.random.default_rng(0)
    for m, K, d in ((1000, 3000, 64), (300, 8000, 32)):
        A = rng.standard_normal((m, K)).astype(np.float32)
        X = rng.standard_normal((K, d)).astype(np.float32)
        Y32 = (A @ X).astype(np.float64)
        A64, X64 = A.astype(np.float64), X.astype(np.float64)
        Y = A64 @ X64
        sd = np.sqrt((A64 * A64) @ (X64 * X64)) * U32 * np.sqrt(K / 6.0)
        assert np.sqrt(np.mean(((Y32 - Y) / sd) ** 2)) <= 1.0
        # and the model's own noise has unit RMS in those units
        Yn = noisy_product(A64, X64, np.random.default_rng(1))
        r = np.sqrt(np.mean(((Yn - Y) / sd) ** 2))
        assert 0.8 <= r <= 1.2


def _small_case():
    c = workloads.cfg_gapped_fp32(seed=5, m=700, n=600, q=1)
    A = c["A"].astype(np.float64)
    return A, oracle.ruqlp(A, 40, 8, 1, 3, omega_dtype="f32"), ruqlp_model(A, 40, 8, 1, 3)


def test_independent_model_draws_pass_the_gate():
    """Two independent draws of the model lie within the gate of each other:
    the gate's factor C leaves room for the device's own draw."""
    A, ref, m1 = _small_case()
    m2 = ruqlp_model(A, 40, 8, 1, 3, rng_seed=99)
    rep = factor_deviation(m2, ref, m1)
    assert rep["ok"], rep
    assert rep["Q"]["informative_cols"] == 48 and rep["V"]["informative_cols"] == 48


def test_gate_catches_what_delta_cannot():
    """A sign flip shared by column j of Q and row j of L leaves Q L V^T (so
    Delta) unchanged, and a swap of two columns of V with the matching
    columns of L too; the factor gate fails both.  A perturbation of one L
    entry well beyond the model's spread fails it as well."""
    A, ref, model = _small_case()
    Q, L, V = (x.copy() for x in ref)
    Q[:, 5] *= -1.0
    L[5, :] *= -1.0
    assert recon_diff(Q, L, V, *ref) <= 1e-12 * np.linalg.norm(A)
    assert not factor_deviation((Q, L, V), ref, model)["ok"]
    Q, L, V = (x.copy() for x in ref)
    V[:, [3, 4]] = V[:, [4, 3]]
    L[:, [3, 4]] = L[:, [4, 3]]
    assert recon_diff(Q, L, V, *ref) <= 1e-12 * np.linalg.norm(A)
    assert not factor_deviation((Q, L, V), ref, model)["ok"]
    Q, L, V = (x.copy() for x in ref)
    L[30, 10] += 1e-4
    assert not factor_deviation((Q, L, V), ref, model)["ok"]
