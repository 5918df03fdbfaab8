"""Pins for the oracle's bfloat16 rounding (oracle/bf16.py)."""
import numpy as np

from oracle.bf16 import round_bf16


def test_representable_values_are_fixed_points():
    vals = np.array([0.0, -0.0, 1.0, 1.5, -2.75, 2.0 ** -20, 3.0 * 2.0 ** 100, 1.0 + 2.0 ** -7])
    assert np.array_equal(round_bf16(vals), vals)


def test_ties_to_even_and_nearest():
    one = 1.0
    h = 2.0 ** -8                                     # half a bf16 ulp at 1
    assert round_bf16(one + h) == 1.0                 # tie -> even (1.0)
    assert round_bf16(one + 3 * h) == 1.0 + 2.0 ** -6  # tie -> even (lsb 0)
    assert round_bf16(one + 1.1 * h) == 1.0 + 2.0 ** -7
    assert round_bf16(one + 0.9 * h) == 1.0
    assert round_bf16(-(one + 1.1 * h)) == -(1.0 + 2.0 ** -7)


def test_spacing_and_overflow():
    x = np.random.default_rng(0).uniform(1.0, 2.0, 10000)
    r = round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 + 2.0 ** -23)  # via binary32
    assert np.all(np.round(r * 2 ** 7) == r * 2 ** 7)
    assert np.isinf(round_bf16(np.array([3.4e38]))[0])
    assert np.isnan(round_bf16(np.array([np.nan]))[0])
