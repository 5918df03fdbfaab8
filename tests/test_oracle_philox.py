"""Pins for the oracle's Gaussian generator (oracle/philox.py)."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 0x52514C50), (123456789, 2**63 + 11)])
@pytest.mark.parametrize("start", [0, 1, 2**32 - 1, 2**40 + 3])
def test_block_function_matches_numpy_philox(key, start):
    # numpy's Philox bit generator implements the same published block
    # function; it advances the counter before each block, so its output for
    # counter c is the block function at c + 1.
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=[start, 0, 0, 0])
    raw = bg.random_raw(4 * 5).reshape(5, 4)
    ctr = np.zeros((5, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(start + 1, start + 6, dtype=np.uint64)
    mine = philox.philox4x64_10(ctr, key)
    assert np.array_equal(mine, raw)


def test_block_function_counter_carry_matches_numpy():
    # counter word 0 wraps into word 1
    bg = np.random.Philox(key=np.array([9, 9], np.uint64), counter=np.array([2**64 - 1, 4, 0, 0], np.uint64))
    raw = bg.random_raw(4)
    mine = philox.philox4x64_10(np.array([[0, 5, 0, 0]], dtype=np.uint64), (9, 9))
    assert np.array_equal(mine[0], raw)


def test_uniform_ranges_and_endpoints():
    w = np.array([0, 2**64 - 1, 2**11 - 1, 2**11], dtype=np.uint64)
    u1, u2 = philox.uniform_pair(w, w)
    assert u1.min() > 0.0 and u1.max() <= 1.0
    assert u2.min() >= 0.0 and u2.max() < 1.0
    assert u1[0] == 2.0 ** -53 and u2[0] == 0.0
    assert u1[1] == 1.0 and u2[1] == 1.0 - 2.0 ** -53
    assert u2[2] == 0.0 and u2[3] == 2.0 ** -53


def test_box_muller_closed_forms():
    # u1 = 1 gives radius 0; u2 = 0 and 1/4 put all mass on one output.
    z0, z1 = philox.box_muller(np.array([1.0, np.exp(-0.5), np.exp(-2.0)]),
                               np.array([0.3, 0.0, 0.25]))
    assert z0[0] == 0.0 and z1[0] == 0.0
    assert z0[1] == pytest.approx(1.0, abs=1e-15) and z1[1] == 0.0
    assert z0[2] == pytest.approx(0.0, abs=1e-15) and z1[2] == pytest.approx(2.0, abs=1e-15)


def test_gaussian_matrix_index_map():
    n, d, seed = 37, 5, 99
    G = philox.gaussian_matrix(seed, n, d)
    assert G.shape == (n, d)
    for (i, j) in [(0, 0), (1, 0), (36, 0), (0, 1), (7, 3), (36, 4)]:
        l = j * n + i
        blk = philox.philox4x64_10(np.array([[l // 4, 0, 0, 0]], np.uint64), (seed, philox.SKETCH_KEY1))[0]
        pair = (l % 4) // 2
        u1, u2 = philox.uniform_pair(blk[2 * pair], blk[2 * pair + 1])
        z = philox.box_muller(u1, u2)[l % 2]
        assert G[i, j] == z


def test_gaussian_distribution():
    G = philox.gaussian_matrix(2024, 1000, 600).ravel()
    N = G.size
    assert abs(G.mean()) < 5 / np.sqrt(N)
    assert abs(G.var() - 1.0) < 5 * np.sqrt(2.0 / N)
    assert abs(stats.skew(G)) < 5 * np.sqrt(6.0 / N)
    assert abs(stats.kurtosis(G)) < 5 * np.sqrt(24.0 / N)
    assert stats.kstest(G, "norm").pvalue > 1e-4
    # tails: P(|z| > 3) = 0.0026998
    frac = np.mean(np.abs(G) > 3.0)
    assert abs(frac - 0.0026998) < 6 * np.sqrt(0.0027 / N)


def test_streams_and_seeds_differ():
    a = philox.gaussian_matrix(1, 64, 3)
    b = philox.gaussian_matrix(2, 64, 3)
    c = philox.gaussian_matrix(1, 64, 3, stream=1)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(a, philox.gaussian_matrix(1, 64, 3))
