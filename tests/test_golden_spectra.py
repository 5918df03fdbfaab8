"""The spectrum builder and the optimal-error helper reproduce the SVD
curves printed in the paper (Section V-B figures; tests/golden)."""
import os

import numpy as np

from oracle.metrics import optimal_error
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _load():
    rows = []
    with open(os.path.join(HERE, "golden", "svd_error_curves.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, norm, r, val = line.split()
            rows.append((name, norm, int(r), float(val)))
    return rows


def test_printed_svd_error_curves():
    rows = _load()
    assert len(rows) == 64
    n, k = 800, 16
    for name, norm, r, val in rows:
        z = 1 if name == "SlowDecay" else 2
        sigma = workloads.spectrum("lowrank_decay", n, k=k, z=z)
        got = optimal_error(sigma, r, 2 if norm == "2" else "fro")
        # the paper prints 15 significant digits
        assert abs(got - val) <= 2e-15 * max(1.0, abs(val)) + 1e-15 * 10, (name, norm, r, got, val)
