"""Pins for the oracle's CSR helpers (oracle/csr.py)."""
import numpy as np
import pytest

from oracle.csr import csr_matmul, csr_transpose, csr_to_dense
import workloads


@pytest.mark.parametrize("m,n,nnz", [(50, 40, 300), (500, 3000, 4000), (7, 9, 0), (33, 5, 165)])
def test_csr_matmul_matches_dense(m, n, nnz):
    rowptr, colidx, vals = workloads.csr_uniform(m, n, nnz, seed=m + n + nnz)
    X = np.random.default_rng(1).standard_normal((n, 6))
    D = csr_to_dense(rowptr, colidx, vals, m, n)
    Y = csr_matmul(rowptr, colidx, vals, m, n, X, block_rows=17)
    assert np.allclose(Y, D @ X, rtol=1e-13, atol=1e-13)


def test_csr_to_dense_independent_of_helper():
    # a 3 x 4 matrix written out by hand
    rowptr = np.array([0, 2, 2, 4], np.int32)
    colidx = np.array([1, 3, 0, 2], np.int32)
    vals = np.array([1.5, -2.0, 4.0, 0.25], np.float32)
    D = np.array([[0, 1.5, 0, -2.0], [0, 0, 0, 0], [4.0, 0, 0.25, 0]])
    assert np.array_equal(csr_to_dense(rowptr, colidx, vals, 3, 4), D)
    X = np.arange(8.0).reshape(4, 2)
    assert np.array_equal(csr_matmul(rowptr, colidx, vals, 3, 4, X), D @ X)
    rt, ct, vt = csr_transpose(rowptr, colidx, vals, 3, 4)
    assert rt.tolist() == [0, 1, 2, 3, 4]
    assert ct.tolist() == [2, 0, 2, 0]
    assert vt.tolist() == [4.0, 1.5, 0.25, -2.0]


@pytest.mark.parametrize("m,n,nnz", [(60, 45, 500), (1000, 20, 5000), (5, 300, 40)])
def test_csr_transpose(m, n, nnz):
    rowptr, colidx, vals = workloads.csr_uniform(m, n, nnz, seed=7 + nnz)
    rt, ct, vt = csr_transpose(rowptr, colidx, vals, m, n)
    D = csr_to_dense(rowptr, colidx, vals, m, n)
    assert np.array_equal(csr_to_dense(rt, ct, vt, n, m), D.T)
    # within each row of A^T, original row indices strictly increase
    for j in range(n):
        seg = ct[rt[j]:rt[j + 1]]
        assert np.all(np.diff(seg) > 0)


def test_csr_generator_shape():
    rowptr, colidx, vals = workloads.csr_uniform(300, 200, 600, seed=4)
    assert rowptr[0] == 0 and rowptr[-1] == 600 and np.all(np.diff(rowptr) >= 0)
    for i in range(300):
        seg = colidx[rowptr[i]:rowptr[i + 1]]
        assert np.all(np.diff(seg) > 0)
    assert colidx.min() >= 0 and colidx.max() < 200
