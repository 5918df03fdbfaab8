"""Parity of each step of the HIP path with the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from oracle import philox
from oracle.csr import csr_matmul, csr_transpose
import workloads
from tests.gpu_util import announce, to_dev, to_np

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------- Gaussian
@pytest.mark.parametrize("rows,cols,ld", [(37, 5, 5), (800, 25, 32), (8000, 210, 224), (1, 1, 1), (5, 3, 7)])
def test_gaussian_fp64_matches_oracle(gpu_lib, rows, cols, ld):
    announce("gaussian f64", rows, cols, ld)
    G = to_np(gpu_lib.gaussian(rows, cols, seed=1234, dtype=torch.float64, ld=ld))
    ref = philox.gaussian_matrix(1234, rows, cols)
    # same Philox words; log/sin/cos of two libraries differ by a few ulp
    assert np.allclose(G[:, :cols], ref, rtol=1e-14, atol=1e-15)
    assert np.all(G[:, cols:] == 0.0)


@pytest.mark.parametrize("rows,cols", [(8000, 210), (50000, 110)])
def test_gaussian_fp32_matches_oracle(gpu_lib, rows, cols):
    announce("gaussian f32", rows, cols)
    G = gpu_lib.gaussian(rows, cols, seed=77, dtype=torch.float32)
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    ref = philox.gaussian_matrix(77, rows, cols).astype(np.float32)
    # float32 results agree except where a few-ulp float64 difference straddles
    # a float32 rounding boundary (then they differ by one float32 ulp)
    diff = G.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64)
    assert np.abs(diff).max() <= 1
    assert np.count_nonzero(diff) <= 1e-5 * diff.size + 2


def test_gaussian_streams_differ(gpu_lib):
    a = to_np(gpu_lib.gaussian(64, 3, seed=5, stream_id=0))
    b = to_np(gpu_lib.gaussian(64, 3, seed=5, stream_id=1))
    assert np.allclose(b, philox.gaussian_matrix(5, 64, 3, stream=1), rtol=1e-14, atol=1e-15)
    assert not np.allclose(a, b)


# ---------------------------------------------------------------- GEMM
GEMM_CASES = [
    (1000, 800, 25), (129, 77, 1), (300, 200, 33), (8000, 500, 210), (257, 1031, 256), (64, 64, 64),
    (5, 3000, 7),
    # wider than one column tile: equal column passes
    (3000, 700, 300), (2000, 1500, 544), (600, 700, 530), (40, 900, 257),
]


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("m,n,d", GEMM_CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gemm_matches_matmul(gpu_lib, trans, m, n, d, dtype):
    announce("gemm", trans, m, n, d, dtype)
    rng = np.random.default_rng(m * 7 + n + d)
    A = rng.standard_normal((m, n))
    X = rng.standard_normal((m if trans else n, d))
    A_np = A.astype(np.float32) if dtype == torch.float32 else A
    X_np = X.astype(np.float32) if dtype == torch.float32 else X
    Y = to_np(gpu_lib.gemm(to_dev(A_np), to_dev(X_np), trans=trans))
    A64, X64 = A_np.astype(np.float64), X_np.astype(np.float64)
    ref = (A64.T @ X64) if trans else (A64 @ X64)
    bound = (np.abs(A64).T @ np.abs(X64)) if trans else (np.abs(A64) @ np.abs(X64))
    K = m if trans else n
    u = 2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24
    assert np.all(np.abs(Y - ref) <= 2 * K * u * bound + 1e-300)


def test_gemm_unaligned_leading_dimension(gpu_lib):
    announce("gemm unaligned lda")
    rng = np.random.default_rng(3)
    big = rng.standard_normal((300, 203)).astype(np.float32)
    Abig = to_dev(big)
    A = Abig[:, 1:200]                  # row stride 203, base not 16-byte aligned
    X = rng.standard_normal((199, 17)).astype(np.float32)
    for trans in (False, True):
        Xt = rng.standard_normal((300, 17)).astype(np.float32) if trans else X
        Y = to_np(gpu_lib.gemm(A, to_dev(Xt), trans=trans))
        A64 = big[:, 1:200].astype(np.float64)
        ref = A64.T @ Xt.astype(np.float64) if trans else A64 @ Xt.astype(np.float64)
        assert np.allclose(Y, ref, rtol=1e-4, atol=1e-4)


@pytest.mark.gpu
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("m,n,d", [(1000, 777, 37), (300, 2000, 210), (8000, 8000, 210), (129, 67, 256),
                                   (5, 3, 1), (3000, 2000, 520), (700, 300, 257)])
def test_gemm_bf16_matches_rounded_product(gpu_lib, trans, m, n, d):
    """bfloat16 products: the kernel multiplies round_bf16(A) and
    round_bf16(X) exactly and accumulates in float32, so it must match the
    float64 product of the rounded operands to float32 accumulation error."""
    from oracle.bf16 import round_bf16
    announce("gemm bf16", trans, m, n, d)
    rng = np.random.default_rng(m + 3 * n + d)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((m if trans else n, d)).astype(np.float32)
    Y = to_np(gpu_lib.gemm(to_dev(A), to_dev(X), trans=trans, bf16=True))
    Ab, Xb = round_bf16(A), round_bf16(X)
    ref = (Ab.T @ Xb) if trans else (Ab @ Xb)
    bound = (np.abs(Ab).T @ np.abs(Xb)) if trans else (np.abs(Ab) @ np.abs(Xb))
    K = m if trans else n
    # products of bfloat16 values are exact in float32; only the sums round
    assert np.all(np.abs(Y - ref) <= 2 * K * 2.0 ** -24 * bound + 1e-30)
    # and the rounding of the operands is really applied
    ref32 = (A.astype(np.float64).T @ X) if trans else (A.astype(np.float64) @ X)
    if K > 8:
        assert np.abs(Y - ref32).max() > 1e-4 * np.abs(ref32).max()


# ---------------------------------------------------------------- orth (CholeskyQR2)
def _conditioned(m, d, cond, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, d)))
    W, _ = np.linalg.qr(rng.standard_normal((d, d)))
    return (U * np.logspace(0, -np.log10(cond), d)) @ W.T


@pytest.mark.parametrize("m,d,cond", [(1000, 25, 1e3), (8000, 210, 1e4), (500, 256, 1e2), (17, 17, 10.0),
                                      (300, 1, 1.0), (4000, 110, 1e6),
                                      # d > 256: the Cholesky keeps its trailing tiles in memory
                                      (3000, 320, 1e4), (2000, 544, 1e2), (1200, 417, 1e6), (600, 257, 10.0),
                                      # diagonal blocks of 13 and 15 tile columns
                                      (1500, 400, 1e3), (2000, 470, 1e3),
                                      # tall enough for two row fragments per wave in the solve
                                      (70000, 100, 1e3), (30000, 300, 1e2)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_orth_matches_householder(gpu_lib, m, d, cond, dtype):
    announce("orth", m, d, cond, dtype)
    Y = _conditioned(m, d, cond, m + d)
    Y_in = Y.astype(np.float32) if dtype == torch.float32 else Y
    Q, R = gpu_lib.orth(to_dev(Y_in), want_r=True)
    Q, R = to_np(Q), to_np(R)
    Qo, Ro = oracle.householder_qr(Y_in.astype(np.float64))
    u_out = 2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24
    u64 = 2.0 ** -53
    # The QR is unique (diag(R) > 0).  The device computes in float64 and
    # rounds Q once to the output type, so the forward error is bounded by
    # ~cond * u64 (QR perturbation) plus the output rounding.
    tol = 100 * np.sqrt(d) * (cond * u64 + u_out)
    assert np.linalg.norm(Q.T @ Q - np.eye(d)) <= 50 * d * u_out
    assert np.linalg.norm(Q - Qo) <= tol
    assert np.linalg.norm(R - Ro) <= tol * np.linalg.norm(Ro)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) >= 0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_orth_rank_deficient_completes_basis(gpu_lib, dtype):
    announce("orth rank-deficient", dtype)
    rng = np.random.default_rng(9)
    B = rng.standard_normal((400, 6))
    Y = np.hstack([B, B @ rng.standard_normal((6, 4)), np.zeros((400, 2)), B[:, :3]])  # rank 6, d = 15
    Y_in = Y.astype(np.float32) if dtype == torch.float32 else Y
    ctx = gpu_lib.default_context(0)
    Q, R = gpu_lib.orth(to_dev(Y_in), want_r=True, ctx=ctx)
    Q, R = to_np(Q), to_np(R)
    info = ctx.info()
    d = Y.shape[1]
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert np.linalg.norm(Q.T @ Q - np.eye(d)) <= tol
    assert np.linalg.norm(Q @ R - Y_in) <= tol * np.linalg.norm(Y)
    assert info["completed_cols"] == 9 and info["breakdown_pass"] == 1
    dep = [6, 7, 8, 9, 10, 11, 12, 13, 14]
    assert np.all(R[dep, :] == 0.0)


@pytest.mark.parametrize("rows", [1500, 30000])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_orth_rank_deficient_wide(gpu_lib, dtype, rows):
    """d = 300 > 256 with 40 dependent columns spread over the column
    blocks: the wide Cholesky marks them and the solve substitutes (with
    one and with two row fragments per wave)."""
    announce("orth rank-deficient wide", dtype, rows)
    rng = np.random.default_rng(19)
    B = rng.standard_normal((rows, 260))
    cols, dep = [], []
    for c in range(260):
        cols.append(B[:, c:c + 1])
        if c % 6 == 4 and len(dep) < 40:  # a combination of the columns so far
            dep.append(len(cols))
            cols.append(B[:, : c + 1] @ rng.standard_normal((c + 1, 1)))
    Y = np.hstack(cols)
    assert Y.shape[1] == 300 and dep[0] == 5 and dep[-1] == 278
    Y_in = Y.astype(np.float32) if dtype == torch.float32 else Y
    ctx = gpu_lib.default_context(0)
    Q, R = gpu_lib.orth(to_dev(Y_in), want_r=True, ctx=ctx)
    Q, R = to_np(Q), to_np(R)
    info = ctx.info()
    d = Y.shape[1]
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert np.linalg.norm(Q.T @ Q - np.eye(d)) <= 10 * tol
    assert np.linalg.norm(Q @ R - Y_in) <= 10 * tol * np.linalg.norm(Y)
    assert info["completed_cols"] == 40 and info["breakdown_pass"] == 1
    # a dependent column is a combination of the earlier columns of Q: its
    # diagonal entry of R is exactly zero (the rest of its row is not, as
    # later columns have components along the random completing directions)
    assert np.all(np.diag(R)[dep] == 0.0)
    assert np.all(np.diag(R)[[j for j in range(d) if j not in dep]] > 0.0)


# ---------------------------------------------------------------- CSR
@pytest.mark.parametrize("m,n,nnz,d", [(1000, 700, 5000, 25), (20000, 10000, 200000, 110), (50, 40, 0, 3),
                                       (300, 5, 1200, 256)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spmm_matches_oracle(gpu_lib, m, n, nnz, d, dtype):
    announce("spmm", m, n, nnz, d, dtype)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    rowptr, colidx, vals = workloads.csr_uniform(m, n, nnz, seed=m + nnz, dtype=npdt)
    X = np.random.default_rng(1).standard_normal((n, d)).astype(npdt)
    Y = to_np(gpu_lib.spmm(to_dev(rowptr), to_dev(colidx), to_dev(vals), m, n, to_dev(X)))
    ref = csr_matmul(rowptr, colidx, vals, m, n, X)
    u = 2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24
    absbound = csr_matmul(rowptr, colidx, np.abs(vals), m, n, np.abs(X))
    maxrow = max(1, int(np.diff(rowptr).max())) if m else 1
    assert np.all(np.abs(Y - ref) <= 2 * maxrow * u * absbound)


@pytest.mark.parametrize("m,n,nnz", [(1000, 700, 5000), (100000, 50000, 5000000), (40, 3, 0), (7, 1, 7)])
def test_csr_transpose_bit_exact(gpu_lib, m, n, nnz):
    announce("csr transpose", m, n, nnz)
    rowptr, colidx, vals = workloads.csr_uniform(m, n, nnz, seed=11)
    rt, ct, vt = gpu_lib.csr_transpose(to_dev(rowptr), to_dev(colidx), to_dev(vals), m, n)
    torch.cuda.synchronize()
    rt_o, ct_o, vt_o = csr_transpose(rowptr, colidx, vals, m, n)
    assert np.array_equal(rt.cpu().numpy(), rt_o)
    assert np.array_equal(ct.cpu().numpy(), ct_o)
    assert np.array_equal(vt.cpu().numpy().view(np.uint32), vt_o.astype(np.float32).view(np.uint32))
