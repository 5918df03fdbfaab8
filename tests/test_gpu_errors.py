"""Argument and workspace errors of the method entry points, through the C
ABI with a real context: each returns its status synchronously and leaves
the outputs untouched (nothing is enqueued)."""
import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

OK, INVALID, UNSUPPORTED, OOM = 0, 1, 2, 3
FP32 = 1


def _buffers(m, n, d, dev):
    A = torch.randn(m, n, device=dev)
    outs = [torch.full((m, d), 7.0, device=dev), torch.full((d, d), 7.0, device=dev),
            torch.full((n, d), 7.0, device=dev)]
    return A, outs


def _dense(lib, ctx, A, m, n, lda, k, p, q, outs, ws, ws_bytes):
    P = ctypes.c_void_p
    return lib.rqlp_decompose(ctx.handle, P(A.data_ptr()), m, n, lda, k, p, q, FP32, 1,
                              P(outs[0].data_ptr()), P(outs[1].data_ptr()), P(outs[2].data_ptr()),
                              P(ws.data_ptr()) if ws is not None else None, ws_bytes,
                              P(torch.cuda.current_stream().cuda_stream))


def _untouched(outs):
    torch.cuda.synchronize()
    return all(bool(torch.all(o == 7.0)) for o in outs)


def test_dense_errors(gpu_lib):
    announce("errors: rqlp_decompose")
    lib = gpu_lib._lib()
    ctx = gpu_lib.Context(0)
    dev = torch.device("cuda", 0)
    m, n, k, p, q = 600, 560, 40, 10, 1
    A, outs = _buffers(m, n, k + p, dev)
    need = lib.rqlp_workspace_size(m, n, k, p, q, FP32)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    # workspace one byte short
    assert _dense(lib, ctx, A, m, n, n, k, p, q, outs, ws, need - 1) == OOM
    # lda < n
    assert _dense(lib, ctx, A, m, n, n - 1, k, p, q, outs, ws, need) == INVALID
    # d > min(m, n)
    assert _dense(lib, ctx, A, m, n, n, n, 1, q, outs, ws, need) == INVALID
    # k < 1, p < 0, q < 0
    assert _dense(lib, ctx, A, m, n, n, 0, p, q, outs, ws, need) == INVALID
    assert _dense(lib, ctx, A, m, n, n, k, -1, q, outs, ws, need) == INVALID
    assert _dense(lib, ctx, A, m, n, n, k, p, -1, outs, ws, need) == INVALID
    assert _untouched(outs)
    # d > 544 (valid request this build does not cover)
    A2, outs2 = _buffers(700, 600, 550, dev)
    assert _dense(lib, ctx, A2, 700, 600, 600, 540, 10, 0, outs2, None, 0) == UNSUPPORTED
    assert _untouched(outs2)
    # and the exact size works
    assert _dense(lib, ctx, A, m, n, n, k, p, q, outs, ws, need) == OK
    torch.cuda.synchronize()
    assert not _untouched(outs)
    ctx.close()


def test_csr_errors(gpu_lib):
    announce("errors: rqlp_decompose_csr")
    lib = gpu_lib._lib()
    ctx = gpu_lib.Context(0)
    dev = torch.device("cuda", 0)
    m, n, k, p, q = 500, 400, 30, 5, 1
    rng = np.random.default_rng(1)
    dense = (rng.random((m, n)) < 0.02) * rng.standard_normal((m, n))
    rows, cols = np.nonzero(dense)
    rowptr = torch.tensor(np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m))]).astype(np.int32),
                          device=dev)
    colidx = torch.tensor(cols.astype(np.int32), device=dev)
    vals = torch.tensor(dense[rows, cols].astype(np.float32), device=dev)
    nnz = int(colidx.numel())
    P = ctypes.c_void_p

    def call(kk, pp, outs, ws, ws_bytes, mm=m, nn=n):
        return lib.rqlp_decompose_csr(ctx.handle, P(rowptr.data_ptr()), P(colidx.data_ptr()), P(vals.data_ptr()),
                                      mm, nn, nnz, kk, pp, q, FP32, 1, P(outs[0].data_ptr()),
                                      P(outs[1].data_ptr()), P(outs[2].data_ptr()),
                                      P(ws.data_ptr()) if ws is not None else None, ws_bytes,
                                      P(torch.cuda.current_stream().cuda_stream))

    _, outs = _buffers(m, n, k + p, dev)
    need = lib.rqlp_workspace_size_csr(m, n, nnz, k, p, q, FP32)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    assert call(k, p, outs, ws, need - 1) == OOM
    assert call(n, 1, outs, ws, need) == INVALID              # d > min(m, n)
    assert _untouched(outs)
    _, outs_w = _buffers(m, n, 260, dev)
    assert call(250, 10, outs_w, None, 0) == UNSUPPORTED      # d > 256 for CSR
    assert lib.rqlp_workspace_size_csr(m, n, nnz, 250, 10, q, FP32) == 0
    assert _untouched(outs_w)
    assert call(k, p, outs, ws, need) == OK
    torch.cuda.synchronize()
    assert not _untouched(outs)
    ctx.close()
