"""rqlp_decompose_noalloc (the entry point that allocates nothing) against
rqlp_decompose on the same inputs: bitwise equal results, on calls in a row
whose later inputs are smaller, also after a call that filled the scratch
array with non-finite values."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


def _case(m, n, rho, seed, dtype):
    sigma = workloads.spectrum("geometric", min(m, n), rho=rho)
    A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed=seed, trunc=0.0)
    return to_dev(A.astype(dtype))


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_matches_decompose(gpu_lib, dtype):
    announce("noalloc vs decompose", dtype)
    ctx = gpu_lib.Context(0)
    cases = [(2600, 2100, 180, 12, 1), (900, 700, 40, 8, 0), (1500, 1300, 100, 10, 2)]
    for i, (m, n, k, p, q) in enumerate(cases):
        A = _case(m, n, 0.98, 10 + i, dtype)
        ref = [x.clone() for x in gpu_lib.decompose(A, k, p, q, seed=5 + i, ctx=ctx)]
        got = gpu_lib.decompose_noalloc(A, k, p, q, seed=5 + i, ctx=ctx)
        torch.cuda.synchronize()
        assert _same(got, ref), f"case {i} ({m}x{n}, k={k}, p={p}, q={q}) differs"
    # fill the scratch array with NaN / Inf by a call on a poisoned input,
    # then a smaller clean call must still give the reference bits
    Ap = _case(2600, 2100, 0.98, 20, dtype)
    Ap[::7, ::5] = float("nan")
    Ap[3::11, 2::9] = float("inf")
    gpu_lib.decompose_noalloc(Ap, 200, 10, 1, seed=1, ctx=ctx)
    torch.cuda.synchronize()
    A = _case(700, 650, 0.97, 21, dtype)
    ref = [x.clone() for x in gpu_lib.decompose(A, 50, 6, 1, seed=2, ctx=ctx)]
    got = gpu_lib.decompose_noalloc(A, 50, 6, 1, seed=2, ctx=ctx)
    torch.cuda.synchronize()
    assert _same(got, ref)
    assert ctx.info()["nonfinite"] == 0
    ctx.close()


def test_noalloc_rejects_oversized(gpu_lib):
    announce("noalloc rejects oversized")
    lib = gpu_lib._lib()
    m = n = 20000
    assert lib.rqlp_workspace_size(m, n, 500, 20, 1, 1) > gpu_lib.NOALLOC_SCRATCH_BYTES
    ctx = gpu_lib.Context(0)
    A = torch.zeros(8, device="cuda")
    out = torch.full((8,), 3.0, device="cuda")
    P = ctypes.c_void_p
    st = lib.rqlp_decompose_noalloc(ctx.handle, P(A.data_ptr()), m, n, n, 500, 20, 1, 1, 0, P(out.data_ptr()),
                                    P(out.data_ptr()), P(out.data_ptr()), None)
    assert st == 3  # RQLP_ERR_OUT_OF_MEMORY, nothing enqueued
    torch.cuda.synchronize()
    assert bool(torch.all(out == 3.0))
    ctx.close()
