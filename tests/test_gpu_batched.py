"""Batched decompositions (rqlp_decompose_batched): every result is bitwise
the solo rqlp_decompose result of the same problem, with and without graph
replay, and the solo path is itself parity-tested against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle.metrics import recon_diff
import workloads
from tests.gpu_util import announce, to_dev, to_np

pytestmark = pytest.mark.gpu


def _batch(dtype, count=7, seed=5, q=1):
    reqs = workloads.serving_requests(count, seed, m_range=(64, 1500), n_range=(40, 900), kmax=120)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    As = [to_dev(workloads.request_matrix(r, npdt)) for r in reqs]
    params = [(r["k"], r["p"], q, r["seed"]) for r in reqs]
    return reqs, As, params


def _solo(gpu_lib, As, params, bf16=False):
    out = []
    for A, (k, p, q, seed) in zip(As, params):
        out.append(tuple(x.clone() for x in gpu_lib.decompose(A, k, p, q, seed=seed, bf16=bf16)))
    return out


def _same(outs, ref):
    for (Q, L, V), (Qr, Lr, Vr) in zip(outs, ref):
        assert torch.equal(Q, Qr) and torch.equal(L, Lr) and torch.equal(V, Vr)


@pytest.mark.parametrize("grouped", [True, False])
@pytest.mark.parametrize("dtype,bf16", [(torch.float32, False), (torch.float64, False), (torch.float32, True)])
def test_batched_equals_solo(gpu_lib, dtype, bf16, grouped):
    announce("batched vs solo", dtype, bf16, "grouped" if grouped else "streams")
    reqs, As, params = _batch(dtype)
    ref = _solo(gpu_lib, As, params, bf16)
    ctx = gpu_lib.Context(0)
    ctx.set_batch_grouping(grouped)
    outs = gpu_lib.decompose_batched(As, params, ctx=ctx, bf16=bf16)
    torch.cuda.synchronize()
    _same(outs, ref)
    # and the first problem against the oracle (the solo path's own gate)
    if not bf16:
        A64 = to_np(As[0]).astype(np.float64)
        k, p, q, seed = params[0]
        Qo, Lo, Vo = oracle.ruqlp(A64, k, p, q, seed, omega_dtype="f32" if dtype == torch.float32 else "f64")
        delta = recon_diff(*(to_np(x) for x in outs[0]), Qo, Lo, Vo) / np.linalg.norm(A64)
        assert delta <= (1e-5 if dtype == torch.float32 else 1e-12)


def test_graph_replays_match_eager(gpu_lib):
    """A batch submitted repeatedly is captured on its second submission and
    replayed afterwards; every replay, with other device work and
    synchronizations in between, gives the eager results bitwise."""
    announce("batched graph replay")
    reqs, As, params = _batch(torch.float32, count=6, seed=11)
    ref = _solo(gpu_lib, As, params)
    ctx = gpu_lib.Context(0)
    ctx.set_graphs(True)
    outs = [tuple(torch.empty_like(x) for x in r) for r in ref]
    ws = gpu_lib.alloc_workspace(gpu_lib.workspace_size_batched(
        [(A.shape[0], A.shape[1], k, p, q) for A, (k, p, q, s) in zip(As, params)], torch.float32), As[0].device)
    junk = torch.randn(512, 512, device=As[0].device)
    for rep in range(5):  # eager, capture + replay, then replays
        for o in outs:
            for x in o:
                x.fill_(float("nan"))
        junk = junk @ junk.T * 1e-3  # unrelated eager work between submissions
        gpu_lib.decompose_batched(As, params, ctx=ctx, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        _same(outs, ref)
    # a changed descriptor is not replayed from the old graph
    params2 = [(k, p, q, s + 1) for (k, p, q, s) in params]
    ref2 = _solo(gpu_lib, As, params2)
    for rep in range(3):
        gpu_lib.decompose_batched(As, params2, ctx=ctx, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        _same(outs, ref2)


def test_grouped_mixed_classes_and_blocked(gpu_lib):
    """Grouped factorizations across every register-slot class, more
    problems than one grouped launch holds, unequal q (problems leave the
    lockstep at different segments), a dependent-column problem and one
    blocked (d > 256) factorization: bitwise the solo results."""
    announce("grouped mixed classes")
    rng = np.random.default_rng(7)
    As, params = [], []
    ks = [6, 20, 50, 90, 120, 150, 200, 240, 250] * 3 + [300]
    for i, k in enumerate(ks):
        m, n = int(rng.integers(k + 40, k + 700)), int(rng.integers(k + 20, k + 400))
        A = rng.standard_normal((m, n)).astype(np.float32)
        As.append(to_dev(A))
        params.append((k, 10 if k < 300 else 4, i % 3, 100 + i))
    # rank 2 with k + p = 6: dependent columns in every pass
    As.append(to_dev((np.outer(np.arange(1.0, 61.0), np.ones(40)) + np.outer(np.ones(60), np.arange(40.0)))
                     .astype(np.float32)))
    params.append((4, 2, 1, 9))
    ref = _solo(gpu_lib, As, params)
    ctx = gpu_lib.Context(0)
    ws = gpu_lib.alloc_workspace(gpu_lib.workspace_size_batched(
        [(A.shape[0], A.shape[1], k, p, q) for A, (k, p, q, s) in zip(As, params)], torch.float32), As[0].device)
    outs = [tuple(torch.empty_like(x) for x in r) for r in ref]
    for rep in range(2):  # the same workspace twice
        for o in outs:
            for x in o:
                x.fill_(float("nan"))
        gpu_lib.decompose_batched(As, params, ctx=ctx, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        _same(outs, ref)


def test_batched_info_covers_batch(gpu_lib):
    announce("batched info")
    reqs, As, params = _batch(torch.float64, count=3, seed=2, q=0)
    # a rank-2 problem with k + p = 6: four completed columns per orth
    A = to_dev(np.outer(np.arange(1.0, 51.0), np.ones(30)) + np.outer(np.ones(50), np.arange(30.0)))
    As.append(A)
    params.append((4, 2, 0, 9))
    ctx = gpu_lib.Context(0)
    gpu_lib.decompose_batched(As, params, ctx=ctx)
    torch.cuda.synchronize()
    info = ctx.info()
    assert info["completed_cols"] > 0 and info["nonfinite"] == 0


def test_grouped_plan_cache_reuse_and_eviction(gpu_lib):
    """Grouped batches keep their argument tables per batch descriptor: the
    same batch again reuses them, and more distinct batches than the cache
    holds evict the oldest; every call gives the solo results bitwise."""
    announce("grouped plan cache")
    reqs, As, params = _batch(torch.float32, count=5, seed=17)
    ctx = gpu_lib.Context(0)
    ws = gpu_lib.alloc_workspace(gpu_lib.workspace_size_batched(
        [(A.shape[0], A.shape[1], k, p, q) for A, (k, p, q, s) in zip(As, params)], torch.float32), As[0].device)
    outs = [(torch.empty((A.shape[0], k + p), device=A.device), torch.empty((k + p, k + p), device=A.device),
             torch.empty((A.shape[1], k + p), device=A.device)) for A, (k, p, q, s) in zip(As, params)]
    for rep in range(11):  # ten distinct descriptors, the first one again at the end
        shift = rep % 10
        ps = [(k, p, q, s + shift) for (k, p, q, s) in params]
        gpu_lib.decompose_batched(As, ps, ctx=ctx, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        if rep in (0, 3, 9, 10):
            _same(outs, _solo(gpu_lib, As, ps))


def test_large_batch_equals_solo(gpu_lib):
    """A batch of 60 problems (three lockstep groups of 20) gives the bits of
    every solo run.  The shapes cover several column widths, both products,
    alignment of the leading dimension, and a wide sketch (d > 256, two
    column passes)."""
    announce("large batch")
    rng = np.random.default_rng(7)
    As, params = [], []
    for i in range(60):
        m = int(rng.integers(3600, 4600))
        n = int(rng.integers(500, 900))
        k = [10, 40, 90, 150, 280][i % 5]
        if k + 10 > min(m, n):
            k = min(m, n) - 10
        A = rng.standard_normal((m, n)).astype(np.float32)
        As.append(to_dev(A))
        params.append((k, 10, 1, 1000 + i))
    ref = _solo(gpu_lib, As, params)
    ctx = gpu_lib.Context(0)
    outs = gpu_lib.decompose_batched(As, params, ctx=ctx)
    torch.cuda.synchronize()
    _same(outs, ref)

