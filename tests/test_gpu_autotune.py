"""The split-K autotuner (rqlp_autotune): tuned plans keep parity with the
oracle, are reproducible bit for bit through save / load, and clearing the
table returns the default plans."""
import numpy as np
import pytest
import torch

import oracle
from oracle.metrics import recon_diff
import workloads
from tests.gpu_util import announce, to_dev, to_np

pytestmark = pytest.mark.gpu


def _matrix(m, n, dtype, seed=4):
    sigma = workloads.spectrum("geometric", min(m, n), rho=0.98)
    A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed, trunc=0.0)
    return to_dev(A, dtype)


@pytest.mark.parametrize("m,n,k,p,dtype", [(3000, 2000, 100, 10, torch.float32), (1500, 1200, 60, 4, torch.float64)])
def test_tuned_plans_keep_parity_and_roundtrip(gpu_lib, tmp_path, m, n, k, p, dtype):
    announce("autotune", m, n, k, p, dtype)
    A = _matrix(m, n, dtype)
    q, seed = 1, 12
    ctx = gpu_lib.Context(0)
    nn, tn = ctx.autotune(A, k + p)
    assert nn >= 1 and tn >= 1 and ctx.autotune_count() == 2
    tuned = [x.clone() for x in gpu_lib.decompose(A, k, p, q, seed=seed, ctx=ctx)]
    # parity with the oracle holds under the tuned plans
    A64 = to_np(A)
    Qo, Lo, Vo = oracle.ruqlp(A64, k, p, q, seed, omega_dtype="f32" if dtype == torch.float32 else "f64")
    delta = recon_diff(*(to_np(x) for x in tuned), Qo, Lo, Vo) / np.linalg.norm(A64)
    assert delta <= (1e-5 if dtype == torch.float32 else 1e-12)
    # the saved table reproduces the tuned results bit for bit in a fresh context
    path = tmp_path / "plans.txt"
    ctx.autotune_save(path)
    text = path.read_text().split("\n")
    assert text[0] == "rqlp-plans 1" and sum(1 for t in text if t.startswith("gemm ")) == 2
    ctx2 = gpu_lib.Context(0)
    ctx2.autotune_load(path)
    assert ctx2.autotune_count() == 2
    again = gpu_lib.decompose(A, k, p, q, seed=seed, ctx=ctx2)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(tuned, again))
    # clearing returns the default plans
    ctx2.autotune_clear()
    assert ctx2.autotune_count() == 0
    dflt = gpu_lib.decompose(A, k, p, q, seed=seed, ctx=ctx2)
    ref = gpu_lib.decompose(A, k, p, q, seed=seed, ctx=gpu_lib.Context(0))
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(dflt, ref))


def test_malformed_plan_file_is_rejected(gpu_lib, tmp_path):
    announce("autotune malformed file")
    ctx = gpu_lib.Context(0)
    bad = tmp_path / "bad.txt"
    bad.write_text("rqlp-plans 1\ngemm 4 0 100 20\n")
    with pytest.raises(gpu_lib.RqlpError):
        ctx.autotune_load(bad)
    assert ctx.autotune_count() == 0
    bad.write_text("something else\n")
    with pytest.raises(gpu_lib.RqlpError):
        ctx.autotune_load(bad)
