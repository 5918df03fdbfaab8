"""The product autotuner (rqlp_autotune: row tile and split-K count): tuned
plans keep parity with the oracle, are reproducible bit for bit through
save / load, the row tile leaves the bits unchanged, and clearing the table
returns the default plans."""
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
    assert text[0] == "rqlp-plans 2" and sum(1 for t in text if t.startswith("gemm ")) == 2
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


def test_row_tile_keeps_bits(gpu_lib, tmp_path):
    """The same split counts with the other row tile (128 <-> 256 rows per
    workgroup) give the same bits: each output's summation order depends on
    the split only.  Version 1 plan files (no row tile) still load."""
    announce("autotune row tile")
    m, n, k, p, q, seed = 2600, 1900, 90, 10, 1, 5
    A = _matrix(m, n, torch.float32)
    ctx = gpu_lib.Context(0)
    ctx.autotune(A, k + p)
    path = tmp_path / "plans.txt"
    ctx.autotune_save(path)
    tuned = [x.clone() for x in gpu_lib.decompose(A, k, p, q, seed=seed, ctx=ctx)]
    lines = path.read_text().strip().split("\n")
    for mb in ("2", "4"):
        flipped = [lines[0]] + [" ".join(t.split()[:-1] + [mb]) for t in lines[1:]]
        path.write_text("\n".join(flipped) + "\n")
        c2 = gpu_lib.Context(0)
        c2.autotune_load(path)
        out = gpu_lib.decompose(A, k, p, q, seed=seed, ctx=c2)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(tuned, out)), mb
    A64 = to_np(A)
    Qo, Lo, Vo = oracle.ruqlp(A64, k, p, q, seed, omega_dtype="f32")
    assert recon_diff(*(to_np(x) for x in tuned), Qo, Lo, Vo) / np.linalg.norm(A64) <= 1e-5
    v1 = ["rqlp-plans 1"] + [" ".join(t.split()[:-1]) for t in lines[1:]]
    path.write_text("\n".join(v1) + "\n")
    c3 = gpu_lib.Context(0)
    c3.autotune_load(path)
    assert c3.autotune_count() == 2
    out = gpu_lib.decompose(A, k, p, q, seed=seed, ctx=c3)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(tuned, out))


def test_float64_rejects_wide_row_tile(gpu_lib, tmp_path):
    announce("autotune float64 row tile")
    bad = tmp_path / "bad64.txt"
    bad.write_text("rqlp-plans 2\ngemm 8 0 1000 30 800 2 4\n")
    ctx = gpu_lib.Context(0)
    with pytest.raises(gpu_lib.RqlpError):
        ctx.autotune_load(bad)
    assert ctx.autotune_count() == 0
