"""Parity of the whole method (rqlp_decompose / rqlp_decompose_csr) with the
oracle.  Delta = ||Q L V^T - Qo Lo Vo^T||_F / ||A||_F must be <= 1e-12 on the
float64 path and <= 1e-5 on the float32 path.

Where the sketch has full column rank the factors are unique (unpivoted QR
with a positive diagonal), so Q, L and V are also compared with the oracle's
factor by factor, against the sensitivity of each factor to the working
precision's accumulation error (tests/fp32_model.py): Q and V column by
column, L entry by entry.  That covers the L-values diag(L), the
rank-revealing output of Algorithm 1 (Section III-A, Corollary 1), which the
norm Delta cannot see (a sign flip shared by a column of Q and a row of L
leaves Q L V^T unchanged)."""
import numpy as np
import pytest
import torch

import oracle
from oracle.metrics import recon_diff, recon_error, orth_error
import workloads
from tests import pins
from tests.fp32_model import factor_deviation, ruqlp_model
from tests.gpu_util import announce, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def _run(gpu_lib, A_np, k, p, q, seed, dtype):
    A = to_dev(A_np)
    Q, L, V = gpu_lib.decompose(A, k, p, q, seed=seed)
    return to_np(Q), to_np(L), to_np(V)


def _omega_dtype(dtype):
    return "f32" if dtype == torch.float32 else "f64"


def _orth_tol(dtype, d):
    """||Q^T Q - I||_F bound.  Float32: the second CholeskyQR pass runs in
    float64 and Q is rounded once to float32, which perturbs Q^T Q - I by
    about d u32 / sqrt(rows) <= sqrt(d) u32; allow 16 sqrt(d) u32.  Float64:
    CholeskyQR2's own orthogonality error, 100 d u64-ish."""
    if dtype == torch.float32:
        return 16.0 * np.sqrt(d) * 2.0 ** -24
    return 100 * d * 1e-15


def _check_against_oracle(A_np, Qg, Lg, Vg, k, p, q, seed, dtype, factors=True):
    A64 = A_np.astype(np.float64)
    Qo, Lo, Vo = oracle.ruqlp(A64, k, p, q, seed, omega_dtype=_omega_dtype(dtype))
    nA = np.linalg.norm(A64)
    delta = recon_diff(Qg, Lg, Vg, Qo, Lo, Vo) / nA
    tol = TOL[dtype]
    d = k + p
    assert delta <= tol, f"Delta {delta:.3e} > {tol}"
    eq, ev = orth_error(Qg), orth_error(Vg)
    assert eq <= _orth_tol(dtype, d) and ev <= _orth_tol(dtype, d), (eq, ev)
    assert np.all(np.triu(Lg, 1) == 0.0)
    assert np.all(np.diag(Lg) >= 0.0)
    if factors:
        model = ruqlp_model(A64, k, p, q, seed, dtype=_omega_dtype(dtype))
        rep = factor_deviation((Qg, Lg, Vg), (Qo, Lo, Vo), model, dtype=_omega_dtype(dtype))
        print(f"factors {A_np.shape} k={k} p={p} q={q} {dtype}: Delta={delta:.3e} orth Q {eq:.2e} V {ev:.2e} "
              f"ratios Q {rep['Q']['max_ratio']:.3f} V {rep['V']['max_ratio']:.3f} L {rep['L']['max_ratio']:.3f} "
              f"informative cols Q {rep['Q']['informative_cols']}/{d} V {rep['V']['informative_cols']}/{d} "
              f"max|dL| {rep['L']['max_err']:.2e} max|d diag L| {rep['L']['diag_max_err']:.2e}", flush=True)
        assert rep["ok"], rep
    return delta, (Qo, Lo, Vo)


def test_small_fp64_config(gpu_lib):
    """1000 x 800 FP64, sigma_i = 0.9^i, k = 20, p = 5, q = 0."""
    announce("decompose cfg small fp64")
    c = workloads.cfg_small_fp64(seed=1)
    Qg, Lg, Vg = _run(gpu_lib, c["A"], 20, 5, 0, 42, torch.float64)
    delta, (Qo, Lo, Vo) = _check_against_oracle(c["A"], Qg, Lg, Vg, 20, 5, 0, 42, torch.float64)
    # factors are unique here (full-rank sketch): compare them directly
    assert np.linalg.norm(Qg - Qo) < 1e-11 and np.linalg.norm(Vg - Vo) < 1e-11
    assert np.linalg.norm(Lg - Lo) < 1e-11 * np.linalg.norm(Lo)
    ok, info = pins.check_sv_interlacing(c["sigma"], Lg)
    assert ok, info


@pytest.mark.parametrize("m,n,k,p,q", [(600, 450, 30, 10, 0), (600, 450, 30, 10, 2), (450, 600, 20, 5, 1),
                                       (300, 300, 250, 6, 1), (97, 61, 60, 1, 1), (200, 40, 1, 0, 0),
                                       # d > 256 (wide Cholesky, column passes), up to the largest d = 544
                                       (1500, 1200, 300, 20, 1), (1100, 900, 520, 24, 0), (700, 900, 260, 1, 1)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_shapes_and_edges(gpu_lib, m, n, k, p, q, dtype):
    announce("decompose shapes", m, n, k, p, q, dtype)
    # CholeskyQR2 needs cond(A Omega) well below 1 / sqrt(u64) ~ 7e7; with
    # rho = 0.97 the sketch of width 544 would reach ~1e8, so wide sketches
    # take a slower decay
    rho = 0.97 if k + p <= 256 else 0.99
    sigma = workloads.spectrum("geometric", min(m, n), rho=rho)
    A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed=m + n, trunc=0.0)
    A = A.astype(np.float32) if dtype == torch.float32 else A
    Qg, Lg, Vg = _run(gpu_lib, A, k, p, q, 3, dtype)
    _check_against_oracle(A, Qg, Lg, Vg, k, p, q, 3, dtype)


@pytest.mark.parametrize("q", [0, 1])
def test_gapped_fp32_midsize(gpu_lib, q):
    announce("decompose gapped fp32 midsize", q)
    c = workloads.cfg_gapped_fp32(seed=5, m=3000, n=2500, q=q)
    Qg, Lg, Vg = _run(gpu_lib, c["A"], 200, 10, q, 8, torch.float32)
    _check_against_oracle(c["A"], Qg, Lg, Vg, 200, 10, q, 8, torch.float32)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_exact_recovery_rank_deficient(gpu_lib, dtype):
    """rank(A) = 12 <= k = 20: A is recovered exactly; the extra columns are
    completed with random directions and their L-values are exactly zero."""
    announce("decompose rank-deficient", dtype)
    sigma = np.zeros(300)
    sigma[:12] = np.linspace(3.0, 1.0, 12)
    A, _, _, _ = workloads.dense_from_spectrum(500, 300, sigma, seed=4, trunc=0.0)
    A = A.astype(np.float32) if dtype == torch.float32 else A
    ctx = gpu_lib.default_context(0)
    Qg, Lg, Vg = _run(gpu_lib, A, 20, 5, 1, 9, dtype)
    info = ctx.info()
    tol = TOL[dtype]
    assert recon_error(A, Qg, Lg, Vg) <= tol
    assert orth_error(Qg) <= 100 * 25 * (tol if dtype == torch.float32 else 1e-15)
    assert orth_error(Vg) <= 100 * 25 * (tol if dtype == torch.float32 else 1e-15)
    assert info["completed_cols"] > 0 and info["nonfinite"] == 0
    assert np.all(np.abs(np.diag(Lg)[12:]) <= tol * np.abs(np.diag(Lg)).max())
    # the reconstruction (unique) matches the oracle's
    Qo, Lo, Vo = oracle.ruqlp(A.astype(np.float64), 20, 5, 1, 9, omega_dtype=_omega_dtype(dtype))
    assert recon_diff(Qg, Lg, Vg, Qo, Lo, Vo) / np.linalg.norm(A) <= tol


def test_zero_matrix(gpu_lib):
    announce("decompose zero matrix")
    A = np.zeros((120, 90))
    Qg, Lg, Vg = _run(gpu_lib, A, 10, 4, 1, 2, torch.float64)
    assert np.all(Lg == 0.0)
    assert orth_error(Qg) < 1e-13 and orth_error(Vg) < 1e-13


def test_nonfinite_input_is_reported(gpu_lib):
    announce("decompose NaN input")
    A = np.random.default_rng(0).standard_normal((100, 80))
    A[3, 7] = np.nan
    ctx = gpu_lib.default_context(0)
    _run(gpu_lib, A, 5, 2, 0, 1, torch.float64)
    assert ctx.info()["nonfinite"] == 1
    # a clean call afterwards resets the record
    _run(gpu_lib, np.nan_to_num(A), 5, 2, 0, 1, torch.float64)
    assert ctx.info()["nonfinite"] == 0


def test_bitwise_deterministic(gpu_lib):
    announce("decompose determinism")
    c = workloads.cfg_gapped_fp32(seed=6, m=2000, n=1800, q=1)
    A = to_dev(c["A"])
    r1 = [t.clone() for t in gpu_lib.decompose(A, 100, 10, 1, seed=3)]
    r2 = [t.clone() for t in gpu_lib.decompose(A, 100, 10, 1, seed=3)]
    torch.cuda.synchronize()
    for a, b in zip(r1, r2):
        assert torch.equal(a, b)


@pytest.mark.parametrize("q", [1, 0])
def test_full_size_gapped_fp32(gpu_lib, q):
    """8000 x 8000 FP32, gapped spectrum, k = 200, p = 10, q in {1, 0}: the
    benchmark workload, in the launch configuration the benchmark uses.
    Beyond Delta, the factors are compared with the oracle's (the sketch has
    full rank), diag(L) >= 0, and the L-values reveal the gap: the first 200
    are ~1 and the last 10 ~ sigma_201 = 1e-3."""
    announce("decompose full 8000^2 fp32", q)
    c = workloads.cfg_gapped_fp32(seed=2, q=q)
    Qg, Lg, Vg = _run(gpu_lib, c["A"], 200, 10, q, 2024, torch.float32)
    _, (Qo, Lo, Vo) = _check_against_oracle(c["A"], Qg, Lg, Vg, 200, 10, q, 2024, torch.float32)
    dg = np.diag(Lg)
    assert dg[:200].min() > 100.0 * dg[200:].max()
    # sigma_i(L) <= sigma_i(A), up to the float32 rounding of A and of the factors
    ok, info = pins.check_sv_interlacing(c["sigma"], Lg, rel=1e-5)
    assert ok, info


# ---------------------------------------------------------------- bfloat16 products
# Stated tolerances of the bfloat16 form (RQLP_BF16_REFINED), all against
# the oracle with the same bfloat16 rounding of the product operands
# (operand_dtype="bf16": A, Omega, Q and W rounded to bfloat16, products
# then exact):
#  - Delta <= 5e-4.  The device accumulates in float32 and rounds its
#    float32 Q to bfloat16, so an operand within float32 noise of a rounding
#    boundary (spacing 2^-8) can round to the neighbour.  The float32
#    accumulation model of tests/fp32_model.py applied to the bfloat16
#    operands moves the reconstruction by 1.8e-4 to 3.2e-4 at these shapes.
#  - the error e = ||A - Q L V^T||_F / ||A||_F within 0.5 % of the emulated
#    oracle's own e.  The same model moves e by at most 0.08 % (relative).
#  - against the plain float64 oracle (context, the price of bfloat16
#    operands): Delta <= 2e-2.
TOL_BF16_EMUL = 5e-4
TOL_BF16_E_REL = 5e-3
TOL_BF16_F64 = 2e-2


@pytest.mark.parametrize("m,n,k,p,q", [(2000, 1500, 100, 20, 1), (1200, 1500, 60, 10, 0), (1000, 3000, 150, 20, 1),
                                       (4000, 3000, 280, 20, 1),
                                       # the 20000 x 15000 workload's shape class: d = 520, q = 1
                                       (6000, 4500, 500, 20, 1)])
def test_bf16_products(gpu_lib, m, n, k, p, q):
    announce("decompose bf16", m, n, k, p, q)
    sigma = workloads.spectrum("polynomial", min(m, n), power=1.5)
    big = k + p > 512
    if big:  # the structured orthogonal factors of the full-size workload (exact spectrum, seconds)
        A = workloads.dense_fast_orth(m, n, sigma, seed=m + 2 * n, dtype=np.float32)
    else:
        A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed=m + 2 * n, dtype=np.float32, trunc=0.0)
    seed = 11
    Q, L, V = gpu_lib.decompose(to_dev(A), k, p, q, seed=seed, bf16=True)
    Qg, Lg, Vg = to_np(Q), to_np(L), to_np(V)
    A64 = A.astype(np.float64)
    nA = np.linalg.norm(A64)
    Qe, Le, Ve = oracle.ruqlp(A64, k, p, q, seed, omega_dtype="bf16", operand_dtype="bf16")
    d_emul = recon_diff(Qg, Lg, Vg, Qe, Le, Ve) / nA
    e_gpu = recon_error(A64, Qg, Lg, Vg)
    e_emul = recon_error(A64, Qe, Le, Ve)
    print(f"bf16 {m}x{n} k={k} p={p} q={q}: Delta(emulated)={d_emul:.3e} "
          f"e={e_gpu:.5e} e_emul={e_emul:.5e} (rel {(e_gpu - e_emul) / e_emul:+.2e})", flush=True)
    assert d_emul <= TOL_BF16_EMUL
    assert abs(e_gpu - e_emul) <= TOL_BF16_E_REL * e_emul
    if not big:  # context: the distance to the float64 method (the largest case skips this second oracle run)
        Qd, Ld, Vd = oracle.ruqlp(A64, k, p, q, seed, omega_dtype="f64")
        d_f64 = recon_diff(Qg, Lg, Vg, Qd, Ld, Vd) / nA
        print(f"  Delta(f64)={d_f64:.3e} e_f64={recon_error(A64, Qd, Ld, Vd):.5e}", flush=True)
        assert d_f64 <= TOL_BF16_F64
    d = k + p
    assert orth_error(Qg) <= _orth_tol(torch.float32, d) and orth_error(Vg) <= _orth_tol(torch.float32, d)
    assert np.all(np.triu(Lg, 1) == 0.0) and np.all(np.diag(Lg) >= 0.0)


def test_bf16_full_size_properties(gpu_lib):
    """The 20000 x 15000 bfloat16 workload itself (sigma_i = i^-1.5, k = 500,
    p = 20, q = 1), where the oracle would take minutes: properties that
    hold at any size.  Orthonormal Q and V, L lower triangular with
    diag(L) >= 0; sigma_i(L) <= sigma_i(A) up to the bfloat16 rounding of A
    (Corollary 1: L = R^T of qr(round(A)^T round(Q)), and
    ||round(A) - A||_2 <= ||round(A) - A||_F <= 2^-9 ||A||_F); the error
    e = ||A - Q L V^T||_F / ||A||_F between the rank-d optimum (Eckart-Young,
    from the known spectrum) and 1.6 times it; the leading singular values
    of L within 1 % (plus the bfloat16 floor) of sigma_i."""
    announce("decompose bf16 full size 20000x15000")
    c = workloads.cfg_poly_bf16(seed=4)
    k, p, q = c["k"], c["p"], c["q"]
    d = k + p
    Q, L, V = gpu_lib.decompose(to_dev(c["A"]), k, p, q, seed=2024, bf16=True)
    Qg, Lg, Vg = to_np(Q), to_np(L), to_np(V)
    A64 = c["A"].astype(np.float64)
    nA = np.linalg.norm(A64)
    sigma = np.sort(c["sigma"])[::-1]
    eq, ev = orth_error(Qg), orth_error(Vg)
    assert eq <= _orth_tol(torch.float32, d) and ev <= _orth_tol(torch.float32, d), (eq, ev)
    assert np.all(np.triu(Lg, 1) == 0.0) and np.all(np.diag(Lg) >= 0.0)
    sl = np.linalg.svd(Lg, compute_uv=False)
    floor = 2.0 ** -9 * nA
    assert np.all(sl <= 1.01 * sigma[:d] + floor), float(np.max(sl - 1.01 * sigma[:d] - floor))
    assert np.all(np.abs(sl[:20] - sigma[:20]) <= 0.01 * sigma[:20] + floor)
    e = recon_error(A64, Qg, Lg, Vg)
    e_opt = np.sqrt(np.sum(sigma[d:] ** 2)) / nA
    print(f"bf16 full size: e={e:.4e} optimum {e_opt:.4e} (ratio {e / e_opt:.3f}) orth Q {eq:.2e} V {ev:.2e}",
          flush=True)
    assert e_opt * (1 - 1e-3) <= e <= 1.6 * e_opt


# ---------------------------------------------------------------- CSR
@pytest.mark.parametrize("m,n,density,k,p,q", [(3000, 2000, 0.01, 30, 10, 1), (2000, 3000, 0.005, 20, 5, 0)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_csr_matches_oracle(gpu_lib, m, n, density, k, p, q, dtype):
    announce("decompose csr", m, n, density, k, p, q, dtype)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    rowptr, colidx, vals = workloads.csr_uniform(m, n, int(density * m * n), seed=m, dtype=npdt)
    Q, L, V = gpu_lib.decompose_csr(to_dev(rowptr), to_dev(colidx), to_dev(vals), m, n, k, p, q, seed=4)
    Qg, Lg, Vg = to_np(Q), to_np(L), to_np(V)
    Qo, Lo, Vo = oracle.ruqlp_csr(rowptr, colidx, vals, m, n, k, p, q, 4, omega_dtype=_omega_dtype(dtype))
    nA = np.linalg.norm(vals.astype(np.float64))
    assert recon_diff(Qg, Lg, Vg, Qo, Lo, Vo) / nA <= TOL[dtype]
    assert np.all(np.triu(Lg, 1) == 0.0)


def test_csr_full_size(gpu_lib):
    """CSR 100000 x 50000, 0.1 % density, N(0,1) FP32, k = 100, p = 10, q = 1."""
    announce("decompose csr full size")
    c = workloads.cfg_sparse(seed=3)
    m, n = c["m"], c["n"]
    Q, L, V = gpu_lib.decompose_csr(to_dev(c["rowptr"]), to_dev(c["colidx"]), to_dev(c["vals"]), m, n,
                                    100, 10, 1, seed=7)
    Qg, Lg, Vg = to_np(Q), to_np(L), to_np(V)
    Qo, Lo, Vo = oracle.ruqlp_csr(c["rowptr"], c["colidx"], c["vals"], m, n, 100, 10, 1, 7, omega_dtype="f32")
    nA = np.linalg.norm(c["vals"].astype(np.float64))
    assert recon_diff(Qg, Lg, Vg, Qo, Lo, Vo) / nA <= 1e-5


# ---------------------------------------------------------------- the paper's own orientation
@pytest.mark.parametrize("m,n,k,p,q", [(600, 450, 30, 10, 1), (450, 600, 20, 5, 0), (1000, 800, 20, 5, 0),
                                       (700, 500, 120, 8, 2)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_paper_orientation_matches_oracle(gpu_lib, m, n, k, p, q, dtype):
    """rqlp_decompose_paper against oracle.ruqlp_paper (Algorithm 1 as
    printed): the same Delta gates; the factors are unique here."""
    announce("decompose paper orientation", m, n, k, p, q, dtype)
    sigma = workloads.spectrum("geometric", min(m, n), rho=0.97)
    A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, seed=m + 3 * n, trunc=0.0)
    A = A.astype(np.float32) if dtype == torch.float32 else A
    Qg, Lg, Pg = (to_np(x) for x in gpu_lib.decompose_paper(to_dev(A), k, p, q, seed=6))
    A64 = A.astype(np.float64)
    Qo, Lo, Po = oracle.ruqlp_paper(A64, k, p, q, 6, omega_dtype=_omega_dtype(dtype))
    tol = TOL[dtype]
    assert recon_diff(Qg, Lg, Pg, Qo, Lo, Po) / np.linalg.norm(A64) <= tol
    d = k + p
    assert orth_error(Qg) <= _orth_tol(dtype, d) and orth_error(Pg) <= _orth_tol(dtype, d)
    assert np.all(np.triu(Lg, 1) == 0.0) and np.all(np.diag(Lg) >= 0.0)
    if dtype == torch.float64:
        assert np.linalg.norm(Lg - Lo) <= 1e-10 * np.linalg.norm(Lo)


def test_paper_orientation_full_size(gpu_lib):
    """rqlp_decompose_paper on the 8000 x 8000 benchmark input (q = 1)
    against oracle.ruqlp_paper: Delta, orthonormal Q and P, L lower
    triangular with diag(L) >= 0, the L-values' gap (the first 200 ~ 1, the
    last 10 ~ sigma_201 = 1e-3), sigma_i(L) <= sigma_i(A), and diag(L)
    against the oracle's (its sketch has full rank, so L is unique)."""
    announce("decompose paper orientation full 8000^2 fp32")
    c = workloads.cfg_gapped_fp32(seed=2, q=1)
    Qg, Lg, Pg = (to_np(x) for x in gpu_lib.decompose_paper(to_dev(c["A"]), 200, 10, 1, seed=2024))
    A64 = c["A"].astype(np.float64)
    Qo, Lo, Po = oracle.ruqlp_paper(A64, 200, 10, 1, 2024, omega_dtype="f32")
    assert recon_diff(Qg, Lg, Pg, Qo, Lo, Po) / np.linalg.norm(A64) <= 1e-5
    assert orth_error(Qg) <= _orth_tol(torch.float32, 210) and orth_error(Pg) <= _orth_tol(torch.float32, 210)
    assert np.all(np.triu(Lg, 1) == 0.0) and np.all(np.diag(Lg) >= 0.0)
    dg, do = np.diag(Lg), np.diag(Lo)
    assert dg[:200].min() > 100.0 * dg[200:].max()
    ok, info = pins.check_sv_interlacing(c["sigma"], Lg, rel=1e-5)
    assert ok, info
    # the leading L-values are ~1 and well separated: float32 noise moves
    # them by ~1e-6 relative; the trailing ones (~1e-3) by ~1e-6 absolute
    assert np.all(np.abs(dg - do) <= 1e-4 * np.abs(do) + 1e-5), float(np.max(np.abs(dg - do)))
