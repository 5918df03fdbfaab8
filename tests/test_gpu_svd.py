"""The SVD-like form (Remark 1) on the GPU against the oracle
(oracle/svdlike.py): the small SVD (rqlp_svd_small) and the whole form
(rqlp_decompose_svd)."""
import numpy as np
import pytest
import torch

import oracle
from oracle.svdlike import svd_small as svd_small_oracle, ruqlp_svd
import workloads
from tests.gpu_util import announce, to_dev, to_np

pytestmark = pytest.mark.gpu


def _vectors_close(Ug, Uo, s, tol):
    """Columns whose singular value is separated from its neighbours by a
    relative gap of at least 1e-3 are unique (with the sign convention) and
    must agree to tol / gap."""
    d = s.size
    for j in range(d):
        gap = np.inf
        if j > 0:
            gap = min(gap, s[j - 1] - s[j])
        if j < d - 1:
            gap = min(gap, s[j] - s[j + 1])
        rel = gap / s[0]
        if rel < 1e-3 or s[j] == 0:
            continue
        assert np.abs(Ug[:, j] - Uo[:, j]).max() <= tol / rel, (j, rel)


def _lower(d, seed):
    rng = np.random.default_rng(seed)
    return np.tril(rng.standard_normal((d, d))) + 4.0 * np.eye(d)


@pytest.mark.parametrize("d", [1, 7, 32, 50, 130, 257, 544])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_svd_small_matches_oracle(gpu_lib, d, dtype):
    announce("svd_small", d, dtype)
    M = _lower(d, d)
    Mt = to_dev(M, dtype)
    Ug, Sg, Vg = (to_np(x) for x in gpu_lib.svd_small(Mt))
    Mr = to_np(Mt)  # the input as the device holds it
    Uo, So, Vo = svd_small_oracle(Mr)
    tol = 1e-13 if dtype == torch.float64 else 1e-6
    assert np.abs(Sg - So).max() <= tol * So[0] * max(1.0, np.sqrt(d))
    assert np.abs(Ug @ np.diag(Sg) @ Vg.T - Mr).max() <= tol * So[0] * d
    assert np.abs(Vg.T @ Vg - np.eye(d)).max() <= tol * d
    assert np.abs(Ug.T @ Ug - np.eye(d)).max() <= tol * d
    _vectors_close(Ug, Uo, So, tol * 10)
    _vectors_close(Vg, Vo, So, tol * 10)


def test_svd_small_special_cases(gpu_lib):
    """A diagonal matrix needs no rotation: the result is the oracle's signed
    permutation exactly; a zero column gives a zero singular value and a zero
    left vector."""
    announce("svd_small special cases")
    dv = np.array([0.5, -4.0, 2.0, -1.0, 3.0, 0.0, 7.0])
    Ug, Sg, Vg = (to_np(x) for x in gpu_lib.svd_small(to_dev(np.diag(dv))))
    Uo, So, Vo = svd_small_oracle(np.diag(dv))
    assert np.array_equal(Sg, So) and np.array_equal(Ug, Uo) and np.array_equal(Vg, Vo)
    # 40 x 40 with one zero column: sigma_40 = 0 and its left vector is zero
    M = _lower(40, 3)
    M[:, 17] = 0.0
    Ug, Sg, Vg = (to_np(x) for x in gpu_lib.svd_small(to_dev(M)))
    assert Sg[-1] == 0.0 and np.all(Ug[:, -1] == 0.0)
    assert np.abs(Ug @ np.diag(Sg) @ Vg.T - M).max() <= 1e-13 * Sg[0] * 40


@pytest.mark.parametrize("m,n,k,p,q,dtype", [
    (600, 400, 20, 10, 1, torch.float64),
    (700, 500, 40, 8, 0, torch.float32),
    (1200, 900, 250, 10, 1, torch.float64),   # d = 260: blocked Cholesky, 9 column blocks
])
def test_decompose_svd_matches_oracle(gpu_lib, m, n, k, p, q, dtype):
    announce("decompose_svd", m, n, k, p, q, dtype)
    sigma = workloads.spectrum("geometric", min(m, n), rho=0.97)
    A, _, _, _ = workloads.dense_from_spectrum(m, n, sigma, 11, trunc=0.0)
    At = to_dev(A, dtype)
    A64 = to_np(At)
    Ug, Sg, Wg = (to_np(x) for x in gpu_lib.decompose_svd(At, k, p, q, seed=8))
    Uo, So, Wo = ruqlp_svd(A64, k, p, q, 8, omega_dtype="f64" if dtype == torch.float64 else "f32")
    bar = 1e-12 if dtype == torch.float64 else 1e-5
    nA = np.linalg.norm(A64)
    delta = np.linalg.norm(Ug @ np.diag(Sg) @ Wg.T - Uo @ np.diag(So) @ Wo.T) / nA
    assert delta <= bar
    assert np.abs(Sg - So).max() <= bar * So[0]
    d = k + p
    assert np.abs(Ug.T @ Ug - np.eye(d)).max() <= bar * 10
    assert np.abs(Wg.T @ Wg - np.eye(d)).max() <= bar * 10
    _vectors_close(Ug, Uo, So, bar * 10)
    _vectors_close(Wg, Wo, So, bar * 10)


def test_decompose_svd_is_the_qlv_form_at_full_size(gpu_lib):
    """The 8000^2 float32 workload (k = 200, p = 10, q = 1): the SVD-like form
    equals the decomposition it is built from, (Q^T U) diag(S) (W^T V) = L,
    with orthonormal U and W; and its singular values interlace L's."""
    announce("decompose_svd full size 8000^2")
    m = n = 8000
    k, p, q = 200, 10, 1
    sigma = workloads.spectrum("gapped", n, gap_at=200)
    A = to_dev(workloads.dense_fast_orth(m, n, sigma, 2024, np.float32))
    Q, L, V = gpu_lib.decompose(A, k, p, q, seed=2024)
    U, S, W = gpu_lib.decompose_svd(A, k, p, q, seed=2024)
    torch.cuda.synchronize()
    d = k + p
    Q64, V64, U64, W64 = (x.double() for x in (Q, V, U, W))
    back = (Q64.T @ U64) @ torch.diag(S.double()) @ (W64.T @ V64)
    L64 = L.double()
    assert (torch.linalg.norm(back - L64) / torch.linalg.norm(L64)).item() <= 1e-5
    eye = torch.eye(d, dtype=torch.float64, device=A.device)
    assert (U64.T @ U64 - eye).abs().max().item() <= 1e-5
    assert (W64.T @ W64 - eye).abs().max().item() <= 1e-5
    s_ref = torch.linalg.svdvals(L64.cpu())
    assert (S.double().cpu() - s_ref).abs().max().item() <= 1e-5 * s_ref[0].item()


def test_svd_small_leading_dimensions(gpu_lib):
    """Strided input and outputs (ld > d): the same values as the packed call."""
    announce("svd_small leading dimensions")
    d = 45
    M = _lower(d, 8)
    big = np.zeros((d, 64))
    big[:, :d] = M
    Mt = to_dev(big)[:, :d]  # row stride 64
    U = torch.full((d, 50), float("nan"), dtype=torch.float64, device="cuda")[:, :d]
    V = torch.full((d, 70), float("nan"), dtype=torch.float64, device="cuda")[:, :d]
    S = torch.empty(d, dtype=torch.float64, device="cuda")
    gpu_lib.svd_small(Mt, out=(U, S, V))
    Ur, Sr, Vr = gpu_lib.svd_small(to_dev(M))
    torch.cuda.synchronize()
    assert torch.equal(U, Ur) and torch.equal(S, Sr) and torch.equal(V, Vr)


def test_decompose_svd_bf16_is_its_qlv_form(gpu_lib):
    """The bfloat16 form: U diag(S) W^T reproduces the bfloat16 decomposition
    Q L V^T it is built from (the same launch sequence up to L), to float32
    rounding of the SVD and the two products."""
    announce("decompose_svd bf16")
    m, n, k, p, q = 3000, 2000, 120, 8, 1
    sigma = workloads.spectrum("polynomial", n)
    A = to_dev(workloads.dense_fast_orth(m, n, sigma, 5, np.float32))
    Q, L, V = (to_np(x) for x in gpu_lib.decompose(A, k, p, q, seed=4, bf16=True))
    U, S, W = (to_np(x) for x in gpu_lib.decompose_svd(A, k, p, q, seed=4, bf16=True))
    ref = Q @ L @ V.T
    assert np.linalg.norm(U @ np.diag(S) @ W.T - ref) / np.linalg.norm(ref) <= 1e-5
    assert np.all(np.diff(S) <= 0)
    assert np.abs(U.T @ U - np.eye(k + p)).max() <= 1e-5
