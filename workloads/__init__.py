"""Seeded synthetic inputs shaped like the paper's test matrices.

Shared by the tests, the benchmark and the oracle checks.  This module
holds none of the decomposition's arithmetic: it only builds input
matrices (and their known singular values) from a seed.

Dense inputs are A = U diag(sigma) V^T with Haar-distributed orthonormal
columns U, V (QR of an i.i.d. Gaussian matrix with the columns multiplied
by the signs of diag(R), so the distribution is exactly Haar).  Spectra:

* geometric   sigma_i = rho^i                              (1000 x 800 FP64 case)
* gapped      sigma_i = 1 (i <= g), 1e-3 * 0.95^(i-g) after (8000^2 FP32 case)
* polynomial  sigma_i = i^-1.5                              (20000 x 15000 case)
* the four theorem-evaluation matrices of Section V-B (LowRankLargeGap,
  LowRankMediumGap, LowRankSlowDecay, LowRankFastDecay).

The 20000 x 15000 case is built with structured orthogonal factors instead
(dense_fast_orth): U = P_m C_m D_m (first n columns) and V = P_n C_n D_n,
with C the orthonormal DCT-II matrix, D a random sign diagonal and P a
random row permutation.  They are exactly orthogonal, so A has exactly the
prescribed singular values, and cost O(m n log m) instead of the O(m n^2)
of Haar factors.  For a Gaussian test matrix the method's output
distribution depends only on the singular values (V^T Omega is again
Gaussian), so this changes nothing but the rounding pattern of A.

Terms with sigma_i below `trunc` * sigma_1 are dropped before the product
(A keeps only the first r singular triplets).  At the default 1e-10 this
changes A by far less than its float32 rounding.

Sparse inputs: exactly nnz distinct positions drawn uniformly over all
m*n cells, N(0,1) values, CSR with sorted column indices (the sparse case
of Section V-A at 0.1 % density).
"""

import numpy as np


def _rng(seed):
    return np.random.default_rng(np.random.SeedSequence([int(seed), 0x57AD]))


def haar_columns(rng, m, r):
    """m x r matrix with orthonormal columns, Haar distributed (the first r
    columns of a Haar orthogonal matrix)."""
    G = rng.standard_normal((m, r))
    Qm, Rm = np.linalg.qr(G)
    s = np.sign(np.diag(Rm))
    s[s == 0] = 1.0
    return Qm * s[None, :]


def spectrum(kind, count, **kw):
    """Singular values sigma_1..sigma_count (1-based formulas)."""
    i = np.arange(1, count + 1, dtype=np.float64)
    if kind == "geometric":
        return kw.get("rho", 0.9) ** i
    if kind == "gapped":
        g = kw.get("gap_at", 200)
        return np.where(i <= g, 1.0, 1e-3 * 0.95 ** (i - g))
    if kind == "polynomial":
        return i ** (-kw.get("power", 1.5))
    if kind == "lowrank_decay":
        # Section V-B: k ones, then 2^-z, 3^-z, ..., (n-k+1)^-z
        k, z = kw["k"], kw["z"]
        return np.where(i <= k, 1.0, np.maximum(i - k + 1.0, 1.0) ** (-z))
    if kind == "lowrank_linear":
        # Section V-B: decreasing linearly from 1 to 1e-10 over all n
        # positions, zero after the first k (the paper's wording is ambiguous;
        # this reading is the one that reproduces its printed Theorem-bound
        # curves)
        k, n = kw["k"], kw["n"]
        s = np.linspace(1.0, 1e-10, count)
        return np.where(i <= k, s, 0.0)
    raise ValueError(kind)


def dense_from_spectrum(m, n, sigma, seed, dtype=np.float64, trunc=1e-10):
    """A = U diag(sigma) V^T, Haar U (m x r), V (n x r); returns (A, sigma_r,
    U, V) where r counts the kept singular values."""
    sigma = np.asarray(sigma, dtype=np.float64)
    keep = sigma >= trunc * sigma.max() if sigma.size and sigma.max() > 0 else np.zeros(0, bool)
    sigma_r = sigma[keep]
    r = sigma_r.size
    rng = _rng(seed)
    U = haar_columns(rng, m, r)
    V = haar_columns(rng, n, r)
    A = (U * sigma_r[None, :]) @ V.T
    return A.astype(dtype), sigma_r, U, V


def dense_fast_orth(m, n, sigma, seed, dtype=np.float32):
    """A = U diag(sigma) V^T (m >= n, len(sigma) = n) with the structured
    orthogonal factors described above; returns A in `dtype`."""
    import scipy.fft
    if m < n or len(sigma) != n:
        raise ValueError("need m >= n and n singular values")
    rng = _rng(seed)
    dm = rng.choice(np.array([-1.0, 1.0]), size=m)
    dn = rng.choice(np.array([-1.0, 1.0]), size=n)
    pm = rng.permutation(m)
    pn = rng.permutation(n)
    sig = np.asarray(sigma, dtype=np.float64)
    # V diag(sigma) = (C_n D_n diag(sigma))[pn]
    vs = scipy.fft.dct(np.diag(dn * sig), type=2, norm="ortho", axis=0, workers=-1)[pn]
    # A = U (V diag(sigma))^T = (C_m (D_m [ (V diag(sigma))^T ; 0 ]))[pm]
    Z = np.zeros((m, n), dtype=np.float64)
    Z[:n] = dm[:n, None] * vs.T
    del vs
    A = scipy.fft.dct(Z, type=2, norm="ortho", axis=0, workers=-1, overwrite_x=True)
    del Z
    return np.ascontiguousarray(A[pm].astype(dtype))


def lowrank_plus_noise(n, k, mu, seed):
    """Section V-B LowRankLargeGap / LowRankMediumGap:
    A = U Sigma V^T + mu * sigma_k * A_N with A_N a Gaussian matrix scaled to
    unit spectral norm (the reading of "normalized").  Returns A (float64)."""
    sigma = spectrum("lowrank_linear", n, k=k, n=n)
    rng = _rng(seed)
    U = haar_columns(rng, n, k)
    V = haar_columns(rng, n, k)
    A = (U * sigma[None, :k]) @ V.T
    AN = rng.standard_normal((n, n))
    AN /= np.linalg.norm(AN, 2)
    return A + mu * sigma[k - 1] * AN


def csr_uniform(m, n, nnz, seed, dtype=np.float32):
    """CSR matrix with exactly nnz distinct uniformly placed entries, N(0,1)
    values.  Returns (rowptr int32, colidx int32, vals dtype)."""
    if nnz > m * n:
        raise ValueError("nnz > m*n")
    rng = _rng(seed)
    cells = np.zeros(0, dtype=np.int64)
    while cells.size < nnz:
        extra = rng.integers(0, m * n, size=int((nnz - cells.size) * 1.05) + 16, dtype=np.int64)
        cells = np.unique(np.concatenate([cells, extra]))
    if cells.size > nnz:
        cells = np.sort(rng.choice(cells, size=nnz, replace=False))
    rows = cells // n
    cols = (cells % n).astype(np.int32)
    counts = np.bincount(rows, minlength=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    vals = rng.standard_normal(nnz).astype(dtype)
    return rowptr.astype(np.int32), cols, vals


# Named workloads ---------------------------------------------------------

def cfg_small_fp64(seed=1):
    """1000 x 800 FP64, sigma_i = 0.9^i, k=20, p=5, q=0."""
    A, s, U, V = dense_from_spectrum(1000, 800, spectrum("geometric", 800, rho=0.9), seed,
                                     np.float64, trunc=0.0)
    return dict(A=A, sigma=s, U=U, V=V, k=20, p=5, q=0, prec="f64")


def cfg_gapped_fp32(seed=2, m=8000, n=8000, q=1):
    """8000 x 8000 FP32, gapped spectrum, k=200, p=10."""
    A, s, U, V = dense_from_spectrum(m, n, spectrum("gapped", min(m, n), gap_at=200), seed,
                                     np.float32)
    return dict(A=A, sigma=s, U=U, V=V, k=200, p=10, q=q, prec="f32")


def cfg_poly_bf16(seed=4, m=20000, n=15000):
    """20000 x 15000 FP32 input, sigma_i = i^-1.5 (structured orthogonal
    factors), k=500, p=20, q=1, bfloat16 products."""
    sigma = spectrum("polynomial", min(m, n), power=1.5)
    A = dense_fast_orth(m, n, sigma, seed, np.float32)
    return dict(A=A, sigma=sigma, k=500, p=20, q=1, prec="bf16")


def serving_requests(count, seed, m_range=(512, 8192), n_range=(256, 4096), kmax=256, p=10):
    """Request shapes of the serving stream: m, n uniform in their ranges,
    k uniform in [8, min(kmax, min(m, n) - p)], p fixed, a geometric decay
    rate rho uniform in [0.8, 0.99] and a matrix seed per request."""
    rng = _rng(seed)
    out = []
    for _ in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        k = int(rng.integers(8, min(kmax, min(m, n) - p) + 1))
        rho = float(rng.uniform(0.8, 0.99))
        out.append(dict(m=m, n=n, k=k, p=p, rho=rho, seed=int(rng.integers(1, 2 ** 31))))
    return out


def request_matrix(req, dtype=np.float32):
    """A request's matrix: sigma_i = rho^i up to the rank where it falls
    below 1e-8, zero after, with structured orthogonal factors."""
    m, n, rho = req["m"], req["n"], req["rho"]
    r = min(m, n)
    i = np.arange(1, r + 1, dtype=np.float64)
    sig = rho ** i
    sig[i > np.ceil(np.log(1e-8) / np.log(rho))] = 0.0
    if m >= n:
        return dense_fast_orth(m, n, sig, req["seed"], dtype)
    return np.ascontiguousarray(dense_fast_orth(n, m, sig, req["seed"], dtype).T)


def cfg_sparse(seed=3, m=100000, n=50000, density=1e-3):
    """CSR 100000 x 50000, 0.1 % density, N(0,1) FP32, k=100, p=10, q=1."""
    nnz = int(round(density * m * n))
    rowptr, colidx, vals = csr_uniform(m, n, nnz, seed)
    return dict(rowptr=rowptr, colidx=colidx, vals=vals, m=m, n=n, k=100, p=10, q=1, prec="f32")
