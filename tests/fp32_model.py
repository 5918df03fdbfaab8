"""Factor-level gates for the float32 and float64 paths (test helper).

The device runs every product with A in float32 with float32 accumulation,
stores Q and W in float32, and keeps the Gram matrices and Cholesky factors
in float64.  To first order its result is the exact method applied to
products carrying float32 accumulation errors.  This helper runs the
oracle's own steps (oracle.ruqlp._ruqlp_core: Householder orth and qr, no
arithmetic of its own) with products perturbed by that error model:

  Y = fl32( A fl32(X) + E ),  E_ij ~ N(0, 1) * 2^-24 * sqrt(K / 6) * s_ij,
  s_ij = sqrt( sum_k (A_ik fl32(X)_kj)^2 ),

which is the standard random-rounding model of a K-term float32 sum (each
addition's relative error uniform in [-u, u], partial sums a random walk:
variance u^2/3 * sum_t s_t^2 ~ u^2 K/6 * sum_k (a_k x_k)^2).  The device
splits the sum into chunks and adds the chunk sums, which only lowers its
error, so the model over-estimates the device's noise.

The float64 path takes the same model with u = 2^-53 and no storage
rounding (its products accumulate in float64).

The spread between the model's factors and the oracle's is the sensitivity
of each factor to float32 accumulation: a column of Q (or V) of a badly
conditioned sketch moves by about cond * u * sqrt(K), a well-conditioned one
by about u * sqrt(K).  The gates ask the device factors to lie within C
times that spread of the oracle's (plus a floor at the output rounding), per
column for Q and V and entry by entry (per column of L) for L.  A sign flip
shared by a column of Q and a row of L, a transposed block or a permuted
column moves a factor by O(1) and fails wherever the sensitivity is below
1/C.
"""

import numpy as np

from oracle.ruqlp import _ruqlp_core

U32 = 2.0 ** -24
U64 = 2.0 ** -53
UNIT = {"f32": U32, "f64": U64}


def _store(x, dtype):
    if dtype == "f32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


def noisy_product(M, X, rng, dtype="f32"):
    """store(M store(X) + E) with the accumulation model above."""
    Xs = _store(X, dtype)
    Y = M @ Xs
    K = M.shape[1]
    s = np.sqrt((M * M) @ (Xs * Xs))
    Y += rng.standard_normal(Y.shape) * (UNIT[dtype] * np.sqrt(K / 6.0)) * s
    return _store(Y, dtype)


def ruqlp_model(A, k, p, q, seed, dtype="f32", rng_seed=12345):
    """The oracle's RU-QLP (Omega rounded to `dtype`) with the products of
    the accumulation model of `dtype` ("f32" or "f64"); returns (Q, L, V)
    in float64."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    rng = np.random.default_rng(rng_seed)
    At = A.T
    return _ruqlp_core(lambda X: noisy_product(A, X, rng, dtype), lambda X: noisy_product(At, X, rng, dtype), n, k,
                       p, q, seed, dtype)


def factor_deviation(dev, ref, model, dtype="f32", C=4.0):
    """Compare device factors (Q, L, V) with the oracle's, against C times the
    model's spread.  Returns a report dict; report["ok"] is the verdict.

    Q, V: per column j, ||g_j - o_j|| <= C ||n_j - o_j|| + floor.
    L:    per entry (i >= j), |Lg_ij - Lo_ij| <= C max_i |Ln_ij - Lo_ij| + floor max|Lo|.
    floor = 16 u of the output type.  Columns whose bound reaches 1 carry no information (the factor is not
    determined at float32 precision there); they are counted, not skipped.
    """
    (Qg, Lg, Vg), (Qo, Lo, Vo), (Qn, Ln, Vn) = dev, ref, model
    floor = 16.0 * UNIT[dtype]
    rep = {"ok": True}
    for name, G, O, N in (("Q", Qg, Qo, Qn), ("V", Vg, Vo, Vn)):
        eg = np.linalg.norm(G - O, axis=0)
        en = np.linalg.norm(N - O, axis=0)
        bound = C * en + floor
        bad = np.nonzero(eg > bound)[0]
        rep[name] = {"max_ratio": float(np.max(eg / bound)), "bad_cols": bad.tolist()[:10],
                     "informative_cols": int(np.sum(bound < 1.0)), "max_err": float(eg.max())}
        rep["ok"] &= bad.size == 0
    lg = np.abs(np.tril(Lg - Lo))
    ln = np.abs(np.tril(Ln - Lo))
    bound_col = C * ln.max(axis=0) + floor * np.abs(Lo).max()
    ratio = lg / bound_col[None, :]
    bad = np.argwhere(ratio > 1.0)
    rep["L"] = {"max_ratio": float(ratio.max()), "bad_entries": bad.tolist()[:10],
                "max_err": float(lg.max()), "diag_max_err": float(np.abs(np.diag(Lg) - np.diag(Lo)).max())}
    rep["ok"] &= bad.size == 0
    return rep
