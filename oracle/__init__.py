"""Plain FP64 CPU oracle for randomized unpivoted QLP (RU-QLP).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this package:
only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may use it.  It shares no code with the HIP library under
``paper_2209_12464_amd/csrc``; the two meet only through the seeded input
generators in ``workloads/`` (which hold none of the method's arithmetic).

What it computes follows the paper:

* Section III-A, Algorithm 1 (RU-QLP) and Section III-B, Algorithm 2
  (power iteration with orthonormalization), applied in the column-sketch
  orientation: Y = A*Omega, Q = orth(Y), q power steps, B^T = A^T Q,
  [V, Rt] = qr(B^T), L = Rt^T, so that A ~ Q L V^T.  This is the paper's
  algorithm run on A^T (Section III-A with A replaced by A^T), stopping
  before the extra d x d qr of R^T.
* ruqlp_paper follows Algorithm 1 as printed instead (row sketch Phi,
  P-bar = orth(A^T Phi), qr(A P-bar), then the d x d qr of R^T, P = P-bar
  P-tilde, L = R-tilde^T).
* orth() and qr() are the thin unpivoted Householder QR with a positive
  diagonal in R (Section II-B defines the unpivoted QR; the sign convention
  is this oracle's reading, which makes the factors unique for full column
  rank input).
* The Gaussian test matrix (the sketch of Section III-A, randn defined in
  Section II-A) comes from Philox4x64-10 (Salmon et al., SC'11) and the
  Box-Muller transform, so that host and device draw the same numbers.

Module map:
  philox.py       counter-based generator and normal transform
  householder.py  Householder QR with positive diagonal
  ruqlp.py        the method (dense and CSR input)
  svdlike.py      Remark 1: the SVD-like form from an SVD of the d x d factor
  csr.py          CSR products and the CSR transpose, by definition
  metrics.py      reconstruction differences and errors, blockwise
  bf16.py         round-to-nearest-even to bfloat16, by bit definition

Parity status of each function is stated in its docstring ("pinned by ..."
or "parity unpinned").
"""

from .philox import philox4x64_10, gaussian_matrix, uniform_pair, box_muller  # noqa: F401
from .householder import householder_qr  # noqa: F401
from .ruqlp import ruqlp, ruqlp_csr, ruqlp_paper, orth  # noqa: F401
from .svdlike import svd_small, svd_like, ruqlp_svd  # noqa: F401
from .csr import csr_matmul, csr_transpose  # noqa: F401
from .metrics import recon_diff, recon_error, orth_error, recon_error_csr  # noqa: F401
