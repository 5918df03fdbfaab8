"""Round float64 values to bfloat16 (round to nearest, ties to even).

Test infrastructure (see the package docstring).  bfloat16 keeps the sign,
the 8 exponent bits and the top 7 fraction bits of an IEEE binary32 value.
Values are first rounded to binary32 (numpy), then the low 16 bits of the
binary32 pattern are rounded off with ties to even.  NaN stays NaN.

Pinned by: tests/test_oracle_bf16.py (exactly representable values are
fixed points, ties go to the even neighbour, the spacing of results matches
2^(e-7), overflow to infinity).
"""

import numpy as np


def round_bf16(x):
    """Return x rounded to bfloat16, as float64."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = (bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)
