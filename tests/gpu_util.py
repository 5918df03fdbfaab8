"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np
import torch


def announce(*parts):
    """Print and flush what names the GPU case about to run."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)
