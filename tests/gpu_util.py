"""Shared helpers of the GPU tests (no solver arithmetic)."""

import sys

import numpy as np
import torch


def say(*args):
    """Name the case before a GPU step, flushed, so a fault can be attributed."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x), dtype=dtype, device="cuda")


def host(t):
    return t.detach().to(torch.float64).cpu().numpy()


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
