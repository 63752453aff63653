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
    """Norm-wise ||a - b|| / ||b|| (used only where a norm is what is stated,
    e.g. ||x - x_oracle|| / ||x_oracle||)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxerr(got, ref, rows=None):
    """Element-wise error: max_i |got_i - ref_i| / max_i |ref_i|, over all
    entries or only over `rows` (then both maxima run over those rows, so a
    small-valued region is measured against its own scale)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if rows is not None:
        got, ref = got[rows], ref[rows]
    if ref.size == 0:
        return 0.0
    if not np.all(np.isfinite(got)):
        return float("inf")
    return float(np.max(np.abs(got - ref)) / max(float(np.max(np.abs(ref))), 1e-300))


def box_face_rows(nx, ny=1, nz=1):
    """Rows of an x-fastest nx x ny x nz grid that lie on a face of the box
    (where a stencil loses neighbours and kernels clamp or stage halos)."""
    i = np.arange(nx * ny * nz)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    on = (x == 0) | (x == nx - 1)
    if ny > 1:
        on |= (y == 0) | (y == ny - 1)
    if nz > 1:
        on |= (z == 0) | (z == nz - 1)
    return np.nonzero(on)[0]


def tail_rows(n, block=1024):
    """The last (partial, if n is not a multiple) block of `block` rows."""
    r = n % block
    return np.arange(n - (r if r else min(block, n)), n)


def assert_close(got, ref, tol, what="", box=None):
    """Element-wise bound max|got - ref| <= tol max|ref|, then the same bound
    on the last 1024-row block and, for a grid (box = (nx, ny, nz)), on the
    rows of the box faces, each measured against its own scale."""
    e = maxerr(got, ref)
    assert e <= tol, f"{what}: element-wise error {e:.3e} > {tol:.1e}"
    n = np.asarray(ref).shape[0]
    et = maxerr(got, ref, tail_rows(n))
    assert et <= tol, f"{what}: last-block error {et:.3e} > {tol:.1e}"
    if box is not None:
        ef = maxerr(got, ref, box_face_rows(*box))
        assert ef <= tol, f"{what}: box-face error {ef:.3e} > {tol:.1e}"
    return e
