"""Reduced-precision emulation of the chains: the oracle's version.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes in double precision only. This module runs the same
unit chains (Algorithms 1 and 3) with float32 arithmetic, optionally
rounding every stored vector to bfloat16 (round to nearest even), so that a
test can state how far a reduced-precision chain may drift from the float64
one on a given input: delta = ||p_low(A)v - p_64(A)v|| / ||p_64(A)v||.
"""

from __future__ import annotations

import numpy as np

REAL = 0


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _store(x, prec):
    x = x.astype(np.float32)
    return round_bf16(x) if prec == "bf16" else x


def apply_p_low(A32, units, v, prec: str = "fp32") -> np.ndarray:
    """p(A)v with float32 arithmetic (A32: float32 sparse matrix)."""
    prod = _store(np.asarray(v), prec)
    p = np.zeros_like(prod, dtype=np.float32)
    last = len(units) - 1
    for idx, (kind, a, b) in enumerate(units):
        if kind == REAL:
            c = np.float32(1.0 / a)
            p = p + c * prod
            if idx != last:
                prod = _store(prod - c * (A32 @ prod), prec)
        else:
            s = np.float32(1.0 / (a * a + b * b))
            tmp = _store(np.float32(2.0 * a) * prod - A32 @ prod, prec)
            p = p + s * tmp
            if idx != last:
                prod = _store(prod - s * (A32 @ tmp), prec)
    return _store(p, prec)


def apply_phi_low(A32, units, v, prec: str = "fp32") -> np.ndarray:
    """phi(A)v with float32 arithmetic."""
    v = _store(np.asarray(v), prec)
    pi = v.copy()
    for (kind, a, b) in units:
        if kind == REAL:
            pi = _store(pi - np.float32(1.0 / a) * (A32 @ pi), prec)
        else:
            t = _store(A32 @ pi, prec)
            tmp = A32 @ t - np.float32(2.0 * a) * t
            pi = _store(pi + np.float32(1.0 / (a * a + b * b)) * tmp, prec)
    return _store(v - pi, prec)
