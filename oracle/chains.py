"""phi(A)v and p(A)v by the root-product chains: the oracle's version.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A polynomial is a list of units (kind, re, im) in application order: a real
root theta (kind 0, im = 0) or a conjugate pair a +/- bi (kind 1, im = b > 0).

* pi(alpha) = prod_i (1 - alpha/theta_i)  (eq. 2.1); a conjugate pair folds
  into the real factor 1 + (alpha^2 - 2 a alpha)/(a^2 + b^2)  (eq. 2.2).
* phi(A)v = v - pi(A)v  (Algorithm 1).
* p(A)v = sum_k u_k(A)v with u_k = (1/theta_k) prod_{i<k} (1 - A/theta_i)
  (eq. 3.1); a pair contributes prod * (2a - A)/(a^2 + b^2) and then
  advances the product by the folded factor (Algorithm 3). The final unit
  only contributes to the sum: its product update would be unused.
"""

from __future__ import annotations

import numpy as np

REAL, PAIR = 0, 1


def apply_pi(A, units, v: np.ndarray) -> np.ndarray:
    """pi(A)v, the GMRES residual polynomial applied to v (eq. 2.1/2.2)."""
    pi = np.array(v, dtype=np.float64, copy=True)
    for (kind, a, b) in units:
        if kind == REAL:
            pi = pi - (1.0 / a) * (A @ pi)
        else:
            prod = A @ pi
            tmp = A @ prod - 2.0 * a * prod
            pi = pi + (1.0 / (a * a + b * b)) * tmp
    return pi


def apply_phi(A, units, v: np.ndarray) -> np.ndarray:
    """phi(A)v = v - pi(A)v  (Algorithm 1)."""
    v = np.asarray(v, dtype=np.float64)
    return v - apply_pi(A, units, v)


def apply_p(A, units, v: np.ndarray) -> np.ndarray:
    """p(A)v with phi(alpha) = alpha p(alpha)  (Algorithm 3)."""
    prod = np.array(v, dtype=np.float64, copy=True)
    p = np.zeros_like(prod)
    last = len(units) - 1
    for idx, (kind, a, b) in enumerate(units):
        if kind == REAL:
            p = p + (1.0 / a) * prod
            if idx != last:
                prod = prod - (1.0 / a) * (A @ prod)
        else:
            s = 1.0 / (a * a + b * b)
            tmp = 2.0 * a * prod - A @ prod
            p = p + s * tmp
            if idx != last:
                prod = prod - s * (A @ tmp)
    return p


def spmv_count_phi(units) -> int:
    return sum(1 if k == REAL else 2 for (k, _, _) in units)


def spmv_count_p(units) -> int:
    last = len(units) - 1
    c = 0
    for idx, (k, _, _) in enumerate(units):
        if k == REAL:
            c += 0 if idx == last else 1
        else:
            c += 1 if idx == last else 2
    return c


# ---------------------------------------------------------------------------
# double polynomial (section 6): phi2(phi1(A)) and p1(A) p2(phi1(A))
# ---------------------------------------------------------------------------

class PhiOperator:
    """phi1(A) as an operator, ``op @ v = phi1(A) v`` (Algorithm 1): the
    matrix of the second GMRES run of a double polynomial, and the variable
    in which phi2's roots live."""

    def __init__(self, A, units):
        self.A = A
        self.units = units
        self.shape = A.shape

    def __matmul__(self, v):
        return apply_phi(self.A, self.units, v)


def apply_phi_double(A, inner, outer, v: np.ndarray) -> np.ndarray:
    """phi2(phi1(A)) v: Algorithm 1 for phi2 with phi1(A) as the matrix."""
    return apply_phi(PhiOperator(A, inner), outer, v)


def apply_pi_double(A, inner, outer, v: np.ndarray) -> np.ndarray:
    """pi2(phi1(A)) v = v - phi2(phi1(A)) v."""
    return apply_pi(PhiOperator(A, inner), outer, v)


def apply_p_double(A, inner, outer, v: np.ndarray) -> np.ndarray:
    """p(A) v with A p(A) = phi2(phi1(A)): since phi1(a) = a p1(a) and
    phi2(a) = a p2(a), p(A) = p1(A) p2(phi1(A)) (section 6)."""
    return apply_p(A, inner, apply_p(PhiOperator(A, inner), outer, v))
