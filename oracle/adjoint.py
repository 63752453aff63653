"""Gradient of a loss through the solution of A x = b: the oracle's version.

TEST INFRASTRUCTURE ONLY (see the package docstring).

No passage of the paper covers differentiation. For L(x) with x = A^{-1} b
and g = dL/dx, the adjoint lambda solves A^T lambda = g; then dL/db = lambda
and dL/dA_ij = -lambda_i x_j, so a stored nonzero k at (row_k, col_k) has
dL/dval_k = -lambda[row_k] * x[col_k]. The oracle uses a direct sparse solve
(SuperLU through scipy) for both x and lambda.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla


def solve_direct(A, b):
    return sla.spsolve(A.tocsc(), b)


def grad_direct(A, b, g_fn):
    """Returns (x, lambda, dval) for the loss whose gradient in x is g_fn(x)."""
    A = A.tocsr()
    x = solve_direct(A, b)
    g = g_fn(x)
    lam = sla.spsolve(A.T.tocsc(), g)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    dval = -lam[rows] * x[A.indices]
    return x, lam, dval
