"""PP-GMRES(m): the oracle's version.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 4 step 2 of Loe & Morgan: restarted GMRES on phi(A) y = b with
right preconditioning and x = p(A) y, x_0 = 0. Readings (the paper does not
spell these out):

* Each cycle starts from the true residual r = b - A x. The cycle stops
  early when the shortcut residual ||beta e_1 - Hbar z|| (section 3.2,
  Example 3) reaches tol * ||b||, or after m steps.
* The correction is x <- x + p(A)(V_k z); the paper's literal form (one
  y accumulated over cycles, residual b - phi(A) y, a single x = p(A)y at
  the end) is available as ``literal=True``; the two agree to rounding.
* Outer stop: ||b - A x|| <= tol ||b||. NOCONV after max_cycles, or when
  five consecutive cycles together reduce ||r|| by less than 1% (stall;
  stall_cycles = 0 turns this test off).
* The small least-squares problem is solved by numpy's lstsq on Hbar.

Counters follow section 3.1: mvps are sparse products (setup included),
dots are inner products and norms, vops are all length-n vector operations
(dots, norms, axpys and scalings).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import roots as _roots
from .chains import PhiOperator, apply_p, apply_phi, spmv_count_p, spmv_count_phi
from .roots import BREAKDOWN_TOL, REAL

OK, NOCONV = 0, 1


@dataclass
class Info:
    status: int = OK
    cycles: int = 0
    iters: int = 0
    mvps: int = 0
    vops: int = 0
    dots: int = 0
    relres: float = float("nan")
    relres_shortcut: float = float("nan")
    history: list = field(default_factory=list)


def _phi_vops(units) -> int:
    # one axpy per real root, two per pair, one final subtraction
    return sum(1 if k == REAL else 2 for (k, _, _) in units) + 1


def _p_vops(units) -> int:
    # 2r + 3c/2 - 1 axpys (section 3.1), r real and c complex roots
    r = sum(1 for (k, _, _) in units if k == REAL)
    c = 2 * sum(1 for (k, _, _) in units if k != REAL)
    return 2 * r + (3 * c) // 2 - 1


def pp_gmres(A, b: np.ndarray, units, m: int = 50, tol: float = 1e-8, max_cycles: int = 1000,
             orth: str = "mgs", literal: bool = False, stall_cycles: int = 5,
             setup_mvps: int = 0, x0=None, new_poly_degree: int = 0, new_poly_add: bool = True,
             inner_units=None):
    """Solve A x = b by PP(d)-GMRES(m). Returns (x, Info).

    new_poly_degree > 0 is the variant of section 5.2 (ChPoly): at the start
    of every cycle a new polynomial of that degree is built from one GMRES(d)
    cycle whose start vector is the current residual (roots added when
    new_poly_add), and that cycle's phi and p use it; ``units`` is then
    ignored. The setup products count in mvps and its inner products in dots.

    inner_units: a double polynomial (section 6): ``units`` are phi2's and
    the solve uses phi2(phi1(A)) and p1(A) p2(phi1(A)); mvps count products
    with A (each application of phi1(A) is d_eff(phi1) of them).
    """
    if new_poly_degree > 0 and literal:
        raise ValueError("the literal form keeps one polynomial")
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    bnorm = np.linalg.norm(b)
    info = Info(mvps=setup_mvps)
    if inner_units is not None:
        if new_poly_degree > 0 or literal:
            raise ValueError("a double polynomial is fixed")
        op = PhiOperator(A, inner_units)
        n1 = spmv_count_phi(inner_units)
        phi = lambda v: apply_phi(op, units, v)  # noqa: E731
        p_of = lambda v: apply_p(A, inner_units, apply_p(op, units, v))  # noqa: E731
        mv_phi = lambda: spmv_count_phi(units) * n1  # noqa: E731
        mv_p = lambda: spmv_count_p(units) * n1 + spmv_count_p(inner_units)  # noqa: E731
    else:
        phi = lambda v: apply_phi(A, units, v)  # noqa: E731
        p_of = lambda v: apply_p(A, units, v)  # noqa: E731
        mv_phi = lambda: spmv_count_phi(units)  # noqa: E731
        mv_p = lambda: spmv_count_p(units)  # noqa: E731
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    y = np.zeros(n)
    if x0 is None:
        r = b.copy()
    else:
        r = b - A @ x
        info.mvps += 1
    while True:
        beta = np.linalg.norm(r)
        info.dots += 1
        info.vops += 1
        info.relres = beta / bnorm
        info.history.append(info.relres)
        if info.relres <= tol:
            info.status = OK
            break
        if info.cycles >= max_cycles:
            info.status = NOCONV
            break
        h = info.history
        if stall_cycles > 0 and len(h) > stall_cycles and h[-1] > 0.99 * h[-1 - stall_cycles]:
            info.status = NOCONV
            break
        info.cycles += 1
        if new_poly_degree > 0:
            P = _roots.setup(A, r, new_poly_degree, add_roots=new_poly_add, orth=orth)
            units = P.units
            info.mvps += P.d
            info.dots += 1 + sum((2 if orth == "cgs2" else 1) * (j + 1) + 1 for j in range(P.d))
        V = np.zeros((n, m + 1))
        Hb = np.zeros((m + 1, m))
        V[:, 0] = r / beta
        info.vops += 1
        k = 0
        z = np.zeros(0)
        for j in range(m):
            w = phi(V[:, j])
            info.mvps += mv_phi()
            info.vops += _phi_vops(units)
            if orth == "mgs":
                for i in range(j + 1):
                    Hb[i, j] = V[:, i] @ w
                    w = w - Hb[i, j] * V[:, i]
                info.dots += j + 1
                info.vops += 2 * (j + 1)
            else:
                h1 = V[:, : j + 1].T @ w
                w = w - V[:, : j + 1] @ h1
                h2 = V[:, : j + 1].T @ w
                w = w - V[:, : j + 1] @ h2
                Hb[: j + 1, j] = h1 + h2
                info.dots += 2 * (j + 1)
                info.vops += 4 * (j + 1)
            Hb[j + 1, j] = np.linalg.norm(w)
            info.dots += 1
            info.vops += 2
            info.iters += 1
            k = j + 1
            rhs = np.zeros(k + 1)
            rhs[0] = beta
            z, *_ = np.linalg.lstsq(Hb[: k + 1, :k], rhs, rcond=None)
            short = np.linalg.norm(rhs - Hb[: k + 1, :k] @ z)
            info.relres_shortcut = short / bnorm
            lucky = Hb[j + 1, j] <= BREAKDOWN_TOL * np.linalg.norm(Hb[: k + 1, :k])
            if lucky or short <= tol * bnorm:
                break
            V[:, j + 1] = w / Hb[j + 1, j]
        dy = V[:, :k] @ z
        info.vops += k
        if literal:
            y = y + dy
            r = b - phi(y)
            info.mvps += spmv_count_phi(units)
            info.vops += _phi_vops(units) + 2
            # x is formed once at the end; keep it current for the history
        else:
            x = x + p_of(dy)
            info.mvps += mv_p()
            info.vops += _p_vops(units) + 1
            r = b - A @ x
            info.mvps += 1
            info.vops += 1
    if literal:
        x = apply_p(A, units, y)
        info.mvps += spmv_count_p(units)
        info.vops += _p_vops(units)
        info.relres = np.linalg.norm(b - A @ x) / bnorm
    return x, info


def stability_check(A, units, b: np.ndarray) -> float:
    """StCh = ||(b - A p(A) b) - pi(A) b|| (section 3.5).

    r1 = b - A p(A)b uses Algorithm 3, r2 = b - phi(A)b = pi(A)b uses
    Algorithm 1; their difference estimates the attainable residual.
    """
    b = np.asarray(b, dtype=np.float64)
    r1 = b - A @ apply_p(A, units, b)
    r2 = b - apply_phi(A, units, b)
    return float(np.linalg.norm(r1 - r2))


def setup_checked(A, v0: np.ndarray, d: int, b: np.ndarray, tol: float, d_step: int = 0, d_min: int = 1,
                  add_roots: bool = True, orth: str = "mgs"):
    """Polynomial setup followed by the stability check (section 3.5), with
    the degree lowered while the check predicts instability.

    Section 3.5 computes StCh once the polynomial is known, before the
    solve, and lowers the degree when StCh predicts instability. Readings:
    instability is predicted when StCh > tol ||b||. One GMRES(d) cycle runs
    from v0; the polynomial of degree k < d comes from the leading
    (k+1) x k block of its Hessenberg matrix, because the first k Arnoldi
    steps from the same v0 are the GMRES(k) cycle. Degrees d, d - d_step,
    ... (not below d_min) are tried in turn and the first with
    StCh <= tol ||b|| is kept; when none passes, the one with the smallest
    StCh is returned and flagged unstable (NaN counts as infinite).

    Returns (Poly, stch, unstable, tried) with tried = [(k, StCh), ...].
    """
    v0 = np.asarray(v0, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    _, Hbar, k, brk = _roots.arnoldi(lambda v: A @ v, v0, d, orth)
    limit = tol * float(np.linalg.norm(b))
    tried, best = [], None
    kk = k
    while True:
        at_break = brk and kk == k
        theta = _roots.harmonic_ritz(Hbar[: kk + 1, :kk], breakdown=at_break)
        leja, pof, n_add, units = _roots.order_and_add(theta, add_roots)
        P = _roots.Poly(d=kk, theta=theta, leja=leja, pof=pof, n_add=n_add, units=units, breakdown=at_break)
        st = stability_check(A, P.units, b)
        tried.append((kk, st))
        if st <= limit:
            return P, st, False, tried
        key = st if np.isfinite(st) else np.inf
        if best is None or key < best[2]:
            best = (P, st, key)
        if d_step <= 0 or kk - d_step < max(d_min, 1):
            break
        kk -= d_step
    return best[0], best[1], True, tried


def block_jacobi(A, bs: int):
    """The operator A M^{-1} for block-Jacobi (eqs. (1.3)-(1.4) with M the
    block diagonal of A in blocks of bs consecutive rows; the last block
    holds the remaining rows). Each diagonal block is inverted densely
    (numpy.linalg.inv); the polynomial is then built on A M^{-1} (section
    3.1) and x = M^{-1} x~ where x~ solves (A M^{-1}) x~ = b.
    Returns (A M^{-1} as scipy CSR, M^{-1} as scipy CSR)."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    n = A.shape[0]
    blocks = []
    for r0 in range(0, n, bs):
        r1 = min(r0 + bs, n)
        blocks.append(np.linalg.inv(A[r0:r1, r0:r1].toarray()))
    Minv = sp.block_diag(blocks, format="csr")
    return (A @ Minv).tocsr(), Minv


def right_scaled(A, s=None):
    """The operator A M^{-1} for a diagonal right preconditioner M^{-1} =
    diag(s) (eqs. (1.3)-(1.4)); s=None is Jacobi, s_i = 1 / a_ii.

    The polynomial is then built on A M^{-1} (section 3.1: use A M^{-1} for
    the initial GMRES run and the harmonic Ritz values), GMRES solves
    phi(A M^{-1}) y = b, and x = M^{-1} p(A M^{-1}) y = s * x~ where x~ solves
    (A M^{-1}) x~ = b. Entry (i, j) of A M^{-1} is a_ij s_j, one rounding.
    Returns (A M^{-1} as scipy CSR, s). Raises ValueError for Jacobi when a
    diagonal entry is zero or missing.
    """
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    if s is None:
        diag = A.diagonal()
        if np.any(diag == 0.0):
            raise ValueError("zero or missing diagonal entry")
        s = 1.0 / diag
    s = np.asarray(s, dtype=np.float64)
    AS = sp.csr_matrix((A.data * s[A.indices], A.indices.copy(), A.indptr.copy()), shape=A.shape)
    return AS, s
