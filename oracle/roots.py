"""Polynomial construction for PP-GMRES: the oracle's version.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Algorithm 4 step 1 of Loe & Morgan (one GMRES(d) cycle from a random
vector, harmonic Ritz values, modified Leja ordering, Algorithm 2 for added
roots). Readings of passages the paper leaves open are stated next to the
code that implements them:

* degree: d harmonic Ritz values are the roots of pi and phi (degree d);
  p has degree d-1 (section 1).
* modified Leja ordering (section 2 cites Bai, Hu & Reichel, alg. 3.1, but
  does not restate it): a real root is one unit, a conjugate pair is one
  unit represented by its member with positive imaginary part. The first
  unit has the largest modulus; each next unit maximises the product of its
  distances to all roots already placed (both members of placed pairs).
  Exact ties go to the lowest canonical index (units sorted stably by
  (real, imag)). A pair is emitted as (a+bi, a-bi).
* "logs of products" against overflow (Algorithm 2 step 1) is realised as an
  exact renormalisation: every running product is kept as mantissa and
  binary exponent (frexp after each multiply). The ordering is then the one
  exact products would give up to one rounding per multiply, and it is
  reproducible bit for bit in any IEEE double implementation.
* pof(k) (Algorithm 2 step 2) runs over the d original roots i != k in Leja
  order, each factor |theta_i - theta_k| / |theta_i|; a pair uses its
  +imag member (both members have equal pof).
* number of copies (Algorithm 2 step 3): the least integer greater than
  (log10 pof - 4)/14, clamped at zero, i.e. the number of thresholds
  10^4, 10^18, 10^32, ... that pof reaches (pof >= threshold).
* insertion: original units are processed in Leja order. With c copies for
  unit k, s its current index in the unit list and L the list length, copy
  j (j = c..1) goes to index s + 1 + floor(j (L - s - 1) / c): the first copy
  at the end, the others spread evenly between the occurrence and the end.
  Pairs stay together because the list holds units.
* breakdown of the setup cycle (not discussed in the paper): when
  h_{k+1,k} <= 1e-14 ||H_{:,1:k}||_F the Krylov space is invariant, the
  degree drops to k and the roots are eig(H_kk).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BREAKDOWN_TOL = 1e-14
REAL, PAIR = 0, 1
MAX_THRESHOLDS = 22  # 10^4 .. 10^298: the thresholds that are finite doubles


# ---------------------------------------------------------------------------
# GMRES(d) setup cycle: Arnoldi (Algorithm 4 step 1a)
# ---------------------------------------------------------------------------

def arnoldi(op, v0: np.ndarray, d: int, orth: str = "mgs"):
    """Arnoldi process A V_k = V_{k+1} Hbar_{k+1,k} from v0.

    op: callable returning the operator applied to a vector.
    orth: "mgs" (modified Gram-Schmidt, as the paper's experiments use) or
    "cgs2" (classical Gram-Schmidt applied twice).
    Returns (V, Hbar, k, breakdown) with k <= d the Krylov dimension reached.
    """
    n = v0.shape[0]
    V = np.zeros((n, d + 1))
    H = np.zeros((d + 1, d))
    V[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(d):
        w = op(V[:, j])
        if orth == "mgs":
            for i in range(j + 1):
                H[i, j] = V[:, i] @ w
                w = w - H[i, j] * V[:, i]
        elif orth == "cgs2":
            h1 = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h1
            h2 = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h2
            H[: j + 1, j] = h1 + h2
        else:
            raise ValueError(orth)
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= BREAKDOWN_TOL * np.linalg.norm(H[: j + 2, : j + 1]):
            return V[:, : j + 2], H[: j + 2, : j + 1], j + 1, True
        V[:, j + 1] = w / H[j + 1, j]
    return V, H, d, False


# ---------------------------------------------------------------------------
# Harmonic Ritz values (Algorithm 4 step 1b)
# ---------------------------------------------------------------------------

def harmonic_ritz(Hbar: np.ndarray, breakdown: bool = False) -> np.ndarray:
    """Roots of the GMRES polynomial from the (k+1) x k Hessenberg matrix.

    The roots are the eigenvalues of H_kk + h_{k+1,k}^2 f e_k^T where f solves
    H_kk^T f = e_k (the paper's H^{-*} is the transpose for real A). After a
    breakdown the last row is zero and the roots are eig(H_kk).
    Raises ValueError if H_kk is singular or a root is zero.
    """
    k = Hbar.shape[1]
    H = Hbar[:k, :k].copy()
    M = H.copy()
    if not breakdown:
        h = Hbar[k, k - 1]
        ek = np.zeros(k)
        ek[-1] = 1.0
        try:
            f = np.linalg.solve(H.T, ek)
        except np.linalg.LinAlgError as exc:  # singular H_kk
            raise ValueError("singular H_kk") from exc
        if not np.all(np.isfinite(f)):
            raise ValueError("singular H_kk")
        M[:, k - 1] += h * h * f
    theta = np.linalg.eigvals(M)
    if np.any(theta == 0) or not np.all(np.isfinite(theta)):
        raise ValueError("zero or non-finite harmonic Ritz value")
    return theta.astype(np.complex128)


# ---------------------------------------------------------------------------
# Exact mantissa/exponent products
# ---------------------------------------------------------------------------

def _me_mul(me, f: float):
    m, e = me
    m2, e2 = math.frexp(m * f)
    return (m2, e + e2)


def _me_greater(a, b) -> bool:
    """a > b for non-negative numbers held as (mantissa, exponent)."""
    ma, ea = a
    mb, eb = b
    if ma == 0.0:
        return False
    if mb == 0.0:
        return True
    if ea != eb:
        return ea > eb
    return ma > mb


def _me_geq(a, b) -> bool:
    return not _me_greater(b, a)


def _absdiff(ar: float, ai: float, br: float, bi: float) -> float:
    dr = ar - br
    di = ai - bi
    return math.sqrt(dr * dr + di * di)


# ---------------------------------------------------------------------------
# Modified Leja ordering (section 2; Algorithm 2 step 1)
# ---------------------------------------------------------------------------

def _units_from_roots(re, im):
    """Group roots into units: (kind, re, im, idx_plus, idx_minus)."""
    re = [float(x) for x in re]
    im = [float(x) for x in im]
    units = []
    minus_pool = {}
    for i, (a, b) in enumerate(zip(re, im)):
        if b < 0:
            minus_pool.setdefault((a, -b), []).append(i)
    taken = {key: 0 for key in minus_pool}
    for i, (a, b) in enumerate(zip(re, im)):
        if b == 0:
            units.append((REAL, a, 0.0, i, -1))
        elif b > 0:
            key = (a, b)
            pool = minus_pool.get(key, [])
            t = taken.get(key, 0)
            if t >= len(pool):
                raise ValueError("complex root without its conjugate")
            units.append((PAIR, a, b, i, pool[t]))
            taken[key] = t + 1
    n_minus = sum(len(v) for v in minus_pool.values())
    if n_minus != sum(taken.values()):
        raise ValueError("complex root without its conjugate")
    return units


def leja_order(re, im) -> np.ndarray:
    """Modified Leja permutation of the roots (re[i] + 1j im[i]).

    Returns perm (int array of length d) such that the ordered roots are
    (re[perm], im[perm]); conjugate pairs are adjacent, +imag first.
    """
    units = _units_from_roots(re, im)
    # canonical index: stable sort by (real, imag)
    canon = sorted(range(len(units)), key=lambda u: (units[u][1], units[u][2]))
    units = [units[u] for u in canon]
    nu = len(units)
    placed = [False] * nu
    order = []
    # first unit: largest modulus
    best = -1
    best_mod = -1.0
    for u in range(nu):
        a, b = units[u][1], units[u][2]
        mod = math.sqrt(a * a + b * b)
        if mod > best_mod:
            best, best_mod = u, mod
    scores = [(0.5, 1)] * nu  # the empty product, 1.0 = 0.5 * 2^1
    while True:
        placed[best] = True
        order.append(best)
        kind, a, b = units[best][0], units[best][1], units[best][2]
        new_roots = [(a, b)] if kind == REAL else [(a, b), (a, -b)]
        for u in range(nu):
            if placed[u]:
                continue
            ua, ub = units[u][1], units[u][2]
            s = scores[u]
            for (ra, rb) in new_roots:
                s = _me_mul(s, _absdiff(ua, ub, ra, rb))
            scores[u] = s
        if len(order) == nu:
            break
        best = -1
        for u in range(nu):
            if placed[u]:
                continue
            if best < 0 or _me_greater(scores[u], scores[best]):
                best = u
    perm = []
    for u in order:
        kind, _, _, ip, imn = units[u]
        perm.append(ip)
        if kind == PAIR:
            perm.append(imn)
    return np.asarray(perm, dtype=np.int64)


# ---------------------------------------------------------------------------
# pof and number of added roots (Algorithm 2 steps 2 and 3)
# ---------------------------------------------------------------------------

def _unit_list(re, im):
    """Units of an ordered root list: (kind, re, im, root_position)."""
    out = []
    i = 0
    d = len(re)
    while i < d:
        if im[i] == 0:
            out.append((REAL, float(re[i]), 0.0, i))
            i += 1
        else:
            if i + 1 >= d or re[i + 1] != re[i] or im[i + 1] != -im[i] or im[i] < 0:
                raise ValueError("ordered roots must hold conjugate pairs as (a+bi, a-bi)")
            out.append((PAIR, float(re[i]), float(im[i]), i))
            i += 2
    return out


def pof_values(re, im):
    """pof for every unit of a Leja-ordered root list, as (mantissa, exponent).

    pof(k) = prod_{i != k} |1 - theta_k/theta_i| over the original roots,
    each factor evaluated as |theta_i - theta_k| / |theta_i|, multiplied in
    list order with exact renormalisation.
    """
    re = [float(x) for x in re]
    im = [float(x) for x in im]
    units = _unit_list(re, im)
    out = []
    for (_, a, b, pos) in units:
        s = (0.5, 1)
        for i in range(len(re)):
            if i == pos:
                continue
            num = _absdiff(re[i], im[i], a, b)
            den = math.sqrt(re[i] * re[i] + im[i] * im[i])
            s = _me_mul(s, num / den)
        out.append(s)
    return out


def n_add_from_pof(pof_me) -> int:
    """Copies to add for one unit: #{j >= 0 : pof >= 10^(4+14j)}."""
    count = 0
    for j in range(MAX_THRESHOLDS):
        t = math.frexp(float("1e%d" % (4 + 14 * j)))
        if _me_geq(pof_me, t):
            count += 1
        else:
            break
    return count


def insert_roots(unit_kinds, unit_re, unit_im, n_add):
    """Insert n_add[k] copies of every unit k (units in Leja order).

    Returns the final unit list as (kind, re, im) tuples.
    """
    R = [(k, False) for k in range(len(unit_kinds))]  # (unit id, is_copy)
    for k in range(len(unit_kinds)):
        c = int(n_add[k])
        if c == 0:
            continue
        s = R.index((k, False))
        L = len(R)
        for j in range(c, 0, -1):
            q = s + 1 + (j * (L - s - 1)) // c
            R.insert(q, (k, True))
    return [(unit_kinds[k], unit_re[k], unit_im[k]) for (k, _) in R]


# ---------------------------------------------------------------------------
# Whole setup (Algorithm 4 step 1)
# ---------------------------------------------------------------------------

@dataclass
class Poly:
    """The preconditioning polynomial as an ordered list of units."""

    d: int  # degree reached by the setup cycle (number of harmonic Ritz values)
    theta: np.ndarray  # raw harmonic Ritz values (eigensolver order)
    leja: np.ndarray  # Leja-ordered roots (complex)
    pof: list  # (mantissa, exponent) per Leja unit
    n_add: list  # copies added per Leja unit
    units: list = field(default_factory=list)  # final (kind, re, im) list
    breakdown: bool = False

    @property
    def d_eff(self) -> int:
        return sum(1 if k == REAL else 2 for (k, _, _) in self.units)

    @property
    def n_added(self) -> int:
        return self.d_eff - self.d

    def roots(self) -> np.ndarray:
        out = []
        for (k, a, b) in self.units:
            if k == REAL:
                out.append(complex(a, 0.0))
            else:
                out.extend([complex(a, b), complex(a, -b)])
        return np.asarray(out, dtype=np.complex128)

    def pof_float(self) -> np.ndarray:
        return np.asarray([math.ldexp(m, e) if e < 1024 else math.inf for (m, e) in self.pof])


def order_and_add(theta: np.ndarray, add_roots: bool = True):
    """Leja order, pof, n_add and insertion for given roots."""
    re = np.real(theta).astype(np.float64)
    im = np.imag(theta).astype(np.float64)
    perm = leja_order(re, im)
    ore, oim = re[perm], im[perm]
    pof = pof_values(ore, oim)
    units = _unit_list(ore, oim)
    kinds = [u[0] for u in units]
    ures = [u[1] for u in units]
    uims = [u[2] for u in units]
    n_add = [n_add_from_pof(p) if add_roots else 0 for p in pof]
    final = insert_roots(kinds, ures, uims, n_add)
    return ore + 1j * oim, pof, n_add, final


def setup(A, v0: np.ndarray, d: int, add_roots: bool = True, orth: str = "mgs") -> Poly:
    """Build the polynomial from one GMRES(d) cycle on A from v0.

    A: anything supporting ``A @ v`` (scipy sparse or numpy).
    """
    V, Hbar, k, brk = arnoldi(lambda v: A @ v, np.asarray(v0, dtype=np.float64), d, orth)
    theta = harmonic_ritz(Hbar, breakdown=brk)
    leja, pof, n_add, units = order_and_add(theta, add_roots)
    return Poly(d=k, theta=theta, leja=leja, pof=pof, n_add=n_add, units=units, breakdown=brk)


def poly_from_roots(theta, add_roots: bool = False) -> Poly:
    """A polynomial with given roots (Leja-ordered, optionally with added roots)."""
    theta = np.asarray(theta, dtype=np.complex128)
    leja, pof, n_add, units = order_and_add(theta, add_roots)
    return Poly(d=theta.size, theta=theta, leja=leja, pof=pof, n_add=n_add, units=units)


def setup_double(A, inner_units, v0: np.ndarray, d2: int, add_roots: bool = True, orth: str = "mgs") -> Poly:
    """The outer polynomial phi2 of a double polynomial (section 6): one
    GMRES(d2) cycle with the matrix phi1(A) (inner_units) from v0, then the
    harmonic Ritz values, Leja order and added roots of Algorithm 4 step 1
    and Algorithm 2, all in the variable of phi1(A)."""
    from .chains import PhiOperator

    return setup(PhiOperator(A, inner_units), v0, d2, add_roots, orth)
