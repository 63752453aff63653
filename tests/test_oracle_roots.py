"""Pins of the oracle's polynomial construction (section 2, Algorithms 2 and 4)."""

from fractions import Fraction
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import roots
from oracle.roots import REAL, PAIR
from workloads import convdiff2d, diag_example7, diag_squares, diagonal, start_vector, rhs
from _golden import read_kv


def _match_multiset(a, b):
    """Greedy nearest matching of two complex multisets; returns max rel error."""
    a = list(np.asarray(a, dtype=complex))
    b = list(np.asarray(b, dtype=complex))
    assert len(a) == len(b)
    worst = 0.0
    for z in a:
        j = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b[j]) / max(abs(z), 1e-300))
        b.pop(j)
    return worst


# ---------------------------------------------------------------------------
# harmonic Ritz values = roots of the minimum residual polynomial
# ---------------------------------------------------------------------------

def _brute_force_gmres_roots(A, v, d, dps=60):
    """Roots of pi(z) = 1 - sum_j c_j z^j minimising ||pi(A) v|| (mpmath)."""
    with mp.workdps(dps):
        n = A.shape[0]
        Am = mp.matrix(A.tolist())
        vm = mp.matrix([mp.mpf(float(t)) for t in v])
        cols = []
        w = vm
        for _ in range(d):
            w = Am * w
            cols.append(w)
        K = mp.matrix(n, d)
        for j in range(d):
            for i in range(n):
                K[i, j] = cols[j][i]
        G = K.T * K
        rhs_ = K.T * vm
        c = mp.lu_solve(G, rhs_)
        coeffs = [-c[j] for j in reversed(range(d))] + [mp.mpf(1)]
        r = mp.polyroots(coeffs, maxsteps=200, extraprec=200)
        return np.array([complex(z) for z in r])


@pytest.mark.parametrize("seed,n,d", [(0, 8, 3), (1, 10, 4), (2, 12, 5), (3, 9, 6)])
def test_harmonic_ritz_equal_brute_force_min_residual_roots(seed, n, d):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 4 * np.eye(n)  # nonsymmetric, complex spectrum
    v = rng.standard_normal(n)
    for orth in ("mgs", "cgs2"):
        V, H, k, brk = roots.arnoldi(lambda x: A @ x, v, d, orth)
        assert k == d and not brk
        theta = roots.harmonic_ritz(H)
        ref = _brute_force_gmres_roots(A, v, d)
        assert _match_multiset(theta, ref) < 1e-9


def test_d1_closed_form():
    # GMRES(1): theta = ||Av||^2 / (v^T A v)
    A = convdiff2d(12, 3.0).to_scipy()
    v = start_vector(A.shape[0], 5)
    P = roots.setup(A, v, 1)
    Av = A @ v
    expect = (Av @ Av) / (v @ Av)
    assert P.d == 1 and P.theta.imag[0] == 0
    assert abs(P.theta.real[0] - expect) <= 1e-13 * abs(expect)


def test_full_degree_recovers_the_spectrum():
    lam = np.array([0.5, 1.0, 2.0, 3.5, 7.0, 11.0])
    A = diagonal(lam).to_scipy()
    P = roots.setup(A, np.ones(6) + np.arange(6) * 0.1, 6)
    assert P.d == 6
    assert np.max(np.abs(np.sort(P.theta.real) - lam) / lam) < 1e-10
    assert np.all(P.theta.imag == 0)


def test_breakdown_lowers_the_degree():
    lam = np.repeat([1.0, 2.0, 5.0], 10)  # 3 distinct eigenvalues
    A = diagonal(lam).to_scipy()
    P = roots.setup(A, start_vector(30, 3), 10)
    assert P.breakdown and P.d == 3
    assert np.max(np.abs(np.sort(P.theta.real) - [1, 2, 5])) < 1e-10


def test_singular_hessenberg_rejected():
    # A v = 0 makes H_11 = 0: harmonic Ritz values are undefined
    A = np.array([[0.0, 1.0], [0.0, 1.0]])
    with pytest.raises(ValueError):
        roots.setup(A, np.array([1.0, 0.0]), 1)


# ---------------------------------------------------------------------------
# modified Leja ordering
# ---------------------------------------------------------------------------

def test_leja_hand_case():
    # 4 first (largest modulus), then 1 (distance 3); 2 and 3 then tie at
    # exactly 2.0 and the lower canonical index (2) wins.
    perm = roots.leja_order([3.0, 1.0, 4.0, 2.0], [0, 0, 0, 0])
    assert [[3.0, 1.0, 4.0, 2.0][i] for i in perm] == [4.0, 1.0, 2.0, 3.0]


def _exact_leja_real(xs):
    """Modified Leja order with exact rational products (real roots)."""
    xs = [Fraction(x) for x in xs]
    canon = sorted(range(len(xs)), key=lambda i: xs[i])
    order = []
    left = list(canon)
    first = max(left, key=lambda i: (abs(xs[i]), -canon.index(i)))
    order.append(first)
    left.remove(first)
    while left:
        def score(i):
            s = Fraction(1)
            for j in order:
                s *= abs(xs[i] - xs[j])
            return s
        best = None
        for i in left:  # left is in canonical order: strict > keeps the lowest index
            if best is None or score(i) > score(best):
                best = i
        order.append(best)
        left.remove(best)
    return order


@pytest.mark.parametrize("seed", range(6))
def test_leja_real_matches_exact_arithmetic_on_integers(seed):
    # integer roots: the products are exact in double too, so ties are exact
    rng = np.random.default_rng(seed)
    xs = [float(t) for t in rng.integers(-9, 30, size=14) if t != 0]
    perm = roots.leja_order(xs, [0.0] * len(xs))
    exact = _exact_leja_real(xs)
    assert [xs[i] for i in perm] == [xs[i] for i in exact]


@pytest.mark.parametrize("seed", range(6))
def test_leja_real_matches_exact_arithmetic_random(seed):
    rng = np.random.default_rng(100 + seed)
    xs = list(rng.uniform(0.01, 10.0, size=25))
    perm = roots.leja_order(xs, [0.0] * len(xs))
    exact = _exact_leja_real(xs)
    assert list(perm) == exact


def _mp_leja_complex(re, im, dps=80):
    """Modified Leja with units, scores in high precision (no ties expected)."""
    with mp.workdps(dps):
        units = [(re[i], im[i], i) for i in range(len(re)) if im[i] >= 0]
        units.sort(key=lambda u: (u[0], u[1]))
        pts = [mp.mpc(u[0], u[1]) for u in units]
        placed = []
        order = []
        first = max(range(len(units)), key=lambda u: (abs(pts[u]), -u))
        cur = first
        while True:
            order.append(cur)
            placed.append(pts[cur])
            if units[cur][1] != 0:
                placed.append(mp.conj(pts[cur]))
            if len(order) == len(units):
                break
            best, bs = None, None
            for u in range(len(units)):
                if u in order:
                    continue
                s = mp.mpf(1)
                for z in placed:
                    s *= abs(pts[u] - z)
                if bs is None or s > bs:
                    best, bs = u, s
            cur = best
        out = []
        for u in order:
            a, b, _ = units[u]
            out.append(complex(a, b))
            if b != 0:
                out.append(complex(a, -b))
        return out


@pytest.mark.parametrize("seed", range(5))
def test_leja_complex_matches_high_precision(seed):
    rng = np.random.default_rng(200 + seed)
    re, im = [], []
    for _ in range(6):
        a, b = rng.uniform(-3, 5), rng.uniform(0.1, 2)
        re += [a, a]
        im += [b, -b]
    for _ in range(5):
        re.append(rng.uniform(-3, 5))
        im.append(0.0)
    order = rng.permutation(len(re))
    re = [re[i] for i in order]
    im = [im[i] for i in order]
    perm = roots.leja_order(re, im)
    got = [complex(re[i], im[i]) for i in perm]
    assert got == _mp_leja_complex(re, im)


def test_leja_properties():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((40, 40))
    theta = np.linalg.eigvals(A)
    perm = roots.leja_order(theta.real, theta.imag)
    assert sorted(perm) == list(range(40))
    o = theta[perm]
    assert abs(o[0]) == np.max(np.abs(theta))
    i = 0
    while i < 40:
        if o[i].imag != 0:
            assert o[i].imag > 0 and o[i + 1] == np.conj(o[i])
            i += 2
        else:
            i += 1


# ---------------------------------------------------------------------------
# pof and added roots (Algorithm 2)
# ---------------------------------------------------------------------------

def _pof_float(me):
    return math.ldexp(*me)


def test_pof_hand_cases():
    # {1, 100}: pof(100) = |1 - 100| = 99, pof(1) = |1 - 1/100| = 0.99: nothing added
    _, pof, n_add, units = roots.order_and_add(np.array([1.0, 100.0]))
    assert [u[1] for u in units] == [100.0, 1.0]
    assert _pof_float(pof[0]) == 99.0 and abs(_pof_float(pof[1]) - 0.99) < 1e-15
    assert n_add == [0, 0]
    # {1, 1e5}: pof(1e5) = 99999 >= 1e4: one copy, appended at the end
    _, pof, n_add, units = roots.order_and_add(np.array([1.0, 1e5]))
    assert n_add == [1, 0]
    assert [u[1] for u in units] == [1e5, 1.0, 1e5]
    # pof exactly 1e4: the least integer greater than 0 is 1
    _, pof, n_add, _ = roots.order_and_add(np.array([1.0, 10001.0]))
    assert _pof_float(pof[0]) == 1e4 and n_add[0] == 1
    # pof >= 1e18 adds a second copy
    _, pof, n_add, _ = roots.order_and_add(np.array([1.0, 1e19]))
    assert n_add[0] == 2


def test_pof_matches_definition_and_conjugates_agree():
    # pof(k) = prod_{i != k} |1 - theta_k/theta_i|, evaluated here with complex
    # division in 50-digit arithmetic; both members of a pair give the same value
    th = np.array([3 + 2j, 3 - 2j, 0.5, 7.0, -1 + 0.5j, -1 - 0.5j, 12.0])
    leja, pof, _, _ = roots.order_and_add(th)
    units = roots._unit_list(leja.real, leja.imag)
    with mp.workdps(50):
        for u, me in zip(units, pof):
            members = [u[3]] if u[0] == REAL else [u[3], u[3] + 1]
            for k in members:
                direct = mp.mpf(1)
                for i, z in enumerate(leja):
                    if i != k:
                        direct *= abs(1 - mp.mpc(leja[k]) / mp.mpc(z))
                assert abs(float(direct) - _pof_float(me)) <= 1e-13 * float(direct)


def test_spd_smallest_root_never_gets_a_copy():
    # SPD: |1 - theta_1/theta_i| < 1 for the smallest theta_1, so pof(1) < 1
    A = convdiff2d(30).to_scipy()
    P = roots.setup(A, start_vector(A.shape[0], 2), 30)
    units = roots._unit_list(P.leja.real, P.leja.imag)
    k = int(np.argmin([u[1] for u in units]))
    assert _pof_float(P.pof[k]) < 1.0 and P.n_add[k] == 0


def test_example7_added_roots(golden_dir):
    g = read_kv("example7_pof.txt")
    A = diag_example7().to_scipy()
    P = roots.setup(A, start_vector(A.shape[0], 2), int(g["degree"]))
    assert P.n_added == int(g["added_roots"])
    units = roots._unit_list(P.leja.real, P.leja.imag)
    added = {}
    for k, c in enumerate(P.n_add):
        if c:
            added[round(units[k][1])] = _pof_float(P.pof[k])
    assert set(added) == {int(g["root_1"]), int(g["root_2"])}
    # the start vector is random: agree with the printed pof within half a decade
    assert abs(math.log10(added[int(g["root_1"])] / g["pof_1"])) < 0.5
    assert abs(math.log10(added[int(g["root_2"])] / g["pof_2"])) < 0.5


@pytest.mark.slow
def test_table4_1_degree512_adds_four_roots(golden_dir):
    g = read_kv("table4_1_d512.txt")
    A = diag_squares(int(g["n"])).to_scipy()
    # CGS2 for speed (the paper used MGS); the roots agree to rounding
    P = roots.setup(A, start_vector(A.shape[0], 2), int(g["degree"]), orth="cgs2")
    assert P.n_added == int(g["added_roots"])


# ---------------------------------------------------------------------------
# insertion of added roots (positions: parity unpinned, properties pinned)
# ---------------------------------------------------------------------------

def test_insertion_reading_example():
    # units A B C D with 2 copies of B and 1 of D (rule stated in oracle.roots)
    out = roots.insert_roots([REAL] * 4, [1.0, 2.0, 3.0, 4.0], [0.0] * 4, [0, 2, 0, 1])
    assert [u[1] for u in out] == [1.0, 2.0, 3.0, 2.0, 4.0, 2.0, 4.0]


def test_insertion_copies_shift_later_units():
    # Units U0 (real, 2 copies), U1 (real, none), U2 (pair, 3 copies), U3
    # (real, none), worked by hand from the rule "copy j of c goes to
    # s + 1 + floor(j (L - s - 1) / c)", with s the unit's current index and L
    # the list length before its copies:
    #   U0: s = 0, L = 4: j = 2 -> 1 + 3 = 4 (the end), j = 1 -> 1 + 1 = 2
    #       list U0 U1 U0' U2 U3 U0'
    #   U2: the copies of U0 moved it: s = 3, L = 6:
    #       j = 3 -> 4 + 2 = 6 (the end), j = 2 -> 4 + 1 = 5, j = 1 -> 4 + 0 = 4
    #       list U0 U1 U0' U2 U2' U3 U2' U0' U2'
    # and the pair keeps its two members together in the root list
    out = roots.insert_roots([REAL, REAL, PAIR, REAL], [1.0, 2.0, 3.0, 4.0], [0.0, 0.0, 0.5, 0.0], [2, 0, 3, 0])
    assert [u[1] for u in out] == [1.0, 2.0, 1.0, 3.0, 3.0, 4.0, 3.0, 1.0, 3.0]
    assert [u[0] for u in out] == [REAL, REAL, REAL, PAIR, PAIR, REAL, PAIR, REAL, PAIR]
    P = roots.Poly(d=5, theta=np.zeros(5), leja=np.zeros(5), pof=[], n_add=[], units=out)
    r = P.roots()
    assert P.d_eff == 13 and P.n_added == 8
    assert list(r[3:5]) == [3 + 0.5j, 3 - 0.5j] and list(r[11:13]) == [3 + 0.5j, 3 - 0.5j]


@pytest.mark.parametrize("seed", range(8))
def test_insertion_properties(seed):
    rng = np.random.default_rng(seed)
    nu = int(rng.integers(1, 12))
    kinds = [int(k) for k in rng.integers(0, 2, size=nu)]
    re = [float(i + 1) for i in range(nu)]
    im = [1.5 if k == PAIR else 0.0 for k in kinds]
    n_add = [int(c) for c in rng.integers(0, 4, size=nu)]
    out = roots.insert_roots(kinds, re, im, n_add)
    ids = [int(u[1]) - 1 for u in out]
    # multiset: every unit once plus its copies; kinds travel with the unit
    assert sorted(ids) == sorted(sum([[k] * (1 + n_add[k]) for k in range(nu)], []))
    assert all(out[i][0] == kinds[ids[i]] for i in range(len(out)))
    # copies come after the original occurrence
    for k in range(nu):
        pos = [i for i, u in enumerate(ids) if u == k]
        assert len(pos) == 1 + n_add[k]
    # the first copy of the first unit that gets copies is appended at the end
    firsts = [k for k in range(nu) if n_add[k]]
    if firsts:
        k0 = firsts[0]
        tail = roots.insert_roots(kinds[: k0 + 1], re[: k0 + 1], im[: k0 + 1], n_add[: k0 + 1])
        assert int(tail[-1][1]) - 1 == k0
