"""Pins of the oracle's polynomial chains (Algorithms 1 and 3, eqs. 2.1, 2.2, 3.1)."""

import mpmath as mp
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import chains, roots
from oracle.chains import spmv_count_p, spmv_count_phi
from workloads import convdiff2d, diagonal, start_vector


def _units_from(theta):
    return roots.poly_from_roots(np.asarray(theta, dtype=complex)).units


def _random_roots(rng, n_real, n_pair):
    th = list(rng.uniform(0.5, 6.0, size=n_real))
    for _ in range(n_pair):
        a, b = rng.uniform(0.5, 5.0), rng.uniform(0.2, 2.0)
        th += [complex(a, b), complex(a, -b)]
    return np.array(th, dtype=complex)


def _mp_pi(lam, theta):
    prod = mp.mpc(1)
    for t in theta:
        prod *= 1 - mp.mpf(lam) / mp.mpc(t)
    return prod


@pytest.mark.parametrize("seed,n_real,n_pair", [(0, 5, 0), (1, 0, 3), (2, 4, 3), (3, 1, 1), (4, 7, 5)])
def test_diagonal_closed_form(seed, n_real, n_pair):
    # For A = diag(lam): p(A)v = p(lam) * v with p(z) = (1 - pi(z))/z and
    # phi(A)v = (1 - pi(lam)) * v, pi(z) = prod (1 - z/theta_i).
    rng = np.random.default_rng(seed)
    theta = _random_roots(rng, n_real, n_pair)
    units = _units_from(theta)
    lam = rng.uniform(0.1, 6.5, size=40)
    v = rng.standard_normal(40)
    A = sp.diags(lam).tocsr()
    got_p = chains.apply_p(A, units, v)
    got_phi = chains.apply_phi(A, units, v)
    with mp.workdps(50):
        pis = [_mp_pi(l, theta) for l in lam]
        exp_p = np.array([float(mp.re((1 - q) / l)) for q, l in zip(pis, lam)]) * v
        exp_phi = np.array([float(mp.re(1 - q)) for q in pis]) * v
    assert np.max(np.abs(got_p - exp_p)) <= 1e-12 * np.max(np.abs(exp_p))
    assert np.max(np.abs(got_phi - exp_phi)) <= 1e-12 * np.max(np.abs(exp_phi))


def _realified(theta):
    """Block-diagonal real matrix whose eigenvalues are exactly the roots."""
    blocks = []
    for (k, a, b) in _units_from(theta):
        if k == 0:
            blocks.append(np.array([[a]]))
        else:
            blocks.append(np.array([[a, b], [-b, a]]))
    return sp.block_diag(blocks).tocsr()


@pytest.mark.parametrize("seed", range(4))
def test_phi_is_identity_on_its_roots(seed):
    # pi vanishes at every root, so for a matrix whose spectrum is the roots
    # (each simple) pi(A) = 0, phi(A) = I and A p(A) = I (i.e. z p(z) = 1).
    rng = np.random.default_rng(10 + seed)
    theta = _random_roots(rng, 4, 3)
    A = _realified(theta)
    units = _units_from(theta)
    v = rng.standard_normal(A.shape[0])
    assert np.linalg.norm(chains.apply_phi(A, units, v) - v) <= 1e-10 * np.linalg.norm(v)
    assert np.linalg.norm(A @ chains.apply_p(A, units, v) - v) <= 1e-10 * np.linalg.norm(v)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_gmres_d_equivalence(d):
    # With the roots from one GMRES(d) cycle on v, pi(A)v is that cycle's
    # residual and p(A)v its iterate (section 2). The reference is a least
    # squares fit over the Krylov basis by numpy QR, independent of Arnoldi.
    A = convdiff2d(10, 7.0).to_scipy()
    v = start_vector(A.shape[0], 4)
    v = v / np.linalg.norm(v)
    P = roots.setup(A, v, d, add_roots=False)
    K = np.empty((v.size, d))
    w = v.copy()
    for j in range(d):
        K[:, j] = w
        w = A @ w
    AK = A @ K
    Q, R = np.linalg.qr(AK)
    c = np.linalg.solve(R, Q.T @ v)
    x_ref = K @ c
    r_ref = v - A @ x_ref
    r_or = v - chains.apply_phi(A, P.units, v)
    x_or = chains.apply_p(A, P.units, v)
    assert np.linalg.norm(r_or - r_ref) <= 1e-10 * np.linalg.norm(r_ref) + 1e-14
    assert np.linalg.norm(x_or - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


def test_p_and_phi_consistent():
    # phi(A)v = A p(A)v (phi(z) = z p(z)), stability check of section 3.5 ~ 0
    A = convdiff2d(20, 1.0).to_scipy()
    P = roots.setup(A, start_vector(A.shape[0], 2), 12)
    v = start_vector(A.shape[0], 9)
    a = chains.apply_phi(A, P.units, v)
    b = A @ chains.apply_p(A, P.units, v)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


def test_spmv_counts():
    th = np.array([1.0, 2 + 1j, 2 - 1j, 3.0])
    units = _units_from(th)
    assert spmv_count_phi(units) == 4  # d_eff
    assert spmv_count_p(units) == 3  # d_eff - 1
    units2 = _units_from(np.array([1.0, 2 + 1j, 2 - 1j, 5 + 1j, 5 - 1j]))
    assert spmv_count_phi(units2) == 5 and spmv_count_p(units2) == 4


def test_pair_factor_identity():
    # eq. 2.2 on a scalar: (1 - z/t)(1 - z/conj t) = 1 + (z^2 - 2 a z)/(a^2 + b^2)
    a, b = 1.3, 0.7
    t = complex(a, b)
    for z in [0.3, 1.0, 2.5, -1.0]:
        lhs = (1 - z / t) * (1 - z / t.conjugate())
        rhs = 1 + (z * z - 2 * a * z) / (a * a + b * b)
        assert abs(lhs - rhs) < 1e-14
        A = sp.csr_matrix(np.array([[z]]))
        pi = chains.apply_pi(A, [(1, a, b)], np.array([1.0]))
        assert abs(pi[0] - rhs) < 1e-14


# ---------------------------------------------------------------------------
# double polynomial (section 6)
# ---------------------------------------------------------------------------

def test_double_polynomial_diagonal_closed_form():
    # on a diagonal matrix phi2(phi1(A)) v and p(A) v = p1(A) p2(phi1(A)) v act
    # per eigenvalue: phi(l) = 1 - prod(1 - phi1(l)/t2) with
    # phi1(l) = 1 - prod(1 - l/t1), and p(l) = phi(l) / l; evaluated in mpmath
    import mpmath as mp

    from oracle.chains import apply_p_double, apply_phi_double, apply_pi_double

    mp.mp.dps = 40
    lam = np.linspace(1.0, 10.0, 40)
    A = diagonal(lam).to_scipy()
    inner = [(chains.REAL, 9.0, 0.0), (chains.PAIR, 5.0, 2.0), (chains.REAL, 1.5, 0.0)]
    outer = [(chains.REAL, 0.9, 0.0), (chains.PAIR, 0.6, 0.3), (chains.REAL, 0.2, 0.0)]

    def pi_of(units, z):
        out = mp.mpf(1)
        for k, a, b in units:
            if k == chains.REAL:
                out *= 1 - z / a
            else:
                out *= (1 - z / mp.mpc(a, b)) * (1 - z / mp.mpc(a, -b))
        return out

    v = np.ones(lam.size)
    phi_ref, p_ref = [], []
    for l in lam:
        mu = 1 - pi_of(inner, mp.mpf(l))
        ph = 1 - pi_of(outer, mu)
        phi_ref.append(float(mp.re(ph)))
        p_ref.append(float(mp.re(ph / l)))
    phi_ref, p_ref = np.array(phi_ref), np.array(p_ref)
    assert np.max(np.abs(apply_phi_double(A, inner, outer, v) - phi_ref)) <= 1e-13 * np.max(np.abs(phi_ref))
    assert np.max(np.abs(apply_pi_double(A, inner, outer, v) - (1 - phi_ref))) <= 1e-13
    assert np.max(np.abs(apply_p_double(A, inner, outer, v) - p_ref)) <= 1e-13 * np.max(np.abs(p_ref))


def test_double_setup_outer_roots_are_eigenvalues_of_phi1():
    # with d2 = n the Krylov space of phi1(A) is complete: the outer roots are
    # the eigenvalues phi1(l_i) of phi1(A) (closed form on a diagonal matrix)
    lam = np.array([1.0, 1.7, 2.2, 3.1, 4.0, 4.6, 5.5, 6.3, 7.0, 8.2, 9.1, 10.0])
    A = diagonal(lam).to_scipy()
    v0 = start_vector(lam.size, 2)
    P1 = roots.setup(A, v0, 4, orth="cgs2")
    P2 = roots.setup_double(A, P1.units, v0, lam.size, add_roots=False, orth="cgs2")
    pi1 = np.ones(lam.size, dtype=complex)
    for z in P1.roots():
        pi1 *= 1 - lam / z
    want = np.sort((1 - pi1).real)
    got = np.sort(P2.theta.real)
    assert P2.breakdown and np.max(np.abs(P2.theta.imag)) <= 1e-10
    assert np.max(np.abs(got - want)) <= 1e-8 * np.max(np.abs(want))
