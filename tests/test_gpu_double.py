"""GPU parity of the double polynomial phi2(phi1(A)) (section 6)."""

import os

import numpy as np
import pytest
import torch

from oracle import chains as ochains, roots as oroots, solver as osolver
from workloads import biharmonic2d, convdiff2d, rhs, start_vector
from gpu_util import say, dev, host, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import paper_1911_07065_amd.api as api

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return api


def _units(roots):
    """(kind, re, im) units of a root list with conjugate pairs adjacent (a+bi, a-bi)."""
    out, i = [], 0
    while i < len(roots):
        z = roots[i]
        if z.imag != 0.0:
            out.append((ochains.PAIR, z.real, abs(z.imag)))
            i += 2
        else:
            out.append((ochains.REAL, z.real, 0.0))
            i += 1
    return out


def _multiset_relerr(a, b):
    a = list(np.asarray(a, dtype=complex))
    b = list(np.asarray(b, dtype=complex))
    worst = 0.0
    for z in a:
        j = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b[j]) / abs(z))
        b.pop(j)
    return worst


@pytest.fixture(scope="module")
def cfg1(pp):
    csr = convdiff2d(50, 1.0)
    M = pp.Matrix.from_csr(csr)
    v0 = start_vector(csr.n, 2)
    p1 = pp.setup(M, dev(v0), 6)
    p2 = pp.setup_double(M, p1, dev(v0), 5)
    return csr, M, v0, p1, p2


def test_setup_double_matches_oracle(pp, cfg1):
    csr, M, v0, p1, p2 = cfg1
    say("setup double")
    inner = _units(p2.roots("inner"))
    assert np.array_equal(p2.roots("inner"), p1.roots("final"))
    P2 = oroots.setup_double(csr.to_scipy(), inner, v0, 5, orth="cgs2")
    theta = p2.roots("theta")
    assert _multiset_relerr(theta, P2.theta) < 1e-8
    leja, pof, n_add, units = oroots.order_and_add(theta)
    assert np.array_equal(p2.roots("final"), oroots.Poly(5, theta, leja, pof, n_add, units).roots())
    assert p2.composite_degree == p1.d_eff * p2.d_eff
    assert p2.setup_info["mvps"] == 5 * p1.d_eff


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_composite_apply_matches_oracle(pp, cfg1, prec):
    csr, M, v0, p1, p2 = cfg1
    A = csr.to_scipy()
    inner, outer = _units(p2.roots("inner")), _units(p2.roots("final"))
    v = rhs(csr.n, 5)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tol = 1e-12 if prec == "fp64" else 1e-4
    say("composite apply", prec)
    for kind, ref in (("phi", ochains.apply_phi_double), ("pi", ochains.apply_pi_double),
                      ("p", ochains.apply_p_double)):
        y = host(pp.apply(p2, M, dev(v).to(dt), kind)).astype(np.float64)
        assert relerr(y, ref(A, inner, outer, v)) <= tol, kind
    # A p(A) = phi2(phi1(A)) through the library's own products
    yp = host(pp.apply(p2, M, dev(v), "p"))
    assert relerr(A @ yp, host(pp.apply(p2, M, dev(v), "phi"))) <= 1e-10


@pytest.mark.parametrize("inner_prec", ["fp64", "fp32"])
def test_double_solve_matches_oracle(pp, cfg1, inner_prec):
    csr, M, v0, p1, p2 = cfg1
    A = csr.to_scipy()
    b = rhs(csr.n, 1)
    say("double solve", inner_prec)
    x, info = pp.solve(p2, M, dev(b), tol=1e-10, m=50, inner=inner_prec)
    xh = host(x)
    assert info["converged"] and np.linalg.norm(b - A @ xh) <= 1e-10 * np.linalg.norm(b)
    inner, outer = _units(p2.roots("inner")), _units(p2.roots("final"))
    xo, io = osolver.pp_gmres(A, b, outer, m=50, tol=1e-10, orth="cgs2", inner_units=inner)
    say("result double", inner_prec, "relres", np.linalg.norm(b - A @ xh) / np.linalg.norm(b), "x_err_vs_oracle",
        relerr(xh, xo))
    assert relerr(xh, xo) <= 1e-6
    if inner_prec == "fp64":
        assert abs(info["mvps"] - io.mvps) <= 0.05 * io.mvps


def test_double_rejected_by_batch_and_bad_args(pp, cfg1):
    csr, M, v0, p1, p2 = cfg1
    with pytest.raises(Exception):
        pp.setup_double(M, p1, dev(v0), 0)
    with pytest.raises(Exception):
        p1.roots("inner")  # not a composite
    Bt = pp.Batch([csr])
    with pytest.raises(Exception):
        Bt.solve([p2], Bt.interleave(rhs(csr.n, 1)), 1)


def test_example13_table6_1(pp, golden_dir):
    # Example 13: the biharmonic matrix of Example 3 (n = 40000), GMRES(50).
    # The paper stops on the shortcut residual 1e-10 (its true residuals
    # reach 1.4e-10 or better); here the true residual must reach 2e-10.
    # Loose comparison with Tables 3.4 and 6.1 (other random vectors, CGS2),
    # and the section's claim: the composite polynomial needs more than 10x
    # fewer inner products than the best single polynomial.
    single = {int(r[0]): r for r in np.loadtxt(os.path.join(golden_dir, "example3_biharmonic.txt"),
                                               comments="#", ndmin=2)}
    double = {int(r[0]): r for r in np.loadtxt(os.path.join(golden_dir, "table6_1_double.txt"),
                                               comments="#", ndmin=2)}
    csr = biharmonic2d(200)
    A = csr.to_scipy()
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    M = pp.Matrix.from_csr(csr)
    bd, v0d = dev(b), dev(v0)
    dots = {}
    for d in (20, 40):
        say("example 13 double", d)
        p1 = pp.setup(M, v0d, d)
        p2 = pp.setup_double(M, p1, v0d, d)
        x, info = pp.solve(p2, M, bd, tol=2e-10, m=50, inner="fp64")
        assert info["converged"] and np.linalg.norm(b - A @ host(x)) <= 2e-10 * np.linalg.norm(b)
        mv = info["mvps"] + p1.setup_info["mvps"] + p2.setup_info["mvps"]
        dots[("double", d)] = info["dots"] + p1.setup_info["dots"] + p2.setup_info["dots"]
        row = double[d]
        say("double", d, "cycles", info["cycles"], "(paper", row[2], ") mvps", mv, "(paper", row[3] * 1000, ")")
        assert 0.5 * row[2] <= info["cycles"] <= 1.5 * row[2] + 1
        assert 0.5 * row[3] * 1000 <= mv <= 1.5 * row[3] * 1000
    for d in (100, 200):
        say("example 13 single", d)
        p = pp.setup(M, v0d, d)
        x, info = pp.solve(p, M, bd, tol=2e-10, m=50, inner="fp64")
        assert info["converged"]
        mv = info["mvps"] + p.setup_info["mvps"]
        dots[("single", d)] = info["dots"] + p.setup_info["dots"]
        row = single[d]
        say("single", d, "cycles", info["cycles"], "(paper", row[2], ") mvps", mv, "(paper", row[3] * 1000, ")")
        assert 0.7 * row[2] <= info["cycles"] <= 1.3 * row[2]
        assert 0.7 * row[3] * 1000 <= mv <= 1.3 * row[3] * 1000
    assert 10 * dots[("double", 40)] < min(dots[("single", 100)], dots[("single", 200)])
