"""GPU parity of the polynomial setup (Algorithm 4 step 1) and PP-GMRES (step 2)."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla
import torch

from oracle import roots as oroots, solver as osolver
from workloads import convdiff2d, convdiff2d_blockmixed, convdiff3d, diag_example7, diagonal, randsparse, rhs, start_vector
from gpu_util import say, dev, host, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import paper_1911_07065_amd.api as api

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return api


def _multiset_relerr(a, b):
    a = list(np.asarray(a, dtype=complex))
    b = list(np.asarray(b, dtype=complex))
    worst = 0.0
    for z in a:
        j = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b[j]) / abs(z))
        b.pop(j)
    return worst


@pytest.mark.parametrize("N,alpha,d", [(50, 1.0, 10), (40, 30.0, 20), (30, 0.0, 25)])
def test_setup_matches_oracle(pp, N, alpha, d):
    csr = convdiff2d(N, alpha)
    A = csr.to_scipy()
    v0 = start_vector(csr.n, 2)
    say("setup", N, alpha, d)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(v0), d)
    P = oroots.setup(A, v0, d, orth="cgs2")
    theta = poly.roots("theta")
    # harmonic Ritz values: same multiset up to the rounding of two Arnoldi runs
    assert _multiset_relerr(theta, P.theta) < 1e-8
    # ordering and added roots of the library's own theta: bit-exact with the oracle's rules
    leja, pof, n_add, units = oroots.order_and_add(theta)
    assert np.array_equal(poly.roots("leja"), leja)
    assert np.array_equal(poly.roots("final"), oroots.Poly(d, theta, leja, pof, n_add, units).roots())
    assert poly.d == P.d and poly.n_added == P.n_added


@pytest.mark.parametrize("N,alpha,d", [(50, 1.0, 10), (40, 30.0, 20)])
def test_fp32_basis_setup(pp, N, alpha, d):
    # the same GMRES(d) cycle with binary32 Krylov vectors (FP64 dots and
    # Hessenberg): harmonic Ritz values within the rounding of the stored
    # vectors of the oracle's FP64 ones, the Leja order and added roots of
    # the library's own theta bit-exact with the oracle's rules, and a solve
    # with that polynomial reaching the tolerance
    csr = convdiff2d(N, alpha)
    A = csr.to_scipy()
    v0 = start_vector(csr.n, 2)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(v0), d, basis="fp32")
    P = oroots.setup(A, v0, d, orth="cgs2")
    theta = poly.roots("theta")
    err = _multiset_relerr(theta, P.theta)
    say("setup fp32 basis", N, alpha, d, f"theta vs oracle {err:.2e}")
    assert err < 1e-5  # measured 4.5e-8 and 2.3e-7 on these two cases
    leja, pof, n_add, units = oroots.order_and_add(theta)
    assert np.array_equal(poly.roots("leja"), leja)
    assert np.array_equal(poly.roots("final"), oroots.Poly(d, theta, leja, pof, n_add, units).roots())
    b = rhs(csr.n, 1)
    x, info = pp.solve(poly, M, dev(b), tol=1e-8, m=50, inner="fp32")
    rel = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
    assert info["status"] == 0 and rel <= 1e-8, (info, rel)
    with pytest.raises(Exception):
        pp.setup(M, dev(v0), d, basis="bf16")
    # the C ABI refuses any other basis precision itself
    import ctypes

    from paper_1911_07065_amd._lib import lib, SetupInfo
    h, si, vd = ctypes.c_void_p(), SetupInfo(), dev(v0)
    st = lib.pp_gmres_setup_basis(M.handle, vd.data_ptr(), d, 1, 2, None, ctypes.byref(h), ctypes.byref(si))
    assert st == -1 and not h.value  # PP_EINVAL, no polynomial


def test_fp32_basis_setup_full_size(pp):
    # the 128^3 benchmark workload, d = 40: the FP32-basis polynomial solves
    # to 1e-8 in about as many iterations as the FP64-basis one
    csr = convdiff3d(128, 10, 10, 10)
    A = csr.to_scipy()
    v0 = dev(start_vector(csr.n, 2))
    b = rhs(csr.n, 1)
    M = pp.Matrix.from_csr(csr)
    its = {}
    for basis in ("fp64", "fp32"):
        poly = pp.setup(M, v0, 40, basis=basis)
        x, info = pp.solve(poly, M, dev(b), tol=1e-8, m=50, inner="fp32")
        rel = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
        say("full size setup basis", basis, "iters", info["iters"], "relres", rel, "d_eff", poly.d_eff)
        assert info["status"] == 0 and rel <= 1e-8, (basis, info, rel)
        its[basis] = info["iters"]
    assert its["fp32"] <= its["fp64"] + 3


def test_setup_example7_adds_two_roots(pp):
    csr = diag_example7()
    say("setup example 7")
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(start_vector(csr.n, 2)), 125)
    assert poly.n_added == 2
    fin = poly.roots()
    lej = poly.roots("leja")
    extra = [z for z in set(fin.real) if np.sum(fin.real == z) > np.sum(lej.real == z)]
    assert sorted(round(z) for z in extra) == [30, 60]


def test_setup_breakdown(pp):
    csr = diagonal(np.repeat([1.0, 2.0, 5.0], 100))
    say("setup breakdown")
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(start_vector(csr.n, 3)), 10)
    assert poly.breakdown and poly.d == 3
    assert np.allclose(np.sort(poly.roots().real), [1, 2, 5], rtol=1e-10)


@pytest.mark.parametrize("case", ["clusters_no_added_roots", "wide_added_roots", "clusters_all_unstable"])
def test_setup_checked_matches_oracle(pp, case):
    # stability check in the setup (section 3.5) with the degree lowered by
    # 15: the degree kept, the unstable flag and the roots follow the oracle.
    # On these diagonal matrices StCh swings over many orders of magnitude
    # when the roots move by an ulp at some degrees (a root equal to an
    # eigenvalue to the last bit removes that eigencomponent exactly); the
    # degrees tried here (40, 25, 10 and 35, 20) are ones where every root
    # set within 2 ulp of the oracle's gives StCh at least 100 times from
    # the threshold on the same side, so the decisions cannot flip
    from workloads import diag_clusters, diag_wide

    csr = diag_wide() if case.startswith("wide") else diag_clusters()
    add = case == "wide_added_roots"
    d0 = 35 if add else 40
    tol = 0.0 if case.endswith("all_unstable") else 1e-8
    A = csr.to_scipy()
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    say("setup checked", case)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup_checked(M, dev(v0), d0, dev(b), tol=tol, d_step=15, d_min=10, add_roots=add)
    P, st, unstable, tried = osolver.setup_checked(A, v0, d0, b, tol, d_step=15, d_min=10, add_roots=add,
                                                   orth="cgs2")
    assert len(tried) >= 2
    assert poly.d == P.d and poly.unstable == unstable
    theta = poly.roots("theta")
    assert _multiset_relerr(theta, P.theta) < 1e-8
    leja, pof, n_add, units = oroots.order_and_add(theta, add)
    assert np.array_equal(poly.roots("final"), oroots.Poly(poly.d, theta, leja, pof, n_add, units).roots())
    # StCh of the kept polynomial: rounding-level on both sides
    st_or = osolver.stability_check(A, units, b)
    assert poly.stch <= 1e-12 and st_or <= 1e-12
    assert poly.setup_info["mvps"] == d0 + sum(2 * (oroots.setup(A, v0, k, add_roots=add, orth="cgs2").d_eff)
                                               for k, _ in tried)


@pytest.mark.parametrize("case", ["clusters", "wide_added_roots"])
def test_setup_checked_decisions_at_every_degree(pp, case):
    # degrees 40, 30, 20, 10 (section 3.5: lower the degree while the check
    # predicts instability). On these spectra StCh is ill-conditioned in the
    # roots: at degree 20 of the clustered case the oracle's roots give 64
    # and roots equal to them within 1e-8 give 3e-16 (a root that matches an
    # eigenvalue to the last bits removes that eigencomponent). So StCh is
    # compared on identical roots: (1) the library's decision follows the
    # sign of its own StCh against tol ||b||; (2) at every degree the oracle
    # tried, the library's StCh of a degree-k polynomial and the oracle's
    # StCh of the same roots are on the same side of the threshold wherever
    # the oracle's value sits at least 100x from it (an unstable value is
    # amplified rounding, so its size depends on the summation order).
    from workloads import diag_clusters, diag_wide

    csr = diag_wide() if case.startswith("wide") else diag_clusters()
    add = case == "wide_added_roots"
    tol = 1e-8
    A = csr.to_scipy()
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    limit = tol * np.linalg.norm(b)
    say("setup checked every degree", case)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup_checked(M, dev(v0), 40, dev(b), tol=tol, d_step=10, d_min=10, add_roots=add)
    P, st, unstable, tried = osolver.setup_checked(A, v0, 40, b, tol, d_step=10, d_min=10, add_roots=add,
                                                   orth="cgs2")
    assert (poly.stch > limit) == poly.unstable, (poly.stch, limit, poly.unstable)
    assert any(k == 20 for k, _ in tried)  # degree 20 is decided in both cases
    for k, st_own in tried:
        single = pp.setup_checked(M, dev(v0), k, dev(b), tol=tol, d_step=0, add_roots=add)
        st_same = osolver.stability_check(A, single.units(), b)
        say(f"degree {k}: StCh library {single.stch:.3e}, oracle on the library's roots {st_same:.3e}, "
            f"oracle on its own roots {st_own:.3e}, threshold {limit:.1e}")
        if st_same >= 100 * limit or st_same <= limit / 100:
            assert (single.stch <= limit) == (st_same <= limit), (k, single.stch, st_same)


def test_setup_checked_errors(pp):
    csr = convdiff2d(8)
    M = pp.Matrix.from_csr(csr)
    v0, b = dev(start_vector(csr.n, 2)), dev(rhs(csr.n, 1))
    with pytest.raises(Exception):
        pp.setup_checked(M, v0, 4, b, tol=-1.0)
    with pytest.raises(Exception):
        pp.setup_checked(M, v0, 4, b, d_step=-1)
    poly = pp.setup_checked(M, v0, 4, b, tol=1.0)  # stable at once: no lowering
    assert poly.d == 4 and not poly.unstable and poly.stch <= 1.0


def test_setup_errors(pp):
    csr = convdiff2d(8)
    M = pp.Matrix.from_csr(csr)
    with pytest.raises(Exception):
        pp.setup(M, dev(np.zeros(csr.n)), 4)  # zero start vector
    with pytest.raises(Exception):
        pp.setup(M, dev(np.ones(csr.n)), csr.n + 1)  # degree above n


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
def test_cfg1_solve_matches_oracle(pp, inner):
    csr = convdiff2d(50, 1.0)
    A = csr.to_scipy()
    b = rhs(csr.n, 1)
    v0 = start_vector(csr.n, 2)
    say("cfg1 solve", inner)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(v0), 10)
    x, info = pp.solve(poly, M, dev(b), tol=1e-8, m=50, inner=inner)
    xh = host(x)
    rel = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
    assert info["status"] == 0 and rel <= 1e-8, (info, rel)
    assert abs(rel - info["relres"]) <= 1e-12
    P = oroots.setup(A, v0, 10)
    xo, io = osolver.pp_gmres(A, b, P.units, m=50, tol=1e-8)
    # both solutions are within cond(A) * 1e-8 of the exact one
    say("result cfg1", inner, "relres", rel, "x_err_vs_oracle", relerr(xh, xo))
    assert relerr(xh, xo) < 2e-5
    if inner == "fp64":
        assert abs(info["iters"] - io.iters) <= 1


@pytest.mark.parametrize("basis", ["fp64", "fp32"])
def test_setup_repeats_bit_for_bit(pp, basis):
    # the setup's dot passes reduce in a fixed order (wave sums, workgroup
    # partials, one device pass): the same input gives the same harmonic
    # Ritz values and roots bit for bit
    csr = convdiff3d(24, 10, 10, 10)
    M = pp.Matrix.from_csr(csr)
    v0 = dev(start_vector(csr.n, 2))
    say("setup repeatability", basis)
    p0 = pp.setup(M, v0, 16, basis=basis)
    p1 = pp.setup(M, v0, 16, basis=basis)
    for kind in ("theta", "leja", "final"):
        assert np.array_equal(p0.roots(kind), p1.roots(kind)), kind


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
def test_lookahead_keeps_the_iterates(pp, inner):
    # queueing the next step's phi(A) before the host reads the Hessenberg
    # column changes when work is queued, not what is computed: the same x bit
    # for bit, the same counters; the cycles run to their own stopping points
    csr = convdiff3d(24, 10, 10, 10)
    b = rhs(csr.n, 1)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(start_vector(csr.n, 2)), 12)
    say("lookahead", inner)
    runs = {}
    for la in (False, True):
        x, info = pp.solve(poly, M, dev(b), tol=1e-10, m=20, inner=inner, lookahead=la)
        runs[la] = (host(x), info)
    (x0, i0), (x1, i1) = runs[False], runs[True]
    assert i0["status"] == 0 and i1["status"] == 0
    assert np.array_equal(x0, x1)
    for k in ("cycles", "iters", "mvps", "dots", "vops", "fp64_cycles"):
        assert i0[k] == i1[k], k
    assert i0["lookahead_discarded"] == 0 and 0 <= i1["lookahead_discarded"] <= i1["cycles"]
    rel = np.linalg.norm(b - csr.to_scipy() @ x1) / np.linalg.norm(b)
    assert rel <= 1e-10


def test_solve_workspace_bytes_bounds_the_allocation(pp):
    # the query's `additional` covers what a solve allocates on the handle
    # (device memory seen by the driver), and is 0 once the handle holds it
    csr = convdiff3d(64, 10, 10, 10)
    b = rhs(csr.n, 1)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(start_vector(csr.n, 2)), 10)
    M.tune("fp32")
    say("workspace bytes")
    for inner, m in (("fp32", 40), ("fp64", 30)):
        total, add = pp.solve_workspace_bytes(poly, M, m=m, inner=inner)
        ldv = -(-csr.n // 64) * 64
        basis = ldv * (4 if inner == "fp32" else 8) * (m + 1 + 5)
        assert total >= basis and 0 <= add <= total
        bd = dev(b)
        x = torch.empty_like(bd)  # the caller's buffers, allocated before the measurement
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        pp.solve(poly, M, bd, tol=1e-8, m=m, inner=inner, x=x)
        torch.cuda.synchronize()
        grew = free0 - torch.cuda.mem_get_info()[0]
        assert grew <= add + (8 << 20), (inner, grew, add)
        assert pp.solve_workspace_bytes(poly, M, m=m, inner=inner)[1] == 0
    with pytest.raises(Exception):
        pp.solve_workspace_bytes(None, M, m=30)  # no polynomial and no ChPoly


def test_stability_check_matches_oracle(pp):
    csr = convdiff2d(50, 1.0)
    A = csr.to_scipy()
    b = rhs(csr.n, 1)
    M = pp.Matrix.from_csr(csr)
    P = oroots.setup(A, start_vector(csr.n, 2), 10)
    poly = pp.poly_from_roots(P.roots(), keep_order=True)
    say("stability check")
    s = pp.stability_check(poly, M, dev(b))
    so = osolver.stability_check(A, P.units, b)
    assert s < 1e-12 and so < 1e-12


def test_noconv_and_zero_rhs(pp):
    csr = convdiff2d(30, 1.0)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(start_vector(csr.n, 2)), 3)
    b = rhs(csr.n, 1)
    say("noconv")
    x, info = pp.solve(poly, M, dev(b), tol=1e-14, m=3, max_cycles=2, inner="fp64")
    assert info["status"] == 1 and info["cycles"] == 2
    A = csr.to_scipy()
    assert abs(np.linalg.norm(b - A @ host(x)) - info["relres"]) < 1e-10
    x, info = pp.solve(poly, M, dev(np.zeros(csr.n)), tol=1e-8)
    assert info["status"] == 0 and float(torch.abs(x).max()) == 0.0


@pytest.fixture(scope="module")
def cfg2_oracle():
    # the FP64 oracle's solution of the 128^3 workload (about 25 s on the host)
    csr = convdiff3d(128, 10, 10, 10)
    A = csr.to_scipy()
    b = rhs(csr.n, 1)
    say("cfg2 oracle solve (host)")
    P = oroots.setup(A, start_vector(csr.n, 2), 40)
    xo, io = osolver.pp_gmres(A, b, P.units, m=50, tol=1e-8)
    return csr, A, b, xo


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_cfg2_full_size_solve(pp, inner, cfg2_oracle):
    # 3-D convection-diffusion 128^3, degree 40 with added roots, GMRES(50), 1e-8
    csr, A, b, xo = cfg2_oracle
    say("cfg2 solve", inner)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(start_vector(csr.n, 2)), 40)
    x, info = pp.solve(poly, M, dev(b), tol=1e-8, m=50, inner=inner)
    xh = host(x)
    rel = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
    say("cfg2 solve done", inner, info)
    # ||A^-1||_2 <= 1 / lambda_min of the symmetric part (the 7-point
    # Laplacian with diagonal 6: 3 (2 - 2 cos(pi h)), h = 1/129)
    inv2 = 1.0 / (3.0 * (2.0 - 2.0 * np.cos(np.pi / 129.0)))
    bound = inv2 * (np.linalg.norm(b - A @ xh) + np.linalg.norm(b - A @ xo)) / np.linalg.norm(xo)
    say("result cfg2", inner, "relres", rel, "x_err_vs_oracle", relerr(xh, xo), "bound", bound)
    assert info["status"] == 0 and rel <= 1e-8
    assert relerr(xh, xo) <= min(bound * (1 + 1e-9), 1e-5)


def _varah_inv_bound(A):
    """Bound on ||A^-1||_inf for a matrix strictly diagonally dominant by rows
    (Varah 1975): 1 / min_i (|a_ii| - sum_{j != i} |a_ij|)."""
    d = np.abs(A.diagonal())
    off = np.asarray(abs(A).sum(axis=1)).ravel() - d
    assert np.all(d > off)
    return 1.0 / float(np.min(d - off))


def _randsparse_vs_oracle(pp, n, inners, xo_cache, basis="fp64"):
    # random sparse, 16 random columns + diagonal, dominance 1.05, degree 100
    # with added roots, GMRES(30), tol 1e-8: x of each inner precision against
    # the FP64 oracle's x (its own polynomial from the same start vector).
    # ||x - x_or||_inf <= ||A^-1||_inf (||r||_inf + ||r_or||_inf), with the
    # Varah bound for ||A^-1||_inf.
    csr = randsparse(n, 16, seed=7)
    A = csr.to_scipy()
    b = rhs(csr.n, 1)
    v0 = start_vector(csr.n, 2)
    if n not in xo_cache:
        say("random sparse oracle solve (host)", n)
        P = oroots.setup(A, v0, 100, orth="cgs2")
        xo, io = osolver.pp_gmres(A, b, P.units, m=30, tol=1e-8, orth="cgs2")
        assert io.status == osolver.OK
        xo_cache[n] = xo
    xo = xo_cache[n]
    inv_inf = _varah_inv_bound(A)
    M = pp.Matrix.from_csr(csr)
    poly = pp.setup(M, dev(v0), 100, basis=basis)
    for inner in inners:
        say("random sparse solve", n, inner, "setup basis", basis)
        x, info = pp.solve(poly, M, dev(b), tol=1e-8, m=30, inner=inner)
        xh = host(x)
        r = b - A @ xh
        rel = np.linalg.norm(r) / np.linalg.norm(b)
        err2 = relerr(xh, xo)
        err_inf = float(np.max(np.abs(xh - xo)) / np.max(np.abs(xo)))
        bound_inf = inv_inf * (np.max(np.abs(r)) + np.max(np.abs(b - A @ xo))) / np.max(np.abs(xo))
        say(f"result random sparse n={n} {inner}: relres {rel:.2e}, ||x - x_oracle||/||x_oracle|| {err2:.2e}, "
            f"max-norm {err_inf:.2e} (bound {bound_inf:.2e}), cycles {info['cycles']}")
        assert info["status"] == 0 and rel <= 1e-8
        assert err_inf <= bound_inf * (1 + 1e-9) + 1e-15


@pytest.fixture(scope="module")
def randsparse_oracle_x():
    return {}


def test_cfg3_shaped_solve_matches_oracle(pp, randsparse_oracle_x):
    # the random sparse workload's shape at n = 1e5
    _randsparse_vs_oracle(pp, 100_000, ("fp64", "fp32", "bf16"), randsparse_oracle_x)


def test_cfg3_shaped_fp32_basis_solve(pp, randsparse_oracle_x):
    # the same with the polynomial from an FP32-basis setup (degree 100): the
    # FP32 and BF16 forms still land within the bound of the oracle's x
    _randsparse_vs_oracle(pp, 100_000, ("fp32", "bf16"), randsparse_oracle_x, basis="fp32")


def test_cfg3_full_size_solve(pp, randsparse_oracle_x):
    # random sparse n = 1e6, 17 entries per row, degree 100 with added roots,
    # GMRES(30) against the oracle's x (about 35 s on the host)
    _randsparse_vs_oracle(pp, 1_000_000, ("fp64", "fp32", "bf16"), randsparse_oracle_x)


# ---------------------------------------------------------------------------
# composition with a diagonal right preconditioner (eqs. 1.3-1.4)
# ---------------------------------------------------------------------------

def test_jacobi_operator_and_scale(pp):
    from workloads import convdiff2d_colscaled

    csr = convdiff2d_colscaled(40, 5.0, 3.0)
    A = csr.to_scipy()
    say("jacobi operator")
    M = pp.Matrix.from_csr(csr)
    M.right_scale()
    AS, s = osolver.right_scaled(A)
    assert np.array_equal(host(M.scale()), s)  # 1/a_ii, one rounding on both sides
    v = rhs(csr.n, 7)
    ident = pp.poly_from_roots([1.0])  # phi(z) = z: one product with the operator
    y = host(pp.apply(ident, M, dev(v), "phi"))
    assert relerr(y, AS @ v) <= 1e-14
    # new values: the scaling follows their diagonal
    M.set_values(dev(2.0 * csr.val))
    assert np.array_equal(host(M.scale()), 1.0 / (2.0 * A.diagonal()))


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_jacobi_composed_solve_matches_oracle(pp, inner):
    from workloads import convdiff2d_colscaled

    csr = convdiff2d_colscaled(50, 1.0, 3.0)
    A = csr.to_scipy()
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    say("jacobi solve", inner)
    M = pp.Matrix.from_csr(csr)
    M.right_scale()
    poly = pp.setup(M, dev(v0), 10)
    AS, s = osolver.right_scaled(A)
    P = oroots.setup(AS, v0, 10, orth="cgs2")
    theta = poly.roots("theta")
    assert _multiset_relerr(theta, P.theta) < 1e-8
    x, info = pp.solve(poly, M, dev(b), tol=1e-8, m=50, inner=inner)
    xh = host(x)
    assert info["converged"] and info["cycles"] <= 3
    assert np.linalg.norm(b - A @ xh) <= 1e-8 * np.linalg.norm(b)
    xt, _ = osolver.pp_gmres(AS, b, P.units, m=50, tol=1e-8)
    say("result jacobi", inner, "relres", np.linalg.norm(b - A @ xh) / np.linalg.norm(b), "x_err_vs_oracle",
        relerr(xh, s * xt))
    assert relerr(xh, s * xt) <= 2e-5
    # without the composition the same polynomial degree does not converge
    M0 = pp.Matrix.from_csr(csr)
    x0, info0 = pp.solve(pp.setup(M0, dev(v0), 10), M0, dev(b), tol=1e-8, m=50, max_cycles=30, inner=inner)
    assert not info0["converged"]


def test_custom_right_scaling_and_errors(pp):
    csr = convdiff2d(20, 10.0)
    A = csr.to_scipy()
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    s = 10.0 ** np.random.default_rng(4).uniform(-1, 1, csr.n)
    say("custom right scaling")
    M = pp.Matrix.from_csr(csr)
    M.right_scale(dev(s))
    assert np.array_equal(host(M.scale()), s)
    x, info = pp.solve(pp.setup(M, dev(v0), 8), M, dev(b), tol=1e-10, m=50, inner="fp64")
    assert info["converged"] and np.linalg.norm(b - A @ host(x)) <= 1e-10 * np.linalg.norm(b)
    # a zero diagonal: Jacobi fails and the handle stays unscaled
    vals = csr.val.copy()
    rows = np.repeat(np.arange(csr.n), np.diff(csr.rowptr))
    vals[np.flatnonzero(rows == csr.colind)[3]] = 0.0
    Mz = pp.Matrix.from_csr(csr.with_values(vals))
    with pytest.raises(Exception):
        Mz.right_scale()
    assert Mz.scaling is None
    with pytest.raises(Exception):
        Mz.scale()
    ident = pp.poly_from_roots([1.0])
    v = rhs(csr.n, 7)
    assert relerr(host(pp.apply(ident, Mz, dev(v), "phi")), csr.with_values(vals).to_scipy() @ v) <= 1e-14


def test_block_jacobi_operator_matches_oracle(pp):
    # B = A M^{-1} and M^{-1}'s blocks against the oracle (bs = 3 leaves a
    # one-row last block; bs = 40 takes whole grid lines). Two inversions of
    # a block D in double differ by about kappa(D) eps |D^{-1}|, so the
    # columns of block J of B may differ by c kappa(D_J) eps (|A| |M^{-1}|),
    # c = 4 bs; the mixed case has kappa up to 1e4.

    for csr, bs in ((convdiff2d(20, 5.0), 3), (convdiff2d_blockmixed(24, 5.0, 4, 2.0), 4), (convdiff2d(40, 40.0), 40)):
        A = csr.to_scipy()
        say("block jacobi operator", csr.n, bs)
        M = pp.Matrix.from_csr(csr)
        B = M.block_jacobi(bs)
        Bo, Mo = osolver.block_jacobi(A, bs)
        brp, bci = B.rowptr.cpu().numpy(), B.colind.cpu().numpy()
        Bg = sp.csr_matrix((host(B.val), bci, brp), shape=A.shape)
        nblk = (csr.n + bs - 1) // bs
        kap = np.array([np.linalg.cond(A[k * bs:(k + 1) * bs, k * bs:(k + 1) * bs].toarray()) for k in range(nblk)])
        bound = 4 * bs * np.finfo(float).eps * kap[np.arange(csr.n) // bs] * (abs(A) @ abs(Mo)).max(axis=0).toarray()
        assert np.all(np.abs((Bg - Bo).toarray()) <= bound)
        # every row of B holds whole blocks of columns
        for i in range(0, csr.n, max(1, csr.n // 37)):
            cols = bci[brp[i]:brp[i + 1]]
            assert np.array_equal(cols, np.unique(cols))
            for c in np.unique(cols // bs):
                assert np.sum(cols // bs == c) == min(bs, csr.n - c * bs)
        mi = host(B.minv).reshape(-1, bs, bs)
        for k in range(0, nblk, 7):
            m = min(bs, csr.n - k * bs)
            assert np.max(np.abs(mi[k, :m, :m] - Mo[k * bs:k * bs + m, k * bs:k * bs + m].toarray())) <= \
                4 * bs * np.finfo(float).eps * kap[k] * np.max(np.abs(mi[k, :m, :m]))
        v = rhs(csr.n, 7)
        ident = pp.poly_from_roots([1.0])
        # the handle's operator is the B it returned
        assert relerr(host(pp.apply(ident, B, dev(v), "phi")), Bg @ v) <= 1e-13


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_block_jacobi_composed_solve_matches_oracle(pp, inner):

    csr = convdiff2d_blockmixed(40, 5.0, 4, 2.0)
    A = csr.to_scipy()
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    say("block jacobi solve", inner)
    B = pp.Matrix.from_csr(csr).block_jacobi(4)
    poly = pp.setup(B, dev(v0), 10)
    Bo, Mo = osolver.block_jacobi(A, 4)
    P = oroots.setup(Bo, v0, 10, orth="cgs2")
    assert _multiset_relerr(poly.roots("theta"), P.theta) < 1e-8
    x, info = pp.solve(poly, B, dev(b), tol=1e-8, m=50, inner=inner)
    xh = host(x)
    assert info["converged"] and info["cycles"] <= 3
    assert np.linalg.norm(b - A @ xh) <= 1e-8 * np.linalg.norm(b)
    y, _ = osolver.pp_gmres(Bo, b, P.units, m=50, tol=1e-8)
    say("result block-jacobi", inner, "relres", np.linalg.norm(b - A @ xh) / np.linalg.norm(b), "x_err_vs_oracle",
        relerr(xh, Mo @ y))
    assert relerr(xh, Mo @ y) <= 2e-5
    # the same degree on the mixed matrix itself does not converge
    M0 = pp.Matrix.from_csr(csr)
    x0, info0 = pp.solve(pp.setup(M0, dev(v0), 10), M0, dev(b), tol=1e-8, m=50, max_cycles=30, inner=inner)
    assert not info0["converged"]


def test_block_jacobi_errors(pp):
    csr = convdiff2d(12, 3.0)
    M = pp.Matrix.from_csr(csr)
    for bs in (0, 65):
        with pytest.raises(Exception):
            M.block_jacobi(bs)
    # a singular diagonal block: rows 4 and 5 of the block [4, 6) made equal
    A = csr.to_scipy().tolil()
    A[5, 4], A[5, 5] = A[4, 4], A[4, 5]
    A = A.tocsr()
    A.sort_indices()
    Ms = pp.Matrix(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))
    with pytest.raises(Exception, match="singular"):
        Ms.block_jacobi(2)
    B = M.block_jacobi(4)
    with pytest.raises(Exception, match="block-Jacobi"):
        B.transpose()
    # a handle that is already right-preconditioned
    with pytest.raises(Exception, match="right preconditioner"):
        B.block_jacobi(4)
    Ms2 = pp.Matrix.from_csr(csr)
    Ms2.right_scale()
    with pytest.raises(Exception, match="right preconditioner"):
        Ms2.block_jacobi(2)


def test_jacobi_composed_gradient(pp):
    # the adjoint of a Jacobi-composed solve: the transposed handle gets the
    # same diagonal scaling; the gradient is that of A x = b
    from oracle.adjoint import grad_direct
    from workloads import convdiff2d_parts

    A0, dval = convdiff2d_parts(32)
    theta0 = 15.0
    n = A0.n
    b = rhs(n, 1)
    xt = np.random.default_rng(3).standard_normal(n)
    say("jacobi gradient")
    M = pp.Matrix.from_csr(A0)
    base, dirv = dev(A0.val), dev(dval)
    M.set_values(base + theta0 * dirv)
    M.right_scale()
    poly = pp.setup(M, dev(start_vector(n, 2)), 20)
    th = torch.tensor(theta0, dtype=torch.float64, device="cuda", requires_grad=True)
    x = pp.pp_solve_fn(base + th * dirv, dev(b), M, poly, tol=1e-12, m=50, inner="fp64")
    (0.5 * torch.sum((x - dev(xt)) ** 2)).backward()
    A = A0.with_values(A0.val + theta0 * dval).to_scipy()
    _, _, dv = grad_direct(A, b, lambda z: z - xt)
    g_or = float(dv @ dval)
    assert abs(float(th.grad) - g_or) <= 1e-6 * abs(g_or)


# ---------------------------------------------------------------------------
# polynomial changed at every cycle (section 5.2, ChPoly)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_chpoly_matches_oracle(pp, inner):
    csr = convdiff2d(50, 1.0)
    A = csr.to_scipy()
    b = rhs(csr.n, 1)
    say("chpoly cfg1", inner)
    M = pp.Matrix.from_csr(csr)
    x, info = pp.solve(None, M, dev(b), tol=1e-10, m=50, inner=inner, new_poly_degree=10)
    xo, io = osolver.pp_gmres(A, b, None, m=50, tol=1e-10, orth="cgs2", new_poly_degree=10)
    xh = host(x)
    say("result chpoly", inner, "relres", np.linalg.norm(b - A @ xh) / np.linalg.norm(b), "x_err_vs_oracle",
        relerr(xh, xo))
    assert info["converged"] and np.linalg.norm(b - A @ xh) <= 1e-10 * np.linalg.norm(b)
    assert relerr(xh, xo) <= 1e-6
    if inner == "fp64":  # the same path up to the rounding of two Arnoldi runs
        assert abs(info["cycles"] - io.cycles) <= 1 and abs(info["mvps"] - io.mvps) <= 0.05 * io.mvps


def test_chpoly_example12_table5_1(pp, golden_dir):
    # Example 12 at full size: diag(i^2/n), n = 10000, GMRES(50), tol 1e-10.
    # mvps against Table 5.1 (loose: other random vectors, CGS2 instead of
    # MGS), and the table's ordering at d = 10 and 25: ChPoly needs fewer
    # products than the fixed polynomial
    import os
    import time

    from workloads import diag_squares

    rows = {int(r[0]): (r[1] * 1000, r[2] * 1000) for r in
            np.loadtxt(os.path.join(golden_dir, "table5_1_chpoly.txt"), comments="#", ndmin=2)}
    n = 10000
    csr = diag_squares(n)
    A = csr.to_scipy()
    b, v0 = rhs(n, 1), start_vector(n, 2)
    M = pp.Matrix.from_csr(csr)
    for d in (10, 25):
        say("example 12 chpoly", d)
        t0 = time.perf_counter()
        x, ich = pp.solve(None, M, dev(b), tol=1e-10, m=50, max_cycles=20000, inner="fp64", stall_cycles=0,
                          new_poly_degree=d)
        t_ch = time.perf_counter() - t0
        assert ich["converged"] and np.linalg.norm(b - A @ host(x)) <= 1e-10 * np.linalg.norm(b)
        say("example 12 fixed", d)
        t0 = time.perf_counter()
        poly = pp.setup(M, dev(v0), d)
        x, ipp = pp.solve(poly, M, dev(b), tol=1e-10, m=50, max_cycles=20000, inner="fp64", stall_cycles=0)
        t_pp = time.perf_counter() - t0
        assert ipp["converged"]
        ppg, chp = rows[d]
        mv_pp = ipp["mvps"] + poly.d
        say("d", d, "ChPoly mvps", ich["mvps"], "(paper", chp, ") s", round(t_ch, 2), "| PP-G mvps", mv_pp,
            "(paper", ppg, ") s", round(t_pp, 2))
        assert 0.5 * chp <= ich["mvps"] <= 1.5 * chp
        assert 0.5 * ppg <= mv_pp <= 1.5 * ppg
        assert ich["mvps"] < mv_pp


def test_block_jacobi_full_size(pp):
    # the measured block-Jacobi workload (512^2, 4x4 block mixing): B against
    # the oracle's on sampled rows, and the composed solve's true residual
    csr = convdiff2d_blockmixed(512, 5.0, 4, 2.0)
    A = csr.to_scipy()
    say("block jacobi full size", csr.n)
    B = pp.Matrix.from_csr(csr).block_jacobi(4)
    Bo, Mo = osolver.block_jacobi(A, 4)
    brp, bci = B.rowptr.cpu().numpy(), B.colind.cpu().numpy()
    Bg = sp.csr_matrix((host(B.val), bci, brp), shape=A.shape)
    rows = np.random.default_rng(5).choice(csr.n, 2000, replace=False)
    C = A.tocoo()
    inb = C.row // 4 == C.col // 4
    blocks = np.zeros((csr.n // 4, 4, 4))
    blocks[C.row[inb] // 4, C.row[inb] % 4, C.col[inb] % 4] = C.data[inb]
    kap = np.linalg.cond(blocks)
    scale = (abs(A) @ abs(Mo)).max(axis=0).toarray().ravel()
    diff = abs(Bg[rows] - Bo[rows]).tocoo()
    assert np.all(diff.data <= 16 * np.finfo(float).eps * kap[diff.col // 4] * scale[diff.col])
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    x, info = pp.solve(pp.setup(B, dev(v0), 10), B, dev(b), tol=1e-8, m=50, inner="fp32")
    assert info["converged"]
    assert np.linalg.norm(b - A @ host(x)) <= 1e-8 * np.linalg.norm(b)
