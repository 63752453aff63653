"""Pins of the oracle's PP-GMRES solver (Algorithm 4) and its variants."""

import numpy as np
import pytest
import scipy.sparse.linalg as sla
import torch

from oracle import chains, roots, solver
from oracle.mixed import apply_p_low, apply_phi_low, round_bf16
from oracle.adjoint import grad_direct
from workloads import convdiff2d, convdiff2d_parts, diagonal, rhs, start_vector
from _golden import read_table


def _cfg1():
    A = convdiff2d(50, 1.0).to_scipy()
    return A, rhs(A.shape[0], 1), start_vector(A.shape[0], 2)


def test_cfg1_converges_to_tolerance_and_direct_solution():
    A, b, v0 = _cfg1()
    P = roots.setup(A, v0, 10)
    x, info = solver.pp_gmres(A, b, P.units, m=50, tol=1e-8)
    assert info.status == solver.OK
    rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert rel <= 1e-8
    xd = sla.spsolve(A.tocsc(), b)
    # forward error bounded by cond(A) * residual; cond(A) < 2e3 here
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 2e3 * 1e-8


def test_literal_form_agrees():
    A, b, v0 = _cfg1()
    P = roots.setup(A, v0, 10)
    x1, i1 = solver.pp_gmres(A, b, P.units, m=20, tol=1e-10)
    x2, i2 = solver.pp_gmres(A, b, P.units, m=20, tol=1e-10, literal=True)
    assert i1.relres <= 1e-10 and i2.relres <= 1.5e-10
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-8


@pytest.mark.parametrize("cycles", [1, 3])
def test_degree1_is_textbook_gmres(cycles):
    # PP(1)-GMRES(m): phi(A) = A/theta and p = 1/theta, so the iterates are
    # those of GMRES(m) on A; compared against scipy's own GMRES.
    A = convdiff2d(20, 3.0).to_scipy()
    b = rhs(A.shape[0], 1)
    P = roots.setup(A, start_vector(A.shape[0], 2), 1)
    x, info = solver.pp_gmres(A, b, P.units, m=10, tol=1e-30, max_cycles=cycles)
    xs, _ = sla.gmres(A, b, rtol=1e-30, atol=0.0, restart=10, maxiter=cycles)
    assert info.cycles == cycles
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-12


def _mgs_setup_vops(d):
    # vector operations of a GMRES(d) setup cycle with modified Gram-Schmidt,
    # counted here independently of the oracle: the start vector's norm and
    # scaling, then per step j = 1..d, j dots and j axpys, one norm and one
    # scaling
    return 2 + sum(2 * j + 2 for j in range(1, d + 1))


def test_example5_table3_6_loose():
    # PP(50)-GMRES(50): matrix-vector products within 30% of Table 3.6, and
    # vector operations (setup cycle + solve) within 10% of it
    for (al, be, ga, _, pp_mvps, _, pp_vops_k) in read_table("table3_6_convdiff.txt")[:2]:
        A = convdiff2d(200, al, be, ga).to_scipy()
        n = A.shape[0]
        P = roots.setup(A, start_vector(n, 2), 50)
        x, info = solver.pp_gmres(A, rhs(n, 1), P.units, m=50, tol=1e-8, setup_mvps=P.d)
        assert info.status == solver.OK
        assert 0.7 * pp_mvps <= info.mvps <= 1.3 * pp_mvps
        vops = info.vops + _mgs_setup_vops(P.d)
        assert abs(vops - 1000 * pp_vops_k) <= 0.10 * 1000 * pp_vops_k, (vops, pp_vops_k)


@pytest.mark.parametrize("row", range(5))
def test_counters_per_cycle_table4_1(row):
    # Table 4.1 (diag(i^2/n), n = 20000, GMRES(50), MGS) prints cycles, mvps,
    # vops and dots for runs of thousands of full cycles; per cycle they give
    # the cost of one GMRES(50) cycle of PP(d). Three full cycles of the
    # oracle (tolerance out of reach) must match: dots within 0.2% (they do
    # not depend on how the cycle restarts), mvps within 3% and vops within
    # 1.5% (the paper forms p(A) y once at the end and updates the residual
    # without a product; the oracle applies p and recomputes b - A x every
    # cycle: d more mvps and about 2d more vops per cycle)
    from workloads import diag_squares

    d, cycles, mvps_k, vops_k, dots_k = read_table("table4_1_counts.txt")[row]
    d = int(d)
    A = diag_squares(20000).to_scipy()
    P = roots.setup(A, start_vector(20000, 2), d, add_roots=False)
    assert P.d == d and P.d_eff == d
    x, info = solver.pp_gmres(A, rhs(20000, 1), P.units, m=50, tol=1e-30, max_cycles=3, stall_cycles=0)
    assert info.cycles == 3 and info.iters == 150
    # the residual norm at the top of every loop pass (4 passes for 3 cycles)
    per = {"dots": (info.dots - 1) / 3, "vops": (info.vops - 1) / 3, "mvps": info.mvps / 3}
    paper = {"dots": dots_k * 1e3 / cycles, "vops": vops_k * 1e3 / cycles, "mvps": mvps_k * 1e3 / cycles}
    for key, tol in (("dots", 0.002), ("mvps", 0.03), ("vops", 0.015)):
        assert abs(per[key] - paper[key]) <= tol * paper[key], (d, key, per[key], paper[key])


def test_richardson_theorem_3_1():
    # SPD A: adding a root theta_k >= lambda_max/2 does not increase ||pi(A) b||
    A = convdiff2d(25).to_scipy()
    n = A.shape[0]
    b = rhs(n, 1)
    P = roots.setup(A, start_vector(n, 2), 15, add_roots=False)
    lam_max = 8.0  # 4 + 4 cos(pi h) < 8
    pib = chains.apply_pi(A, P.units, b)
    checked = 0
    for (k, a, _) in P.units:
        if k == 0 and a >= lam_max / 2:
            ext = P.units + [(0, a, 0.0)]
            assert np.linalg.norm(chains.apply_pi(A, ext, b)) <= np.linalg.norm(pib) * (1 + 1e-12)
            checked += 1
    assert checked >= 3


def test_stability_check_small_for_stable_polynomial():
    A, b, v0 = _cfg1()
    P = roots.setup(A, v0, 10)
    assert solver.stability_check(A, P.units, b) < 1e-12


def test_noconv_after_max_cycles_returns_best_x():
    A, b, v0 = _cfg1()
    P = roots.setup(A, v0, 3)
    x, info = solver.pp_gmres(A, b, P.units, m=5, tol=1e-12, max_cycles=2)
    assert info.status == solver.NOCONV and info.cycles == 2
    assert np.isclose(np.linalg.norm(b - A @ x) / np.linalg.norm(b), info.relres, rtol=1e-12)


def test_breakdown_polynomial_solves_in_one_step():
    # 3 distinct eigenvalues: degree drops to 3, phi(A) = I, one iteration
    lam = np.repeat([1.0, 2.0, 5.0], 10)
    A = diagonal(lam).to_scipy()
    P = roots.setup(A, start_vector(30, 3), 10)
    b = rhs(30, 1)
    x, info = solver.pp_gmres(A, b, P.units, m=10, tol=1e-10)
    assert info.status == solver.OK and info.iters == 1
    assert np.allclose(x, b / lam, rtol=1e-9)


def test_mixed_emulation_bound():
    A, b, v0 = _cfg1()
    P = roots.setup(A, v0, 10)
    A32 = A.astype(np.float32)
    p64 = chains.apply_p(A, P.units, b)
    d32 = np.linalg.norm(apply_p_low(A32, P.units, b) - p64) / np.linalg.norm(p64)
    d16 = np.linalg.norm(apply_p_low(A32, P.units, b, "bf16") - p64) / np.linalg.norm(p64)
    f64 = chains.apply_phi(A, P.units, b)
    e32 = np.linalg.norm(apply_phi_low(A32, P.units, b) - f64) / np.linalg.norm(f64)
    assert 1e-9 < d32 < 1e-5 and 1e-9 < e32 < 1e-5
    assert d32 < d16 < 1e-1


def test_bf16_rounding_matches_torch():
    # torch's float32 -> bfloat16 conversion rounds to nearest even
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10.0
    x[:4] = [1.0 + 2**-8, 1.0 + 3 * 2**-8, -(1.0 + 2**-8), 0.0]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(round_bf16(x), ref)


def test_adjoint_gradient_vs_finite_differences():
    N = 12
    A0, dval = convdiff2d_parts(N)
    n = N * N
    b = rhs(n, 1)
    xt = np.random.default_rng(3).standard_normal(n)
    alpha = 20.0

    def loss(al):
        A = A0.with_values(A0.val + al * dval).to_scipy()
        x = sla.spsolve(A.tocsc(), b)
        return 0.5 * np.sum((x - xt) ** 2)

    A = A0.with_values(A0.val + alpha * dval).to_scipy()
    x, lam, dv = grad_direct(A, b, lambda x: x - xt)
    g = float(dv @ dval)
    h = 1e-6
    fd = (loss(alpha + h) - loss(alpha - h)) / (2 * h)
    assert abs(g - fd) <= 1e-6 * abs(fd)
    # dL/db = lambda: check one component by finite differences
    e = np.zeros(n)
    e[5] = 1.0
    xp = sla.spsolve(A.tocsc(), b + h * e)
    xm = sla.spsolve(A.tocsc(), b - h * e)
    fdb = (0.5 * np.sum((xp - xt) ** 2) - 0.5 * np.sum((xm - xt) ** 2)) / (2 * h)
    assert abs(lam[5] - fdb) <= 1e-6 * abs(fdb)


# ---------------------------------------------------------------------------
# stability check inside the setup, degree lowering (section 3.5)
# ---------------------------------------------------------------------------

def _clusters_problem():
    from workloads import diag_clusters

    A = diag_clusters().to_scipy()
    n = A.shape[0]
    return A, rhs(n, 1), start_vector(n, 2)


def test_leading_hessenberg_block_is_the_lower_degree_cycle():
    # the reading behind degree lowering: the first k Arnoldi steps from v0
    # are the GMRES(k) cycle, so the leading (k+1) x k block of one GMRES(30)
    # run gives the roots of a separate GMRES(k) setup
    A, b, v0 = _clusters_problem()
    _, Hbar, k, brk = roots.arnoldi(lambda v: A @ v, v0, 30, "cgs2")
    assert k == 30 and not brk
    for kk in (5, 10, 20):
        lead = np.sort_complex(roots.harmonic_ritz(Hbar[: kk + 1, :kk]))
        fresh = np.sort_complex(roots.setup(A, v0, kk, add_roots=False, orth="cgs2").theta)
        assert np.max(np.abs(lead - fresh)) <= 1e-12 * np.max(np.abs(fresh))


@pytest.mark.parametrize("case", ["clusters_no_added_roots", "wide_added_roots"])
def test_setup_checked_keeps_the_first_stable_degree(case):
    # brute force: StCh of a fresh setup at every degree tried; the kept
    # degree is the first whose StCh passes, every earlier one fails
    from workloads import diag_wide

    if case == "clusters_no_added_roots":
        A, b, v0 = _clusters_problem()
        add, want = False, 10
    else:
        A = diag_wide().to_scipy()
        b, v0 = rhs(A.shape[0], 1), start_vector(A.shape[0], 2)
        add, want = True, 20
    P, st, unstable, tried = solver.setup_checked(A, v0, 40, b, 1e-8, d_step=10, d_min=10, add_roots=add,
                                                  orth="cgs2")
    assert not unstable and P.d == want and st <= 1e-8
    assert [k for k, _ in tried] == list(range(40, want - 1, -10))
    for k, _ in tried:
        Pk = roots.setup(A, v0, k, add_roots=add, orth="cgs2")
        sk = solver.stability_check(A, Pk.units, b)
        assert (sk <= 1e-8) == (k == want), (k, sk)


def test_setup_checked_flags_unstable_and_keeps_smallest_stch():
    A, b, v0 = _clusters_problem()
    P, st, unstable, tried = solver.setup_checked(A, v0, 40, b, 0.0, d_step=10, d_min=10, add_roots=False,
                                                  orth="cgs2")
    assert unstable
    vals = {k: (s if np.isfinite(s) else np.inf) for k, s in tried}
    assert P.d == min(vals, key=vals.get) == 10 and st == vals[10]
    # no lowering: only d is tried
    P1, st1, unstable1, tried1 = solver.setup_checked(A, v0, 20, b, 1e-8, d_step=0, add_roots=False, orth="cgs2")
    assert [k for k, _ in tried1] == [20] and unstable1 and P1.d == 20 and st1 > 1.0


# ---------------------------------------------------------------------------
# composition with a diagonal right preconditioner (eqs. 1.3-1.4)
# ---------------------------------------------------------------------------

def test_jacobi_scaled_operator_closed_forms():
    from workloads import convdiff2d_colscaled

    A0 = convdiff2d(30, 5.0).to_scipy()
    A = convdiff2d_colscaled(30, 5.0, 3.0).to_scipy()
    AS, s = solver.right_scaled(A)
    # unit diagonal, and the column scaling cancels: A0 S (D0 S)^{-1} = A0 D0^{-1}
    assert np.max(np.abs(AS.diagonal() - 1.0)) <= 2.0 ** -52
    AS0, _ = solver.right_scaled(A0)
    d = (AS - AS0).tocsr()
    assert np.max(np.abs(d.data)) <= 4 * np.finfo(float).eps * np.max(np.abs(AS0.data))
    with pytest.raises(ValueError):
        solver.right_scaled(diagonal(np.array([1.0, 0.0, 2.0])).to_scipy())


def test_jacobi_composition_solves_badly_scaled_system():
    # x = M^{-1} p(A M^{-1}) y solves A x = b; the composition removes the
    # column scaling that stops the plain polynomial preconditioned solve
    from workloads import convdiff2d_colscaled

    A = convdiff2d_colscaled(50, 1.0, 3.0).to_scipy()
    n = A.shape[0]
    b, v0 = rhs(n, 1), start_vector(n, 2)
    AS, s = solver.right_scaled(A)
    PJ = roots.setup(AS, v0, 10, orth="cgs2")
    xt, infj = solver.pp_gmres(AS, b, PJ.units, m=50, tol=1e-8, max_cycles=50)
    x = s * xt
    assert infj.status == solver.OK and infj.cycles <= 2
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - sla.spsolve(A.tocsc(), b)) <= 1e-5 * np.linalg.norm(x)
    P = roots.setup(A, v0, 10, orth="cgs2")
    _, inf = solver.pp_gmres(A, b, P.units, m=50, tol=1e-8, max_cycles=30)
    assert inf.status == solver.NOCONV


def test_custom_right_scaling_solves():
    A = convdiff2d(20, 10.0).to_scipy()
    n = A.shape[0]
    b, v0 = rhs(n, 1), start_vector(n, 2)
    s = 10.0 ** np.random.default_rng(4).uniform(-1, 1, n)
    AS, s2 = solver.right_scaled(A, s)
    assert np.array_equal(s2, s)
    P = roots.setup(AS, v0, 8, orth="cgs2")
    xt, inf = solver.pp_gmres(AS, b, P.units, m=50, tol=1e-10, max_cycles=50)
    assert np.linalg.norm(b - A @ (s * xt)) <= 1e-10 * np.linalg.norm(b)


def test_block_jacobi_operator_closed_forms():
    import scipy.sparse as sp

    from workloads import convdiff2d_blockmixed

    A0 = convdiff2d(20, 5.0).to_scipy()
    n = A0.shape[0]
    # bs = 1 is Jacobi: a_ij / a_jj
    B1, M1 = solver.block_jacobi(A0, 1)
    AS, s = solver.right_scaled(A0)
    assert np.array_equal(M1.diagonal(), s)
    assert np.max(np.abs((B1 - AS).toarray())) <= 2 * np.finfo(float).eps * np.max(np.abs(AS.data))
    # M^{-1} inverts the diagonal blocks (bs = 3: the last block holds one row)
    B, Minv = solver.block_jacobi(A0, 3)
    Mb = sp.block_diag([A0[r:r + 3, r:r + 3].toarray() for r in range(0, n, 3)], format="csr")
    assert np.max(np.abs((Minv @ Mb - sp.identity(n)).toarray())) <= 1e-14
    # B (M x) = A x, and B's diagonal blocks are the identity
    x = np.random.default_rng(3).standard_normal(n)
    assert np.linalg.norm(B @ (Mb @ x) - A0 @ x) <= 1e-13 * np.linalg.norm(A0 @ x)
    for r in range(0, n, 3):
        blk = B[r:r + 3, r:r + 3].toarray()
        assert np.max(np.abs(blk - np.eye(blk.shape[0]))) <= 1e-14
    # a block-diagonal mixing R on the right cancels: (A0 R) M^{-1} = A0 M0^{-1}
    Am = convdiff2d_blockmixed(20, 5.0, 4, 2.0).to_scipy()
    Bm, _ = solver.block_jacobi(Am, 4)
    B0, _ = solver.block_jacobi(A0, 4)
    assert np.max(np.abs((Bm - B0).toarray())) <= 1e-11 * np.max(np.abs(B0.data))


def test_block_jacobi_composition_solves_mixed_system():
    from workloads import convdiff2d_blockmixed

    A = convdiff2d_blockmixed(40, 5.0, 4, 2.0).to_scipy()
    n = A.shape[0]
    b, v0 = rhs(n, 1), start_vector(n, 2)
    B, Minv = solver.block_jacobi(A, 4)
    PB = roots.setup(B, v0, 10, orth="cgs2")
    y, inf = solver.pp_gmres(B, b, PB.units, m=50, tol=1e-8, max_cycles=30)
    x = Minv @ y
    assert inf.status == solver.OK and inf.cycles <= 2
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - sla.spsolve(A.tocsc(), b)) <= 1e-5 * np.linalg.norm(x)
    P = roots.setup(A, v0, 10, orth="cgs2")
    _, inf0 = solver.pp_gmres(A, b, P.units, m=50, tol=1e-8, max_cycles=30)
    assert inf0.status == solver.NOCONV


# ---------------------------------------------------------------------------
# polynomial changed at every cycle (section 5.2, ChPoly)
# ---------------------------------------------------------------------------

def test_chpoly_first_cycle_uses_the_polynomial_from_b():
    # the first residual is b, so cycle 1 is PP-GMRES with GMRES(d) started at b
    A = convdiff2d(30, 10.0).to_scipy()
    b = rhs(A.shape[0], 1)
    x1, i1 = solver.pp_gmres(A, b, None, m=20, tol=1e-12, max_cycles=1, orth="cgs2", new_poly_degree=8)
    P = roots.setup(A, b, 8, orth="cgs2")
    x2, i2 = solver.pp_gmres(A, b, P.units, m=20, tol=1e-12, max_cycles=1, orth="cgs2")
    assert np.array_equal(x1, x2)
    assert i1.mvps == i2.mvps + P.d and i1.cycles == i2.cycles == 1


def test_chpoly_needs_fewer_mvps_at_low_degree():
    # Table 5.1's trend at low degree, on Example 12's matrix scaled down to
    # n = 2000: the changing polynomial needs far fewer products
    from workloads import diag_squares

    n = 2000
    A = diag_squares(n).to_scipy()
    b, v0 = rhs(n, 1), start_vector(n, 2)
    x, ich = solver.pp_gmres(A, b, None, m=50, tol=1e-10, max_cycles=5000, orth="cgs2", new_poly_degree=10,
                             stall_cycles=0)
    assert ich.status == solver.OK and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    P = roots.setup(A, v0, 10, orth="cgs2")
    _, ipp = solver.pp_gmres(A, b, P.units, m=50, tol=1e-10, max_cycles=5000, orth="cgs2", setup_mvps=P.d,
                             stall_cycles=0)
    assert ipp.status == solver.OK and ich.mvps < ipp.mvps / 2


def test_biharmonic_condition_number_example3(golden_dir):
    # Example 3: the 13-point reading of the operator gives the printed
    # condition number 8.2e7 (the 9-point reading without u_xxyy gives 5.3e7)
    import os

    from workloads import biharmonic2d

    with open(os.path.join(golden_dir, "example3_biharmonic.txt")) as fh:
        cond_paper = float(next(l for l in fh if "condition_number" in l).split()[-1])
    A = biharmonic2d(200).to_scipy()
    assert A.shape[0] == 40000 and np.median(np.diff(A.indptr)) == 13
    smax = sla.svds(A, k=1, which="LM", return_singular_vectors=False)[0]
    lu = sla.splu(A.tocsc())
    x = np.random.default_rng(0).standard_normal(A.shape[0])
    for _ in range(60):  # inverse iteration on A^T A for the smallest singular value
        z = lu.solve(lu.solve(x), trans="T")
        nz = np.linalg.norm(z)
        x = z / nz
    cond = smax * np.sqrt(nz)
    assert abs(cond - cond_paper) <= 0.02 * cond_paper, cond


def test_double_polynomial_solve_small():
    # PP-GMRES with phi2(phi1(A)) solves A x = b (x = p1(A) p2(phi1(A)) z)
    from workloads import biharmonic2d

    A = biharmonic2d(30).to_scipy()
    n = A.shape[0]
    b, v0 = rhs(n, 1), start_vector(n, 2)
    P1 = roots.setup(A, v0, 6, orth="cgs2")
    P2 = roots.setup_double(A, P1.units, v0, 6, orth="cgs2")
    x, info = solver.pp_gmres(A, b, P2.units, m=50, tol=1e-10, orth="cgs2", inner_units=P1.units)
    assert info.status == solver.OK
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - sla.spsolve(A.tocsc(), b)) <= 1e-4 * np.linalg.norm(x)
