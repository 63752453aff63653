"""GPU parity of the batched solver against the FP64 oracle: every system's
Leja order and added roots bit for bit, and every (system, right-hand side)
solution against the oracle's PP-GMRES with that system's polynomial."""

import time

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import roots as oroots, solver as osolver
from workloads import batched_convdiff_specs, convdiff2d, normal_vector, rhs, start_vector
from gpu_util import say, dev, host, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import paper_1911_07065_amd.api as api

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return api


def _systems(specs):
    return [convdiff2d(N, alpha) for (N, alpha, _, _) in specs]


def _rhs_block(specs, R):
    # R normalised N(0,1) right-hand sides per system, from the system's seed
    return [rhs(N * N, seed, count=R) for (N, _, seed, _) in specs]


def _v0(specs):
    return np.concatenate([start_vector(N * N, seed) for (N, _, _, seed) in specs])


def _blockdiag(csrs):
    return sp.block_diag([c.to_scipy() for c in csrs]).tocsr()


def _inv_norm_bound_2d(N):
    """1 / lambda_min of the symmetric part of the h^2-scaled 2-D
    convection-diffusion matrix on an N x N grid (centred convection only
    changes the skew part, so the symmetric part is the 5-point Laplacian with
    diagonal 4, smallest eigenvalue 2 (2 - 2 cos(pi h)), h = 1/(N+1)). Since
    ||A y|| ||y|| >= y^T A y >= lambda_min ||y||^2, this bounds ||A^-1||_2."""
    h = 1.0 / (N + 1)
    return 1.0 / (2.0 * (2.0 - 2.0 * np.cos(np.pi * h)))


def _check_systems_against_oracle(specs, csrs, polys, brs, X, infos, R, m, systems, tag):
    """For each system s listed: its Leja order and final root list equal the
    oracle's rules applied to its own harmonic Ritz values, bit for bit; for
    each right-hand side r, x equals the oracle's PP-GMRES solution with that
    polynomial within the bound ||x - x_or|| <= ||A^-1|| (||r|| + ||r_or||),
    both residuals at most tol ||b||."""
    off = np.concatenate([[0], np.cumsum([c.n for c in csrs])])
    worst = 0.0
    for s in systems:
        A = csrs[s].to_scipy()
        theta = polys[s].roots("theta")
        leja, pof, n_add, units = oroots.order_and_add(theta)
        assert np.array_equal(polys[s].roots("leja"), leja), s
        fin = oroots.Poly(polys[s].d, theta, leja, pof, n_add, units).roots()
        assert np.array_equal(polys[s].roots("final"), fin), s
        inv_bound = _inv_norm_bound_2d(specs[s][0])
        for r in range(R):
            b = brs[s][r]
            xs = X[r, off[s]:off[s + 1]]
            xo, io = osolver.pp_gmres(A, b, units, m=m, tol=1e-8, orth="cgs2")
            res = np.linalg.norm(b - A @ xs)
            res_o = np.linalg.norm(b - A @ xo)
            assert infos[s * R + r]["converged"] and res <= 1e-8 * np.linalg.norm(b), (s, r, res)
            assert io.status == osolver.OK and res_o <= 1e-8 * np.linalg.norm(b)
            err = relerr(xs, xo)
            bound = inv_bound * (res + res_o) / np.linalg.norm(xo)
            worst = max(worst, err)
            say(f"result batched {tag} system {s} (N={specs[s][0]}) rhs {r}: relres {res / np.linalg.norm(b):.2e}, "
                f"||x - x_oracle||/||x_oracle|| {err:.2e} (bound {bound:.2e})")
            assert err <= bound * (1 + 1e-9) + 1e-15, (s, r, err, bound)
    return worst


SMALL = [(16, 3.0, 1000, 5000), (23, 40.0, 1001, 5001), (31, 0.0, 1002, 5002), (40, 12.5, 1003, 5003),
         (9, 7.0, 1004, 5004), (28, 25.0, 1005, 5005)]


@pytest.mark.parametrize("fmt", ["box", "pattern", "sell"])
@pytest.mark.parametrize("inner", ["fp64", "fp32"])
@pytest.mark.parametrize("R", [1, 4])
def test_small_batch_matches_single_solves(pp, inner, R, fmt):
    csrs = _systems(SMALL)
    say("batch small", inner, R, fmt)
    Bt = pp.Batch(csrs)
    assert Bt.format() == "pattern"  # every system is a 5-point stencil: 9 row patterns each
    Bt.set_format(fmt)
    polys = Bt.setup(dev(_v0(SMALL)), 8)
    brs = _rhs_block(SMALL, R)
    bmat = np.concatenate(brs, axis=1)  # (R, n_total)
    x, infos = Bt.solve(polys, Bt.interleave(bmat), R, tol=1e-8, m=30, inner=inner)
    X = host(Bt.deinterleave(x, R))
    Abig = _blockdiag(csrs)
    off = np.concatenate([[0], np.cumsum([c.n for c in csrs])])
    for s, c in enumerate(csrs):
        A = c.to_scipy()
        # the batched polynomial equals the single-system setup's up to rounding
        M = pp.Matrix.from_csr(c)
        single = pp.setup(M, dev(start_vector(c.n, SMALL[s][3])), 8)
        th_b = np.sort_complex(polys[s].roots("theta"))
        th_s = np.sort_complex(single.roots("theta"))
        assert np.max(np.abs(th_b - th_s) / np.abs(th_s)) < 1e-8
        for r in range(R):
            p = s * R + r
            xs = X[r, off[s]:off[s + 1]]
            rel = np.linalg.norm(brs[s][r] - A @ xs) / np.linalg.norm(brs[s][r])
            assert infos[p]["converged"] and rel <= 1e-8, (s, r, infos[p], rel)
            xo, io = pp.solve(single, M, dev(brs[s][r]), tol=1e-8, m=30, inner=inner)
            assert relerr(xs, host(xo)) < 1e-5
    # the whole block system
    R_all = bmat - (Abig @ X.T).T
    assert np.all(np.linalg.norm(R_all, axis=1) <= 1e-8 * np.linalg.norm(bmat, axis=1) * np.sqrt(len(csrs)))


@pytest.mark.parametrize("orth", ["delayed", "cgs2"])
@pytest.mark.parametrize("fmt", ["box", "pattern", "sell"])
@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("R", [1, 4])
def test_small_batch_matches_oracle(pp, inner, R, fmt, orth):
    csrs = _systems(SMALL)
    say("batch small vs oracle", inner, R, fmt, orth)
    Bt = pp.Batch(csrs)
    assert Bt.orth() == "delayed"  # the default: two basis sweeps per step
    Bt.set_orth(orth)
    Bt.set_format(fmt)
    polys = Bt.setup(dev(_v0(SMALL)), 8)
    brs = _rhs_block(SMALL, R)
    x, infos = Bt.solve(polys, Bt.interleave(np.concatenate(brs, axis=1)), R, tol=1e-8, m=30, inner=inner)
    X = host(Bt.deinterleave(x, R))
    _check_systems_against_oracle(SMALL, csrs, polys, brs, X, infos, R, 30, range(len(SMALL)),
                                  f"small {inner} R={R} {fmt}")


@pytest.mark.parametrize("R", [1, 4])
def test_batch_tuner_and_every_launch_shape(pp, R):
    # the batched autotuner picks a valid shape; every shape (format, slices
    # per wave, workgroup order) gives each pair's solution within the
    # oracle bound, and all shapes agree with each other to the solve's
    # accuracy
    csrs = _systems(SMALL)
    say("batch tuner", R)
    Bt = pp.Batch(csrs)
    polys = Bt.setup(dev(_v0(SMALL)), 8)
    brs = _rhs_block(SMALL, R)
    bd = Bt.interleave(np.concatenate(brs, axis=1))
    fmt, spw, remap, us = Bt.tune(R, "fp32")
    assert fmt in ("sell", "pattern", "box") and spw in (1, 2) and remap in (0, 1) and us > 0
    assert Bt.chain_config(R, "fp32") == (fmt, spw, remap, us)
    xs = []
    for shape in [("sell", 1, 0), ("sell", 1, 1), ("pattern", 1, 0), ("pattern", 1, 1), ("pattern", 2, 0),
                  ("pattern", 2, 1), ("box", 1, 0), ("box", 1, 1), ("box", 2, 0), ("box", 2, 1)]:
        say("batch shape", R, shape)
        Bt.set_chain_config(R, "fp32", *shape)
        Bt.set_chain_config(R, "fp64", *shape)
        assert Bt.chain_config(R, "fp32")[:3] == shape
        x, infos = Bt.solve(polys, bd, R, tol=1e-8, m=30, inner="fp32")
        X = host(Bt.deinterleave(x, R))
        _check_systems_against_oracle(SMALL, csrs, polys, brs, X, infos, R, 30, range(len(SMALL)),
                                      f"shape {shape} R={R}")
        xs.append(X)
    for X in xs[1:]:
        assert relerr(X, xs[0]) <= 1e-6
    with pytest.raises(Exception):
        Bt.set_chain_config(R, "fp32", "sell", 2, 1)  # two slices per wave only on the pattern-coded copy


def test_batch_pattern_copy_rules(pp):
    # a batch whose systems lie on different numbers of diagonals has no
    # pattern-coded copy; new values drop it, and the sliced-ELL products
    # then use the new values
    import scipy.sparse as sp

    from workloads.generators import CSR

    T = sp.diags([np.full(99, -1.0), np.full(100, 2.5), np.full(99, -1.2)], [-1, 0, 1], format="csr")
    tri = CSR(n=100, rowptr=T.indptr.astype(np.int32), colind=T.indices.astype(np.int32),
              val=T.data.astype(np.float64))
    say("batch pattern rules")
    assert pp.Batch([convdiff2d(12, 3.0), tri]).format() == "sell"
    with pytest.raises(Exception, match="pattern-coded"):
        pp.Batch([convdiff2d(12, 3.0), tri]).set_format("pattern")
    with pytest.raises(Exception, match="box-stencil"):
        pp.Batch([convdiff2d(12, 3.0), tri]).set_format("box")
    # a 5-point stencil whose coefficients vary along the grid keeps the
    # pattern-coded copy but has no box copy
    var = convdiff2d(12, 3.0)
    rows = np.repeat(np.arange(var.n), np.diff(var.rowptr))
    var = CSR(n=var.n, rowptr=var.rowptr, colind=var.colind, val=var.val * (1.0 + 0.01 * (rows % 5)))
    Bv = pp.Batch([convdiff2d(12, 3.0), var])
    assert Bv.format() == "pattern"
    Bv.set_format("pattern")
    with pytest.raises(Exception, match="box-stencil"):
        Bv.set_format("box")
    specs = SMALL[:3]
    csrs = _systems(specs)
    Bt = pp.Batch(csrs)
    assert Bt.format() == "pattern"
    polys = Bt.setup(dev(_v0(specs)), 8)
    bd = Bt.interleave(np.concatenate(_rhs_block(specs, 1), axis=1))
    x1, i1 = Bt.solve(polys, bd, 1, tol=1e-10, m=30, inner="fp64")
    vals = np.concatenate([c.val for c in csrs])
    Bt.set_values(2.0 * vals)
    assert Bt.format() == "sell"
    with pytest.raises(Exception, match="pattern-coded"):
        Bt.set_format("pattern")
    with pytest.raises(Exception, match="box-stencil"):
        Bt.set_format("box")
    # (2A) x = b: x is half the first solution (same roots, scaled problem)
    polys2 = Bt.setup(dev(_v0(specs)), 8)
    x2, i2 = Bt.solve(polys2, bd, 1, tol=1e-10, m=30, inner="fp64")
    assert all(i["converged"] for i in i1 + i2)
    assert relerr(host(x2), 0.5 * host(x1)) < 1e-8


def test_batch_rejects_coupled_blocks(pp):
    csrs = _systems(SMALL[:2])
    Bt = pp.Batch(csrs)  # valid
    import ctypes
    from paper_1911_07065_amd._lib import lib

    # a pattern whose row 0 reaches into the second system
    n0, n1 = csrs[0].n, csrs[1].n
    rp = np.arange(n0 + n1 + 1, dtype=np.int32)
    ci = np.arange(n0 + n1, dtype=np.int32)
    ci[0] = n0 + 3
    ro = np.array([0, n0, n0 + n1], dtype=np.int64)
    h = ctypes.c_void_p()
    st = lib.pp_batch_create(2, ro.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n0 + n1,
                             ctypes.c_void_p(dev(rp, torch.int32).data_ptr()),
                             ctypes.c_void_p(dev(ci, torch.int32).data_ptr()),
                             ctypes.c_void_p(dev(np.ones(n0 + n1)).data_ptr()), None, ctypes.byref(h))
    assert st == -1


def test_batched_config_full_size(pp):
    # 256 2-D convection-diffusion systems, sides U{64..512}, alpha U[0,50),
    # 4 right-hand sides each, degree 20, GMRES(50), FP32 inner / FP64 outer
    specs = batched_convdiff_specs()
    csrs = _systems(specs)
    n_tot = sum(c.n for c in csrs)
    say("batched full", len(csrs), "systems", n_tot, "rows")
    Bt = pp.Batch(csrs)
    v0 = dev(_v0(specs))
    bmat = np.concatenate(_rhs_block(specs, 4), axis=1)
    bd = Bt.interleave(bmat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    polys = Bt.setup(v0, 20)
    x, infos = Bt.solve(polys, bd, 4, tol=1e-8, m=50, inner="fp32")
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    X = host(Bt.deinterleave(x, 4))
    Abig = _blockdiag(csrs)
    Rres = bmat - (Abig @ X.T).T
    off = np.concatenate([[0], np.cumsum([c.n for c in csrs])])
    worst = 0.0
    for s in range(len(csrs)):
        for r in range(4):
            seg = slice(off[s], off[s + 1])
            worst = max(worst, np.linalg.norm(Rres[r, seg]) / np.linalg.norm(bmat[r, seg]))
    say("batched full: time", round(t_batch, 3), "s, worst relres", worst,
        "max iters", max(i["iters"] for i in infos), "max cycles", max(i["cycles"] for i in infos))
    assert all(i["converged"] for i in infos) and worst <= 1e-8
    # 8 systems of the full batch (every 32nd: sides 70 to 458) against the
    # oracle, every right-hand side, with the polynomial each system got
    sample = list(range(0, len(csrs), 32))
    xw = _check_systems_against_oracle(specs, csrs, polys, _rhs_block(specs, 4), X, infos, 4, 50, sample, "full")
    say("batched full: worst ||x - x_oracle||/||x_oracle|| over", len(sample), "systems x 4 rhs:", xw)
    # the same work as a loop of single-system solves, timed on every 16th
    # system and scaled to the whole batch
    t_loop = 0.0
    sub = list(range(0, len(csrs), 16))
    brs = _rhs_block(specs, 4)
    for s in sub:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        M = pp.Matrix.from_csr(csrs[s])
        M.tune("fp32")
        M.tune("fp64")
        poly = pp.setup(M, dev(start_vector(csrs[s].n, specs[s][3])), 20)
        for r in range(4):
            xs, io = pp.solve(poly, M, dev(brs[s][r]), tol=1e-8, m=50, inner="fp32")
            assert io["converged"]
        torch.cuda.synchronize()
        t_loop += time.perf_counter() - t1
    t_loop *= len(csrs) / len(sub)
    say("loop of single solves (scaled from", len(sub), "systems):", round(t_loop, 3), "s; batched", round(t_batch, 3),
        "s; speed-up", round(t_loop / t_batch, 2))


@pytest.mark.parametrize("orth", ["delayed", "cgs2"])
@pytest.mark.parametrize("fmt", ["box", "pattern", "sell"])
@pytest.mark.parametrize("R", [1, 4])
def test_batched_graph_replays_equal_eager(pp, R, fmt, orth):
    # Arnoldi steps captured into HIP graphs and replayed over several cycles
    # (with eager launches, host work and synchronisations between replays)
    # give the eager result bit for bit: x, every pair's counters and the
    # residual history of every cycle
    specs = SMALL
    csrs = _systems(specs)
    say("batched graphs", R, fmt, orth)
    Bt = pp.Batch(csrs)
    Bt.set_orth(orth)
    Bt.set_format(fmt)
    bd = Bt.interleave(np.concatenate(_rhs_block(specs, R), axis=1))
    polys = Bt.setup(dev(_v0(specs)), 6)
    xe, ie = Bt.solve(polys, bd, R, tol=1e-11, m=8, inner="fp32", graphs=False)
    assert max(i["cycles"] for i in ie) >= 3 and all(i["converged"] for i in ie)
    for _ in range(2):
        xg, ig = Bt.solve(polys, bd, R, tol=1e-11, m=8, inner="fp32", graphs=True)
        assert torch.equal(xg, xe)
        for a, b in zip(ig, ie):
            for k in ("iters", "cycles", "mvps", "dots", "fp64_cycles"):
                assert a[k] == b[k], k
            assert a["relres"] == b["relres"]
        xe2, _ = Bt.solve(polys, bd, R, tol=1e-11, m=8, inner="fp32", graphs=False)
        assert torch.equal(xe2, xe)


@pytest.mark.parametrize("orth", ["delayed", "cgs2"])
def test_batch_repeats_bit_for_bit(pp, orth):
    # every reduction (wave sums, block partials, per-system passes) has a
    # fixed order: the same batch solved twice gives the same roots, x and
    # counters bit for bit
    csrs = _systems(SMALL)
    say("batch repeatability", orth)
    Bt = pp.Batch(csrs)
    Bt.set_orth(orth)
    brs = _rhs_block(SMALL, 4)
    bd = Bt.interleave(np.concatenate(brs, axis=1))
    runs = []
    for _ in range(2):
        polys = Bt.setup(dev(_v0(SMALL)), 8)
        x, infos = Bt.solve(polys, bd, 4, tol=1e-8, m=30, inner="fp32")
        runs.append(([p.roots("final") for p in polys], host(x), infos))
    (r0, x0, i0), (r1, x1, i1) = runs
    assert all(np.array_equal(a, b) for a, b in zip(r0, r1))
    assert np.array_equal(x0, x1)
    for a, b in zip(i0, i1):
        assert a["cycles"] == b["cycles"] and a["iters"] == b["iters"] and a["relres"] == b["relres"]
