"""GPU parity of two chain steps per launch (box stencils) against the oracle.

Two consecutive real roots of Algorithm 1 or 3 run as one launch on a
5- or 7-point stencil matrix. The results must equal the oracle's chains
(and the single-step launches up to rounding order) for boxes whose sides
are not multiples of the tile, for polynomials that mix real roots,
conjugate pairs and added copies, and inside a full solve.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import chains, roots as oroots
from oracle.mixed import apply_p_low, apply_phi_low
from workloads import CSR, convdiff2d, convdiff3d, convdiff3d_box, randsparse, rhs, start_vector
from gpu_util import say, dev, host, relerr, maxerr, assert_close, box_face_rows, tail_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import paper_1911_07065_amd.api as api

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return api


def _wrapped(nx, ny, nz):
    # 7 full diagonals 0, +-1, +-nx, +-nx ny: entries join the end of every
    # grid line to the start of the next, so the matrix is not a box stencil
    n = nx * ny * nz
    offs = [-nx * ny, -nx, -1, 0, 1, nx, nx * ny]
    vals = [-0.5, -0.7, -1.1, 6.0, -0.9, -1.3, -0.6]
    A = sp.diags([np.full(n - abs(o), v) for o, v in zip(offs, vals)], offs, format="csr")
    A.sort_indices()
    return CSR(n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def _varcoef(csr, classes=3):
    # row r's entries scaled by 1 + 0.1 (r mod classes): a box stencil whose
    # rows are not one interior row truncated at the box (variable coefficients)
    rows = np.repeat(np.arange(csr.n), np.diff(csr.rowptr))
    return csr.with_values(csr.val * (1.0 + 0.1 * (rows % classes)))


def _cases():
    # box sides that leave partial tiles in every direction (3-D tiles 32 x 8 x 8
    # and 32 x 8 x 4, 2-D tiles 64 x 32; marching tiles 64 x 4 and 256)
    return {
        "box3d_37x11x10": (convdiff3d_box(37, 11, 10, 10.0, 5.0, 2.0), (37, 11, 10), 12),
        "convdiff3d_20": (convdiff3d(20, 10, 10, 10), (20, 20, 20), 12),
        "convdiff2d_70": (convdiff2d(70, 5.0), (70, 70, 1), 12),
        "box3d_9x7x33": (convdiff3d_box(9, 7, 33, 1.0, 1.0, 1.0), (9, 7, 33), 6),
        "varcoef3d_21x13x11": (_varcoef(convdiff3d_box(21, 13, 11, 3.0, 2.0, 1.0)), (21, 13, 11), 8),
        "varcoef2d_300x17": (_varcoef(convdiff3d_box(300, 17, 1, 3.0, 2.0, 0.0)), (300, 17, 1), 8),
    }


# constant-coefficient stencils (every row the interior row's stencil truncated at the box)
CONSTANT = {"box3d_37x11x10", "convdiff3d_20", "convdiff2d_70", "box3d_9x7x33"}


def test_box_geometry_detected(pp):
    for name, (csr, box, _) in _cases().items():
        M = pp.Matrix.from_csr(csr)
        say("box", name)
        assert M.pair_steps("fp64")[1] == box, name
    for csr in (_wrapped(40, 30, 20), randsparse(5000, 8, seed=3)):
        M = pp.Matrix.from_csr(csr)
        assert M.pair_steps("fp64")[1] is None
        M.set_variant("fp64", 0, 1)
        with pytest.raises(Exception, match="box stencil"):
            M.set_pair_steps(True, "fp64")
    M = pp.Matrix.from_csr(convdiff3d(12, 1, 1, 1))
    with pytest.raises(Exception, match="tune"):
        M.set_pair_steps(True, "fp32")
    M.tune("bf16")
    with pytest.raises(Exception):
        M.set_pair_steps(True, "bf16")
    # forcing a variant runs every step on its own again
    M.tune("fp64")
    M.set_pair_steps(True, "fp64")
    assert M.pair_steps("fp64")[0]
    M.set_variant("fp64", 0, 1)
    assert not M.pair_steps("fp64")[0]


def _polys(pp, A, n, d):
    P = oroots.setup(A, start_vector(n, 2), d)
    th = np.array([7.5, 0.2, 3 + 1j, 3 - 1j, 5 + 0.5j, 5 - 0.5j, 1.0, 0.05, 2.5])
    Q = oroots.poly_from_roots(th, add_roots=True)
    return [("setup", P, pp.poly_from_roots(P.roots(), keep_order=True)),
            ("mixed", Q, pp.poly_from_roots(th, add_roots=True))]


@pytest.mark.parametrize("name", list(_cases()))
def test_pair_steps_match_oracle(pp, name):
    csr, box, d = _cases()[name]
    A = csr.to_scipy()
    A32 = A.astype(np.float32)
    v = rhs(csr.n, 5)
    for pname, P, poly in _polys(pp, A, csr.n, d):
        M = pp.Matrix.from_csr(csr)
        for prec in ("fp64", "fp32"):
            M.tune(prec)
        v32 = v.astype(np.float32)
        ref_phi = chains.apply_phi(A, P.units, v)
        for kind, fn in [("p", chains.apply_p), ("phi", chains.apply_phi), ("pi", chains.apply_pi)]:
            ref = fn(A, P.units, v)
            # the FP32 bound of the other chain tests: 10x the error of the
            # chain emulated in float32 (pi through pi = v - phi)
            flow = apply_p_low if kind == "p" else apply_phi_low
            emu = flow(A32, P.units, v32, "fp32")
            say("pair steps", name, pname, kind)
            got = {}
            for on in (True, False):
                M.set_pair_steps(on, "fp64")
                M.set_pair_steps(on, "fp32")
                g64 = host(pp.apply(poly, M, dev(v), kind))
                g32 = host(pp.apply(poly, M, dev(v32, torch.float32), kind))
                got[on] = g64
                assert_close(g64, ref, 1e-12, f"{name} {pname} {kind} fused={on}", box)
                # element by element, on the whole vector, the box faces (where
                # the fused kernel stages its halo) and the last block
                for idx in (None, box_face_rows(*box), tail_rows(csr.n)):
                    delta = maxerr(emu, ref if kind == "p" else ref_phi, idx)
                    err32 = maxerr(v32 - g32, ref_phi, idx) if kind == "pi" else maxerr(g32, ref, idx)
                    assert err32 <= 10 * delta + 1e-6, (on, err32, delta)
            # the same arithmetic as single launches up to the order of rounding
            assert_close(got[True], got[False], 1e-14, "fused vs single", box)


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_pair_steps_in_a_solve(pp, inner):
    # a full PP-GMRES solve with two steps per launch against the oracle's x
    from oracle import solver as osolver

    csr = convdiff3d_box(40, 36, 30, 10.0, 10.0, 10.0)
    A = csr.to_scipy()
    b, v0 = rhs(csr.n, 1), start_vector(csr.n, 2)
    M = pp.Matrix.from_csr(csr)
    M.tune(inner)
    M.set_pair_steps(True, inner)
    poly = pp.setup(M, dev(v0), 20)
    P = oroots.setup(A, v0, 20, orth="cgs2")
    say("pair steps solve", inner, "d_eff", poly.d_eff)
    x, info = pp.solve(poly, M, dev(b), tol=1e-8, m=50, inner=inner)
    assert M.pair_steps(inner)[0]
    xh = host(x)
    assert info["converged"]
    assert np.linalg.norm(b - A @ xh) <= 1e-8 * np.linalg.norm(b)
    y, _ = osolver.pp_gmres(A, b, P.units, m=50, tol=1e-8)
    assert relerr(xh, y) <= (1e-9 if inner == "fp64" else 2e-5)


def test_pair_steps_full_size(pp):
    # the benchmark's 128^3 workload: phi and p chains with two steps per
    # launch against the oracle (FP64) and against single launches (FP32)
    csr = convdiff3d(128, 10, 10, 10)
    A = csr.to_scipy()
    P = oroots.setup(A, start_vector(csr.n, 2), 10)
    M = pp.Matrix.from_csr(csr)
    M.tune("fp64")
    M.tune("fp32")
    poly = pp.poly_from_roots(P.roots(), keep_order=True)
    v = rhs(csr.n, 5)
    say("pair steps 128^3")
    box = (128, 128, 128)
    for steps in (2, 3, 4):
        # several steps per marching launch on the full-size grid
        for kind, fn in [("phi", chains.apply_phi), ("pi", chains.apply_pi)]:
            ref = fn(A, P.units, v)
            say("march 128^3", kind, steps)
            M.set_march(steps, "fp64")
            assert_close(host(pp.apply(poly, M, dev(v), kind)), ref, 1e-12, f"128^3 {kind} march {steps}", box)
            M.set_march(steps, "fp32")
            got32 = host(pp.apply(poly, M, dev(v, torch.float32), kind))
            emu = apply_phi_low(A.astype(np.float32), P.units, v.astype(np.float32), "fp32")
            ref_phi = chains.apply_phi(A, P.units, v)
            for idx in (None, box_face_rows(*box), tail_rows(csr.n)):
                err = maxerr(v.astype(np.float32) - got32, ref_phi, idx) if kind == "pi" else maxerr(got32, ref, idx)
                assert err <= 10 * maxerr(emu, ref_phi, idx) + 1e-6
            M.set_march(0, "fp64")
            M.set_march(0, "fp32")
    for kind, fn in [("p", chains.apply_p), ("phi", chains.apply_phi)]:
        ref = fn(A, P.units, v)
        M.set_pair_steps(True, "fp64")
        assert_close(host(pp.apply(poly, M, dev(v), kind)), ref, 1e-12, f"128^3 {kind}", box)
        M.set_pair_steps(True, "fp32")
        got32 = host(pp.apply(poly, M, dev(v, torch.float32), kind))
        flow = apply_p_low if kind == "p" else apply_phi_low
        emu = flow(A.astype(np.float32), P.units, v.astype(np.float32), "fp32")
        for idx in (None, box_face_rows(*box), tail_rows(csr.n)):
            assert maxerr(got32, ref, idx) <= 10 * maxerr(emu, ref, idx) + 1e-6


# ---------------------------------------------------------------------------
# several steps per launch, marching along the grid
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("steps", [2, 3, 4])
@pytest.mark.parametrize("name", list(_cases()))
def test_march_matches_oracle(pp, name, steps):
    # phi and pi chains (real roots, conjugate pairs, added copies) with up to
    # `steps` steps per marching launch, on boxes whose sides leave partial
    # tiles, with the default chunk of planes and with 5 planes (a ragged
    # last chunk): element-wise against the oracle, and against single
    # launches up to rounding order; p chains (their steps carry the
    # accumulator) run unfused and must be unchanged
    csr, box, d = _cases()[name]
    A = csr.to_scipy()
    A32 = A.astype(np.float32)
    v = rhs(csr.n, 5)
    v32 = v.astype(np.float32)
    for pname, P, poly in _polys(pp, A, csr.n, d):
        M = pp.Matrix.from_csr(csr)
        assert M.constant_stencil() == (name in CONSTANT)
        for prec in ("fp64", "fp32"):
            M.tune(prec)
            M.set_pair_steps(False, prec)
        ref_phi = chains.apply_phi(A, P.units, v)
        for kind, fn in [("phi", chains.apply_phi), ("pi", chains.apply_pi), ("p", chains.apply_p)]:
            ref = fn(A, P.units, v)
            emu = (apply_p_low if kind == "p" else apply_phi_low)(A32, P.units, v32, "fp32")
            for prec in ("fp64", "fp32"):
                M.set_march(0, prec)
            single64 = host(pp.apply(poly, M, dev(v), kind))
            # default chunk, 5 planes (a ragged last chunk), and 1 to 3 planes
            # of loads in flight (the deeper prefetch runs on constant stencils)
            for cz, depth in ((0, 1), (5, 3), (0, 2)):
                say("march", name, pname, kind, steps, cz, depth)
                for prec in ("fp64", "fp32"):
                    M.set_march(steps, prec, cz, depth)
                assert M.march("fp64")[0] == steps
                g64 = host(pp.apply(poly, M, dev(v), kind))
                g32 = host(pp.apply(poly, M, dev(v32, torch.float32), kind))
                assert_close(g64, ref, 1e-12, f"{name} {pname} {kind} march {steps} cz {cz}", box)
                assert_close(g64, single64, 1e-14, "march vs single launches", box)
                for idx in (None, box_face_rows(*box), tail_rows(csr.n)):
                    delta = maxerr(emu, ref if kind == "p" else ref_phi, idx)
                    err32 = maxerr(v32 - g32, ref_phi, idx) if kind == "pi" else maxerr(g32, ref, idx)
                    assert err32 <= 10 * delta + 1e-6, (kind, cz, depth, err32, delta)


def test_march_chain_bytes_and_launches(pp):
    # phi(A)v of 8 real roots, 4 steps per launch: 2 launches, each reading
    # its input and its matrix data once and writing its result; the last
    # also reads the final vector: 2 F + 5 n s bytes. On this
    # constant-coefficient stencil the matrix data is the interior row's 7
    # coefficients (no pattern bytes are read)
    csr = convdiff3d(20, 10, 10, 10)
    M = pp.Matrix.from_csr(csr)
    n = csr.n
    poly = pp.poly_from_roots(np.linspace(2.0, 9.0, 8), keep_order=True)
    for prec, sv, sx in (("fp64", 8, 8), ("fp32", 4, 4)):
        M.tune(prec)
        M.set_pair_steps(False, prec)
        M.set_march(4, prec)
        F = 7 * sv
        say("march bytes", prec)
        assert pp.chain_bytes(poly, M, "phi", prec) == (2 * F + 5 * n * sx, 2)
        M.set_march(3, prec)  # groups of 3, 3 and 2
        assert pp.chain_bytes(poly, M, "phi", prec)[1] == 3
        M.set_variant(prec, 27, 1)  # a forced variant turns marching off
        assert M.march(prec)[0] == 0
        assert pp.chain_bytes(poly, M, "phi", prec)[1] == 8
    with pytest.raises(Exception, match="box stencil"):
        Mr = pp.Matrix.from_csr(randsparse(5000, 8, seed=3))
        Mr.tune("fp64")
        Mr.set_march(2, "fp64")
