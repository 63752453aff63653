"""GPU parity of the constant-coefficient box-stencil kernels against the oracle.

On a matrix whose every row is the interior row's 5- or 7-point stencil
truncated at the box (Algorithms 1 and 3 applied to it), two kernels read
no per-row matrix data:
 * the single-step variant "box" (4 points of a grid line per lane), whose
   results must agree with the pattern-coded kernel's up to rounding (the
   same terms summed in the same order; the update may round differently);
 * two steps per launch on tiles of whole grid lines (7-point stencils whose
   lines hold 64, 128 or 256 points).
Both are checked element by element against the oracle's chains, on the box
faces and on the last block of rows, for boxes whose sides leave partial
tiles, for polynomials with real roots, conjugate pairs and added copies,
and at the benchmark's 128^3 size.
"""

import numpy as np
import pytest
import torch

from oracle import chains, roots as oroots
from oracle.mixed import apply_p_low, apply_phi_low
from workloads import convdiff2d, convdiff3d, convdiff3d_box, randsparse, rhs, start_vector
from gpu_util import say, dev, host, maxerr, assert_close, box_face_rows, tail_rows

pytestmark = pytest.mark.gpu

BOX = 31  # the single-step variant's index


@pytest.fixture(scope="module")
def pp():
    import paper_1911_07065_amd.api as api

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    assert api.chain_variant_name(BOX) == "box"
    return api


def _polys(pp, A, n, d):
    P = oroots.setup(A, start_vector(n, 2), d)
    th = np.array([7.5, 0.2, 3 + 1j, 3 - 1j, 5 + 0.5j, 5 - 0.5j, 1.0, 0.05, 2.5])
    Q = oroots.poly_from_roots(th, add_roots=True)
    return [("setup", P, pp.poly_from_roots(P.roots(), keep_order=True)),
            ("mixed", Q, pp.poly_from_roots(th, add_roots=True))]


def _varcoef(csr, classes=3):
    rows = np.repeat(np.arange(csr.n), np.diff(csr.rowptr))
    return csr.with_values(csr.val * (1.0 + 0.1 * (rows % classes)))


# constant-coefficient boxes whose lines hold a multiple of 4 points (the
# handle detects the constant stencil on its diagonal copy, built when
# padding the rows to 256-row blocks adds at most a quarter)
STEP_CASES = {
    "box3d_12x13x17": ((12, 13, 17), (4.0, 2.0, 1.0)),
    "box3d_4x30x30": ((4, 30, 30), (1.0, 1.0, 1.0)),  # one lane holds a whole line
    "convdiff3d_20": ((20, 20, 20), (10.0, 10.0, 10.0)),
    "box2d_64x37": ((64, 37, 1), (5.0, 2.0, 0.0)),
    "box2d_8x300": ((8, 300, 1), (1.0, 3.0, 0.0)),
}


def _box_csr(dims, coef):
    return convdiff3d_box(*dims, *coef)


@pytest.mark.parametrize("name", list(STEP_CASES))
def test_box_step_matches_oracle(pp, name):
    dims, coef = STEP_CASES[name]
    csr = _box_csr(dims, coef)
    A = csr.to_scipy()
    A32 = A.astype(np.float32)
    v = rhs(csr.n, 5)
    v32 = v.astype(np.float32)
    M = pp.Matrix.from_csr(csr)
    assert M.constant_stencil()
    for pname, P, poly in _polys(pp, A, csr.n, 8):
        ref_phi = chains.apply_phi(A, P.units, v)
        for kind, fn in [("p", chains.apply_p), ("phi", chains.apply_phi), ("pi", chains.apply_pi)]:
            ref = fn(A, P.units, v)
            emu = (apply_p_low if kind == "p" else apply_phi_low)(A32, P.units, v32, "fp32")
            # the pattern-coded kernel's results: the same row sums
            M.set_variant("fp64", 27, 1)
            coded64 = host(pp.apply(poly, M, dev(v), kind))
            for remap in (0, 1):
                say("box step", name, pname, kind, remap)
                M.set_variant("fp64", BOX, remap)
                M.set_variant("fp32", BOX, remap)
                M.set_variant("bf16", BOX, remap)
                assert M.variant("fp64")[0] == "box"
                g64 = host(pp.apply(poly, M, dev(v), kind))
                assert_close(g64, ref, 1e-12, f"{name} {pname} {kind} fp64", dims)
                assert_close(g64, coded64, 1e-14, f"{name} {pname} {kind} box vs pattern-coded", dims)
                g32 = host(pp.apply(poly, M, dev(v32, torch.float32), kind))
                for idx in (None, box_face_rows(*dims), tail_rows(csr.n)):
                    delta = maxerr(emu, ref if kind == "p" else ref_phi, idx)
                    err = maxerr(v32 - g32, ref_phi, idx) if kind == "pi" else maxerr(g32, ref, idx)
                    assert err <= 10 * delta + 1e-6, (kind, remap, err, delta)
                # bfloat16 storage: against the emulated BF16 chain
                vb = dev(v, torch.bfloat16)
                gb = host(pp.apply(poly, M, vb, kind))
                if kind != "pi":
                    emub = (apply_p_low if kind == "p" else apply_phi_low)(A32, P.units, host(vb), "bf16")
                    assert maxerr(gb, ref) <= 10 * maxerr(emub, ref) + 1e-6


def test_box_step_refused_where_it_does_not_apply(pp):
    cases = {
        "random": randsparse(4000, 8, seed=3),
        "gx not a multiple of 4": convdiff3d_box(9, 17, 15, 1.0, 1.0, 1.0),
        "variable coefficients": _varcoef(convdiff3d_box(12, 16, 15, 3.0, 2.0, 1.0)),
    }
    for what, csr in cases.items():
        say("box refused", what)
        M = pp.Matrix.from_csr(csr)
        with pytest.raises(Exception, match="box kernel"):
            M.set_variant("fp64", BOX, 1)
        # the tuner never picks it there
        M.tune("fp32")
        assert M.variant("fp32")[0] != "box"


def test_box_step_follows_new_values(pp):
    # scaled coefficients keep the stencil constant: the box variant stays and
    # uses the new coefficients; values that break the constant stencil drop it
    dims = (16, 9, 7)
    csr = convdiff3d_box(*dims, 3.0, 2.0, 1.0)
    M = pp.Matrix.from_csr(csr)
    M.set_variant("fp64", BOX, 1)
    M.set_variant("fp32", BOX, 1)
    poly = pp.poly_from_roots([3.0, 7.5, 2 + 1j, 2 - 1j], keep_order=True)
    units = [(chains.REAL, 3.0, 0.0), (chains.REAL, 7.5, 0.0), (chains.PAIR, 2.0, 1.0)]
    v = rhs(csr.n, 5)
    assert_close(host(pp.apply(poly, M, dev(v), "phi")), chains.apply_phi(csr.to_scipy(), units, v), 1e-12, "phi",
                 dims)
    say("box new values")
    M.set_values(dev(-1.5 * csr.val))
    assert M.variant("fp64")[0] == "box" and M.constant_stencil()
    ref2 = chains.apply_phi(-1.5 * csr.to_scipy(), units, v)
    assert_close(host(pp.apply(poly, M, dev(v), "phi")), ref2, 1e-12, "phi new values", dims)
    val3 = csr.val.copy()
    val3[::7] *= 1.0 + 1e-3
    M.set_values(dev(val3))
    assert not M.constant_stencil()
    assert M.variant("fp64")[0] is None
    with pytest.raises(Exception, match="box kernel"):
        M.set_variant("fp64", BOX, 1)
    ref3 = chains.apply_phi(csr.with_values(val3).to_scipy(), units, v)
    assert_close(host(pp.apply(poly, M, dev(v), "phi")), ref3, 1e-12, "phi after the stencil changed", dims)


def test_box_step_bytes(pp):
    # one step moves the interior row's coefficients, the input and the output
    csr = convdiff3d(20, 10, 10, 10)
    M = pp.Matrix.from_csr(csr)
    n = csr.n
    poly = pp.poly_from_roots(np.linspace(2.0, 9.0, 8), keep_order=True)
    for prec, sv in (("fp64", 8), ("fp32", 4)):
        M.set_variant(prec, BOX, 1)
        # 8 launches: each reads its input and 7 coefficients and writes its
        # output; the last also reads the final vector
        assert pp.chain_bytes(poly, M, "phi", prec) == (8 * (7 * sv + 2 * n * sv) + n * sv, 8)


# 7-point constant-coefficient boxes for whole-line tiles: lines of 64, 128
# and 256 points, y and z sides that leave partial tiles
TILE_CASES = {
    "box3d_64x10x7": ((64, 10, 7), (4.0, 2.0, 1.0)),
    "box3d_128x9x6": ((128, 9, 6), (10.0, 10.0, 10.0)),
    "box3d_256x5x3": ((256, 5, 3), (3.0, 1.0, 2.0)),
}


@pytest.mark.parametrize("name", list(TILE_CASES))
def test_box_tile_matches_oracle(pp, name):
    dims, coef = TILE_CASES[name]
    csr = _box_csr(dims, coef)
    A = csr.to_scipy()
    A32 = A.astype(np.float32)
    v = rhs(csr.n, 5)
    v32 = v.astype(np.float32)
    M = pp.Matrix.from_csr(csr)
    for pname, P, poly in _polys(pp, A, csr.n, 10):
        ref_phi = chains.apply_phi(A, P.units, v)
        for kind, fn in [("phi", chains.apply_phi), ("pi", chains.apply_pi), ("p", chains.apply_p)]:
            ref = fn(A, P.units, v)
            emu = (apply_p_low if kind == "p" else apply_phi_low)(A32, P.units, v32, "fp32")
            for prec in ("fp64", "fp32"):
                M.set_variant(prec, BOX, 1)
            single64 = host(pp.apply(poly, M, dev(v), kind))
            single32 = host(pp.apply(poly, M, dev(v32, torch.float32), kind))
            say("box tile", name, pname, kind)
            for prec in ("fp64", "fp32"):
                M.set_march_shape(1, prec)
                assert M.march_shape(prec) == 1 and M.march(prec)[0] == 2
            g64 = host(pp.apply(poly, M, dev(v), kind))
            g32 = host(pp.apply(poly, M, dev(v32, torch.float32), kind))
            assert_close(g64, ref, 1e-12, f"{name} {pname} {kind} tile fp64", dims)
            assert_close(g64, single64, 1e-14, f"{name} {pname} {kind} tile vs single launches", dims)
            for idx in (None, box_face_rows(*dims), tail_rows(csr.n)):
                delta = maxerr(emu, ref if kind == "p" else ref_phi, idx)
                err = maxerr(v32 - g32, ref_phi, idx) if kind == "pi" else maxerr(g32, ref, idx)
                assert err <= 10 * delta + 1e-6, (kind, err, delta)
                assert maxerr(g32, single32, idx) <= 10 * delta + 1e-6
            # launches: the chains fuse their steps two by two (p chains'
            # pairs carry the accumulator through the whole-line kernel too)
            by, launches = pp.chain_bytes(poly, M, kind, "fp64")
            assert launches < (poly.d_eff if kind != "p" else poly.d_eff - 1)
            assert M.pair_steps("fp64")[0]


def test_box_tile_refused_where_it_does_not_apply(pp):
    cases = {
        "lines of 20 points": convdiff3d(20, 1.0, 1.0, 1.0),
        "2-D": convdiff2d(64, 1.0),
        "variable coefficients": _varcoef(convdiff3d_box(64, 6, 5, 3.0, 2.0, 1.0)),
    }
    for what, csr in cases.items():
        say("box tile refused", what)
        M = pp.Matrix.from_csr(csr)
        M.tune("fp64")
        with pytest.raises(Exception, match="whole-line tiles"):
            M.set_march_shape(1, "fp64")
    M = pp.Matrix.from_csr(convdiff3d_box(64, 6, 5, 1.0, 1.0, 1.0))
    with pytest.raises(Exception, match="tune"):
        M.set_march_shape(1, "fp32")
    M.tune("bf16")
    with pytest.raises(Exception):
        M.set_march_shape(1, "bf16")
    # a forced variant and a hand-set marching count return to other kernels
    M.tune("fp32")
    M.set_march_shape(1, "fp32")
    M.set_march(2, "fp32")
    assert M.march_shape("fp32") == 0
    M.set_march_shape(1, "fp32")
    M.set_variant("fp32", BOX, 1)
    assert M.march_shape("fp32") == 0 and M.march("fp32")[0] == 0


def test_box_kernels_full_size(pp):
    # the benchmark's 128^3 workload: the tuned kernels, the box step and
    # whole-line tiles, element-wise against the oracle (FP64) and within the
    # emulated bound (FP32), on the box faces and the last block too
    csr = convdiff3d(128, 10, 10, 10)
    A = csr.to_scipy()
    P = oroots.setup(A, start_vector(csr.n, 2), 10)
    M = pp.Matrix.from_csr(csr)
    poly = pp.poly_from_roots(P.roots(), keep_order=True)
    v = rhs(csr.n, 5)
    v32 = v.astype(np.float32)
    box = (128, 128, 128)
    ref_phi = chains.apply_phi(A, P.units, v)
    ref_p = chains.apply_p(A, P.units, v)
    emu_phi = apply_phi_low(A.astype(np.float32), P.units, v32, "fp32")
    emu_p = apply_p_low(A.astype(np.float32), P.units, v32, "fp32")
    for setting in ("tuned", "box", "tile"):
        for prec in ("fp64", "fp32"):
            if setting == "tuned":
                M.tune(prec)
            else:
                M.set_variant(prec, BOX, 1)
                if setting == "tile":
                    M.set_march_shape(1, prec)
        say("box 128^3", setting, M.variant("fp32"), M.march("fp32"), M.march_shape("fp32"))
        assert_close(host(pp.apply(poly, M, dev(v), "phi")), ref_phi, 1e-12, f"128^3 phi {setting}", box)
        assert_close(host(pp.apply(poly, M, dev(v), "p")), ref_p, 1e-12, f"128^3 p {setting}", box)
        g_phi = host(pp.apply(poly, M, dev(v32, torch.float32), "phi"))
        g_p = host(pp.apply(poly, M, dev(v32, torch.float32), "p"))
        for idx in (None, box_face_rows(*box), tail_rows(csr.n)):
            assert maxerr(g_phi, ref_phi, idx) <= 10 * maxerr(emu_phi, ref_phi, idx) + 1e-6
            assert maxerr(g_p, ref_p, idx) <= 10 * maxerr(emu_p, ref_p, idx) + 1e-6
