"""pp_apply_noalloc (the allocation-free variant of pp_apply) through the C
ABI: its output equals pp_apply's bit for bit (same kernels, same variant),
on two calls in a row, the second with a smaller input, for every kind and
precision; sizes beyond its scratch and untuned precisions are rejected."""

import ctypes

import numpy as np
import pytest
import torch

from oracle import chains, roots as oroots
from workloads import convdiff2d, convdiff3d, rhs, start_vector
from gpu_util import say, dev, host, assert_close

pytestmark = pytest.mark.gpu

KINDS = {"p": 0, "phi": 1, "pi": 2}
PRECS = {"fp64": (0, torch.float64), "fp32": (1, torch.float32), "bf16": (2, torch.bfloat16)}


@pytest.fixture(scope="module")
def pp():
    import paper_1911_07065_amd.api as api

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return api


def _noalloc(lib, poly, M, kind, prec, v, y):
    return lib.pp_apply_noalloc(poly.handle, M.handle, KINDS[kind], PRECS[prec][0], ctypes.c_void_p(v.data_ptr()),
                                ctypes.c_void_p(y.data_ptr()), None)


def test_noalloc_apply_equals_apply_twice_then_smaller(pp):
    from paper_1911_07065_amd._lib import lib

    # first call on the 128^3 matrix (n = 2^21, the FP64 limit of the
    # scratch), then on a smaller 2-D one, so the second call runs on a
    # scratch that still holds the first call's larger vectors
    cases = [("convdiff3d_128", convdiff3d(128, 10, 10, 10)), ("convdiff2d_77", convdiff2d(77, 4.0))]
    th = np.array([11.5, 0.3, 6 + 2j, 6 - 2j, 2.0, 9.0, 4.0 + 0.5j, 4.0 - 0.5j, 0.9, 7.2])
    P = oroots.poly_from_roots(th)
    for name, csr in cases:
        A = csr.to_scipy()
        M = pp.Matrix.from_csr(csr)
        poly = pp.poly_from_roots(P.roots(), keep_order=True)
        v = rhs(csr.n, 3)
        for prec, (_, dt) in PRECS.items():
            M.tune(prec)
            vd = dev(v, dt)
            for kind in KINDS:
                say("noalloc", name, prec, kind)
                ref = pp.apply(poly, M, vd, kind)
                y = torch.full_like(vd, float("nan"))
                st = _noalloc(lib, poly, M, kind, prec, vd, y)
                torch.cuda.synchronize()
                assert st == 0, lib.pp_last_error()
                assert torch.equal(y, ref), (name, prec, kind)
            if prec == "fp64":
                # and against the oracle (element by element)
                y = torch.empty_like(vd)
                assert _noalloc(lib, poly, M, "p", prec, vd, y) == 0
                assert_close(host(y), chains.apply_p(A, P.units, v), 1e-12, f"{name} p vs oracle")


def test_noalloc_rejects_what_it_cannot_hold(pp):
    from paper_1911_07065_amd._lib import lib

    csr = convdiff2d(30, 1.0)
    M = pp.Matrix.from_csr(csr)
    poly = pp.poly_from_roots([2.0, 5.0])
    v = dev(rhs(csr.n, 1))
    y = torch.empty_like(v)
    say("noalloc rejections")
    # precision not tuned yet
    assert _noalloc(lib, poly, M, "phi", "fp64", v, y) == -1
    assert b"tune" in lib.pp_last_error()
    M.tune("fp64")
    assert _noalloc(lib, poly, M, "phi", "fp64", v, y) == 0
    # aliasing and a double polynomial
    assert _noalloc(lib, poly, M, "phi", "fp64", v, v) == -1
    p1 = pp.setup(M, dev(start_vector(csr.n, 2)), 4)
    p2 = pp.setup_double(M, p1, dev(start_vector(csr.n, 2)), 3)
    assert _noalloc(lib, p2, M, "phi", "fp64", v, y) == -1
    # FP64 vectors above 2^21 rows exceed the scratch: rejected before any launch
    big = convdiff3d(129, 1, 1, 1)  # 2,146,689 rows
    Mb = pp.Matrix.from_csr(big)
    Mb.set_variant("fp64", 0, 1)
    vb = torch.zeros(big.n, dtype=torch.float64, device="cuda")
    yb = torch.empty_like(vb)
    assert _noalloc(lib, poly, Mb, "phi", "fp64", vb, yb) == -1
    assert b"scratch" in lib.pp_last_error()
    # the same rows fit in FP32
    Mb.set_variant("fp32", 0, 1)
    vb32 = vb.float()
    yb32 = torch.empty_like(vb32)
    assert _noalloc(lib, poly, Mb, "phi", "fp32", vb32, yb32) == 0
    torch.cuda.synchronize()
    assert torch.equal(yb32, torch.zeros_like(yb32))
