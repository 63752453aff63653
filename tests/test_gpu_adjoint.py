"""GPU parity of the adjoint (transposed chain with the same roots) and its gradients."""

import numpy as np
import pytest
import scipy.sparse.linalg as sla
import torch

from oracle.adjoint import grad_direct
from workloads import convdiff2d, convdiff2d_parts, randsparse, rhs, start_vector
from gpu_util import say, dev, host, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import paper_1911_07065_amd.api as api

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return api


@pytest.mark.parametrize("maker", ["convdiff", "random"])
def test_transpose_pattern_exact(pp, maker):
    csr = convdiff2d(40, 20.0) if maker == "convdiff" else randsparse(3000, 16, seed=7)
    say("transpose", maker)
    M = pp.Matrix.from_csr(csr)
    At = M.transpose()
    ref = csr.to_scipy().T.tocsr()
    ref.sort_indices()
    assert np.array_equal(host(At.rowptr).astype(np.int64), ref.indptr)
    assert np.array_equal(host(At.colind).astype(np.int64), ref.indices)
    assert np.array_equal(host(At.val), ref.data)
    # <A^T u, v> = <u, A v> through the library's own products
    poly = pp.poly_from_roots([1.0])  # phi(z) = z: one sparse product
    u = dev(rhs(csr.n, 3))
    v = dev(rhs(csr.n, 4))
    Atu = pp.apply(poly, At, u, "phi")
    Av = pp.apply(poly, M, v, "phi")
    assert abs(float(Atu @ v) - float(u @ Av)) <= 1e-12 * float(torch.linalg.norm(Atu) * torch.linalg.norm(v))


def _problem(N, theta):
    A0, dval = convdiff2d_parts(N)
    n = N * N
    b = rhs(n, 1)
    xt = np.random.default_rng(3).standard_normal(n)
    return A0, dval, b, xt


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_gradient_vs_oracle_and_finite_differences(pp, inner):
    N, theta0 = 48, 20.0
    A0, dval, b, xt = _problem(N, theta0)
    say("adjoint", N, inner)
    M = pp.Matrix.from_csr(A0)
    base = dev(A0.val)
    dirv = dev(dval)
    th = torch.tensor(theta0, dtype=torch.float64, device="cuda", requires_grad=True)
    bt = dev(b).requires_grad_(True)
    vals0 = (base + th.detach() * dirv)
    M.set_values(vals0)
    poly = pp.setup(M, dev(start_vector(A0.n, 2)), 30)
    opts = dict(tol=1e-12, m=50, inner=inner)
    vals = base + th * dirv
    x = pp.pp_solve_fn(vals, bt, M, poly, **opts)
    loss = 0.5 * torch.sum((x - dev(xt)) ** 2)
    loss.backward()
    g_theta = float(th.grad)
    g_b = host(bt.grad)
    # oracle: direct solves for x and lambda
    A = A0.with_values(A0.val + theta0 * dval).to_scipy()
    xo, lam, dv = grad_direct(A, b, lambda x: x - xt)
    g_or = float(dv @ dval)
    assert abs(g_theta - g_or) <= 1e-6 * abs(g_or), (g_theta, g_or)
    assert relerr(g_b, lam) <= 1e-6

    def L(t):
        At = A0.with_values(A0.val + t * dval).to_scipy()
        xs = sla.spsolve(At.tocsc(), b)
        return 0.5 * np.sum((xs - xt) ** 2)

    h = 1e-6
    fd = (L(theta0 + h) - L(theta0 - h)) / (2 * h)
    assert abs(g_theta - fd) <= 1e-6 * abs(fd), (g_theta, fd)


def test_differentiation_config_full_size(pp):
    # 2-D convection-diffusion on a 1024 x 1024 grid (n = 1,048,576), convection
    # coefficient theta = 20 as a leaf tensor, loss 0.5 ||x(theta, b) - x_t||^2,
    # degree 50; adjoint through the same roots vs the direct-solve gradient
    # and central finite differences with h = 1e-6 (direct solves).
    import time

    N, theta0 = 1024, 20.0
    A0, dval = convdiff2d_parts(N)
    n = N * N
    b = rhs(n, 1)
    xt = np.random.default_rng(3).standard_normal(n)
    say("differentiation full size", n)
    M = pp.Matrix.from_csr(A0)
    base, dirv = dev(A0.val), dev(dval)
    M.set_values(base + theta0 * dirv)
    poly = pp.setup(M, dev(start_vector(n, 2)), 50)
    th = torch.tensor(theta0, dtype=torch.float64, device="cuda", requires_grad=True)
    bt = dev(b).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = pp.pp_solve_fn(base + th * dirv, bt, M, poly, tol=1e-12, m=50, inner="fp64")
    loss = 0.5 * torch.sum((x - dev(xt)) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    g_theta = float(th.grad)
    g_b = host(bt.grad)
    lu_of = lambda t: sla.splu(A0.with_values(A0.val + t * dval).to_scipy().tocsc(), permc_spec="COLAMD")
    lu = lu_of(theta0)
    xo = lu.solve(b)
    lam = lu.solve(xo - xt, trans="T")
    A = A0.with_values(A0.val + theta0 * dval).to_scipy()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    g_or = float(np.dot(-lam[rows] * xo[A.indices], dval))
    # central difference (L(theta+h) - L(theta-h)) / 2h, h = 1e-6, evaluated
    # without cancellation: with D = dA/dtheta, x+ - x- = -2h A(theta+h)^{-1} D x-
    # exactly, and L+ - L- = (x+ - x-)^T (x+ + x- - 2 x_t) / 2 (L ~ 5e5 here,
    # so subtracting the two losses would lose ~1e-6 to rounding)
    h = 1e-6
    D = A0.with_values(dval).to_scipy()
    xm = lu_of(theta0 - h).solve(b)
    dx = -2 * h * lu_of(theta0 + h).solve(D @ xm)
    xp = xm + dx
    fd = float(dx @ (xp + xm - 2 * xt)) / (4 * h)
    say("dL/dtheta gpu", g_theta, "oracle", g_or, "fd", fd, "gpu fwd+bwd s", round(t_gpu, 3),
        "rel x err", relerr(host(x), xo))
    assert abs(g_theta - g_or) <= 1e-6 * abs(g_or)
    assert abs(g_theta - fd) <= 1e-6 * abs(fd)
    assert relerr(g_b, lam) <= 1e-6
