"""Pins of the seeded input generators (closed forms, no solver code)."""

import numpy as np
import pytest

from workloads import convdiff2d, convdiff2d_parts, convdiff3d, randsparse, diag_example7, rhs


@pytest.mark.parametrize("N,expect", [(50, 12300), (1024, 5238784)])
def test_convdiff2d_nnz(N, expect):
    # 5-point stencil: 5 n - 4 N stored entries (the 1024^2 count is the
    # differentiation workload's, from the generator itself)
    A = convdiff2d(N, 1.0)
    assert A.nnz == expect == 5 * N * N - 4 * N
    assert A.n == N * N and A.rowptr[-1] == A.nnz


@pytest.mark.parametrize("N,expect", [(12, 7 * 12**3 - 6 * 12**2), (128, 14581760)])
def test_convdiff3d_nnz(N, expect):
    # 7-point stencil: 7 n - 6 N^2 stored entries, at the headline 128^3 size too
    A = convdiff3d(N, 10, 10, 10)
    assert A.nnz == expect
    assert A.n == N**3 and A.rowptr[-1] == A.nnz


@pytest.mark.parametrize("c", [0.0, 0.3, 0.9])
def test_convdiff2d_eigenvalues_closed_form(c):
    # tridiag(-1-c, 2, -1+c) has eigenvalues 2 - 2 sqrt(1-c^2) cos(k pi h);
    # the 2-D operator is the Kronecker sum of the x and y parts.
    N = 9
    h = 1.0 / (N + 1)
    alpha = 2.0 * c / h  # alpha h / 2 = c
    A = convdiff2d(N, alpha).to_scipy().toarray()
    k = np.arange(1, N + 1)
    ex = 2 - 2 * np.sqrt(1 - c * c) * np.cos(k * np.pi * h)
    ey = 2 - 2 * np.cos(k * np.pi * h)
    expect = np.sort((ex[:, None] + ey[None, :]).ravel())
    got = np.sort(np.linalg.eigvals(A).real)
    # nonsymmetric eigenvalues: dense eigensolver accuracy ~ 1e-11 at c = 0.9
    assert np.max(np.abs(got - expect)) < 1e-10


def test_convdiff3d_eigenvalues_closed_form():
    N = 5
    h = 1.0 / (N + 1)
    c = 0.4
    A = convdiff3d(N, 2 * c / h, 0, 0).to_scipy().toarray()
    k = np.arange(1, N + 1)
    ex = 2 - 2 * np.sqrt(1 - c * c) * np.cos(k * np.pi * h)
    e = 2 - 2 * np.cos(k * np.pi * h)
    expect = np.sort((ex[:, None, None] + e[None, :, None] + e[None, None, :]).ravel())
    got = np.sort(np.linalg.eigvals(A).real)
    assert np.max(np.abs(got - expect)) < 1e-10


def test_convdiff_condition_number_example5():
    # Example 5: the symmetric 200 x 200 problem has condition number 1.6e4
    h = 1.0 / 201
    lam_min = 4 - 4 * np.cos(np.pi * h)
    lam_max = 4 + 4 * np.cos(np.pi * h)
    assert abs(lam_max / lam_min - 1.6e4) / 1.6e4 < 0.03


def test_convdiff2d_parts_exact():
    A0, dval = convdiff2d_parts(30)
    for a in [0.0, 1.0, 20.0, 37.5]:
        assert np.array_equal(A0.val + a * dval, convdiff2d(30, a).val)


def test_randsparse_structure():
    A = randsparse(5000, 16, seed=7)
    assert A.nnz == 17 * 5000
    rp, ci, v = A.rowptr, A.colind, A.val
    for i in range(0, 5000, 97):
        cols = ci[rp[i]:rp[i + 1]]
        vals = v[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        assert i in cols
        d = vals[cols == i][0]
        off = np.abs(vals[cols != i]).sum()
        assert abs(d - 1.05 * off) <= 1e-12 * d


def test_randsparse_deterministic():
    a = randsparse(2000, seed=7)
    b = randsparse(2000, seed=7)
    assert np.array_equal(a.colind, b.colind) and np.array_equal(a.val, b.val)


def test_example7_diagonal():
    A = diag_example7()
    assert A.n == 5000
    assert A.val[9] == 0.1 and A.val[10] == 30 and A.val[11] == 60 and A.val[-1] == 5087


def test_rhs_normalised():
    b = rhs(1000, 1)
    assert abs(np.linalg.norm(b) - 1) < 1e-14


def test_convdiff3d_box_cube_and_structure():
    from workloads import convdiff3d_box

    # on a cube the Kronecker-sum construction is the 7-point stencil itself
    for N, c in ((6, (10.0, 10.0, 10.0)), (9, (0.0, 3.0, -2.0))):
        a = convdiff3d_box(N, N, N, *c).to_scipy()
        b = convdiff3d(N, *c).to_scipy()
        assert abs(a - b).max() == 0.0
    # a box with unequal sides: x fastest, diagonals 0, +-1, +-nx, +-nx ny, and
    # no entry joining the end of a grid line (or plane) to the start of the next
    nx, ny, nz = 7, 5, 4
    A = convdiff3d_box(nx, ny, nz, 1.0, 2.0, 3.0).to_scipy().tocoo()
    off = A.col - A.row
    assert set(np.unique(off)) == {0, 1, -1, nx, -nx, nx * ny, -nx * ny}
    x, y = A.row % nx, (A.row // nx) % ny
    assert not np.any((off == 1) & (x == nx - 1)) and not np.any((off == -1) & (x == 0))
    assert not np.any((off == nx) & (y == ny - 1)) and not np.any((off == -nx) & (y == 0))
    assert A.nnz == 7 * nx * ny * nz - 2 * (ny * nz + nx * nz + nx * ny)
