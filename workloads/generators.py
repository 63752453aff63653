"""Seeded synthetic workloads for polynomial-preconditioned GMRES.

Matrices are returned in CSR form with int32 row pointers and column
indices (sorted ascending within each row) and float64 values. All random
draws use numpy's PCG64 ``default_rng(seed)``.

Operators
---------
* Convection-diffusion, section 3.2 (Example 5) of Loe & Morgan: the PDE
  -u_xx - u_yy + alpha u_x + beta u_y - gamma u on the unit square (and the
  7-point 3-D analogue), zero Dirichlet boundary, uniform grid with N
  interior points per side, h = 1/(N+1). Centred differences, every row
  multiplied by h^2: diagonal 2*dim - gamma h^2, the lower x-neighbour
  -1 - alpha h/2, the upper x-neighbour -1 + alpha h/2 (likewise for y and z).
  Rows are ordered lexicographically with x fastest. Every stencil entry is
  stored even when its coefficient is zero, so the sparsity pattern does
  not depend on the coefficients.
* Random nonsymmetric sparse: every row has 16 distinct off-diagonal
  columns drawn uniformly without replacement, N(0,1) values, and the
  diagonal 1.05 times the row's absolute off-diagonal sum.
* Diagonal matrices of Examples 7 and 11/12 of the paper.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """A square sparse matrix in CSR form (host arrays)."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    colind: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def with_values(self, val: np.ndarray) -> "CSR":
        return CSR(self.n, self.rowptr, self.colind, np.ascontiguousarray(val, dtype=np.float64))


def _csr_from_dense_slots(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray) -> tuple:
    """Pack an (n, k) slot table (columns ascending along axis 1) into CSR."""
    counts = mask.sum(axis=1)
    rowptr = np.zeros(cols.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    assert rowptr[-1] < 2**31
    return rowptr.astype(np.int32), colind, val


def _stencil(N: int, dim: int, coef, gamma: float, with_parts: bool = False):
    """Build the h^2-scaled centred-difference convection-diffusion matrix.

    coef: convection coefficient per axis (x, y[, z]).
    Returns (rowptr, colind, val) or, with with_parts, also the derivative of
    the values with respect to the x-convection coefficient.
    """
    h = 1.0 / (N + 1)
    half_h = 0.5 * h
    n = N**dim
    idx = np.arange(n, dtype=np.int64)
    coords = [(idx // (N**a)) % N for a in range(dim)]  # x fastest
    # slot order gives ascending columns: highest axis first (-), diag, then (+)
    slots = []
    for a in reversed(range(dim)):
        slots.append((a, -1))
    slots.append((None, 0))
    for a in range(dim):
        slots.append((a, +1))
    k = len(slots)
    cols = np.zeros((n, k), dtype=np.int64)
    vals = np.zeros((n, k), dtype=np.float64)
    dvals = np.zeros((n, k), dtype=np.float64)
    mask = np.zeros((n, k), dtype=bool)
    for s, (a, sgn) in enumerate(slots):
        if a is None:
            cols[:, s] = idx
            vals[:, s] = 2.0 * dim - gamma * h * h
            mask[:, s] = True
            continue
        stride = N**a
        ok = coords[a] > 0 if sgn < 0 else coords[a] < N - 1
        cols[:, s] = idx + sgn * stride
        off = coef[a] * half_h
        # lower neighbour: -1 - c h/2 ; upper neighbour: -1 + c h/2
        vals[:, s] = -1.0 - off if sgn < 0 else -1.0 + off
        if a == 0:
            dvals[:, s] = -half_h if sgn < 0 else half_h
        mask[:, s] = ok
    rowptr, colind, val = _csr_from_dense_slots(cols, vals, mask)
    if with_parts:
        dval = dvals[mask].astype(np.float64)
        return rowptr, colind, val, dval
    return rowptr, colind, val


def convdiff2d(N: int, alpha: float = 0.0, beta: float = 0.0, gamma: float = 0.0) -> CSR:
    """2-D convection-diffusion on an N x N interior grid (n = N^2)."""
    rowptr, colind, val = _stencil(N, 2, (float(alpha), float(beta)), float(gamma))
    return CSR(N * N, rowptr, colind, val)


def convdiff2d_parts(N: int, beta: float = 0.0, gamma: float = 0.0):
    """2-D convection-diffusion split as values(alpha) = base + alpha * dval.

    Returns (A0, dval): A0 is the matrix with no x-convection and dval the
    derivative of the values with respect to the x-convection coefficient
    alpha. base + alpha * dval is bit-identical to convdiff2d(N, alpha, ...)
    because the x-neighbour entries are -1 -/+ alpha*(h/2) both ways.
    """
    rowptr, colind, val, dval = _stencil(N, 2, (0.0, float(beta)), float(gamma), with_parts=True)
    return CSR(N * N, rowptr, colind, val), dval


def convdiff2d_colscaled(N: int, alpha: float = 0.0, decades: float = 3.0, seed: int = 9) -> CSR:
    """The 2-D convection-diffusion matrix with its columns scaled by
    10^u, u ~ U(-decades, decades) from the seed: a badly scaled system (unit
    variation of the diagonal over 2*decades orders of magnitude) for the
    composition with a diagonal preconditioner."""
    base = convdiff2d(N, alpha)
    s = 10.0 ** np.random.default_rng(seed).uniform(-decades, decades, size=base.n)
    return base.with_values(base.val * s[base.colind])


def convdiff2d_blockmixed(N: int, alpha: float = 0.0, bs: int = 4, decades: float = 2.0, seed: int = 11) -> CSR:
    """The 2-D convection-diffusion matrix times a block-diagonal matrix R on
    the right (blocks of bs consecutive columns, the last one shorter): each
    block is U diag(10^u) V with U, V random orthogonal (QR of N(0,1)
    draws) and u ~ U(-decades, decades), all from the seed. A badly mixed
    system for the composition with block-Jacobi; the stored pattern holds
    whole blocks of columns."""
    import scipy.sparse as sp

    base = convdiff2d(N, alpha).to_scipy()
    n = base.shape[0]
    rng = np.random.default_rng(seed)
    blocks = []
    for r0 in range(0, n, bs):
        m = min(bs, n - r0)
        U, _ = np.linalg.qr(rng.standard_normal((m, m)))
        V, _ = np.linalg.qr(rng.standard_normal((m, m)))
        blocks.append(U @ np.diag(10.0 ** rng.uniform(-decades, decades, m)) @ V)
    A = (base @ sp.block_diag(blocks, format="csr")).tocsr()
    A.sort_indices()
    return CSR(n=n, rowptr=A.indptr.astype(np.int32), colind=A.indices.astype(np.int32),
               val=A.data.astype(np.float64))


def convdiff3d(N: int, cx: float = 0.0, cy: float = 0.0, cz: float = 0.0, gamma: float = 0.0) -> CSR:
    """3-D convection-diffusion, 7-point stencil on an N^3 interior grid."""
    rowptr, colind, val = _stencil(N, 3, (float(cx), float(cy), float(cz)), float(gamma))
    return CSR(N**3, rowptr, colind, val)


def convdiff3d_box(nx: int, ny: int, nz: int, cx: float = 0.0, cy: float = 0.0, cz: float = 0.0) -> CSR:
    """3-D convection-diffusion on an nx x ny x nz interior grid (rows x
    fastest): the Kronecker sum of the 1-D operators tridiag(-1 - c h/2, 2,
    -1 + c h/2), h = 1/(m+1) per axis. A 7-point stencil on a box whose
    sides differ."""
    import scipy.sparse as sp

    def t1(m, c):
        h = 1.0 / (m + 1)
        e = np.ones(m)
        return sp.diags([(-1.0 - 0.5 * c * h) * e[1:], 2.0 * e, (-1.0 + 0.5 * c * h) * e[1:]], [-1, 0, 1],
                        format="csr")

    Ix, Iy, Iz = (sp.identity(m, format="csr") for m in (nx, ny, nz))
    A = (sp.kron(Iz, sp.kron(Iy, t1(nx, cx))) + sp.kron(Iz, sp.kron(t1(ny, cy), Ix)) +
         sp.kron(t1(nz, cz), sp.kron(Iy, Ix))).tocsr()
    A.sort_indices()
    return CSR(n=nx * ny * nz, rowptr=A.indptr.astype(np.int32), colind=A.indices.astype(np.int32),
               val=A.data.astype(np.float64))


def biharmonic2d(N: int = 200) -> CSR:
    """Example 3's matrix: -(u_xxxx + 2 u_xxyy + u_yyyy) + u_xxx on the unit
    square, N x N interior grid, h = 1/(N+1), u = 0 outside the grid (the
    stencil is cut at the boundary), scaled by h^4, rows lexicographic with
    x fastest. Centred differences: the 13-point biharmonic stencil and
    (-u_{i-2} + 2u_{i-1} - 2u_{i+1} + u_{i+2}) / (2h^3) for u_xxx.
    The mixed term is the reading that gives the paper's 13 nonzeros per row
    and its condition number 8.2e7 at N = 200 (the printed equation shows
    only u_xxxx and u_yyyy)."""
    import scipy.sparse as sp

    h = 1.0 / (N + 1)
    e = np.ones(N)
    I = sp.identity(N, format="csr")
    D4 = sp.diags([e[2:], -4 * e[1:], 6 * e, -4 * e[1:], e[2:]], [-2, -1, 0, 1, 2], format="csr")
    D2 = sp.diags([e[1:], -2 * e, e[1:]], [-1, 0, 1], format="csr")
    D3 = sp.diags([-e[2:], 2 * e[1:], -2 * e[1:], e[2:]], [-2, -1, 1, 2], format="csr") * 0.5
    A = (-(sp.kron(I, D4) + sp.kron(D4, I) + 2.0 * sp.kron(D2, D2)) + h * sp.kron(I, D3)).tocsr()
    A.sort_indices()
    return CSR(n=N * N, rowptr=A.indptr.astype(np.int32), colind=A.indices.astype(np.int32),
               val=A.data.astype(np.float64))


def randsparse(n: int, k: int = 16, seed: int = 7, dominance: float = 1.05) -> CSR:
    """Random nonsymmetric sparse matrix with k off-diagonals per row.

    Columns: k distinct values in [0, n) excluding the row index, uniform
    without replacement (rows with a repeated draw are redrawn). Values
    N(0,1). Diagonal: dominance * sum_j |a_ij|.
    """
    rng = np.random.default_rng(seed)
    rows = np.arange(n, dtype=np.int64)[:, None]
    cols = rng.integers(0, n - 1, size=(n, k), dtype=np.int64)
    cols += cols >= rows  # skip the diagonal
    cols.sort(axis=1)
    while True:
        dup = np.any(cols[:, 1:] == cols[:, :-1], axis=1)
        nd = int(dup.sum())
        if nd == 0:
            break
        redo = rng.integers(0, n - 1, size=(nd, k), dtype=np.int64)
        r = rows[dup]
        redo += redo >= r
        redo.sort(axis=1)
        cols[dup] = redo
    offv = rng.standard_normal((n, k))
    diag = dominance * np.abs(offv).sum(axis=1)
    allc = np.concatenate([cols, rows], axis=1)
    allv = np.concatenate([offv, diag[:, None]], axis=1)
    order = np.argsort(allc, axis=1, kind="stable")
    allc = np.take_along_axis(allc, order, axis=1)
    allv = np.take_along_axis(allv, order, axis=1)
    rowptr = (np.arange(n + 1, dtype=np.int64) * (k + 1)).astype(np.int32)
    return CSR(n, rowptr, allc.reshape(-1).astype(np.int32), allv.reshape(-1).astype(np.float64))


def diagonal(values) -> CSR:
    """Diagonal matrix with the given entries."""
    v = np.asarray(values, dtype=np.float64)
    n = v.size
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), v.copy())


def diag_example7() -> CSR:
    """Example 7: entries 0.01..0.1 (step 0.01), 30, 60, 100, 101, ..., 5087; n = 5000."""
    small = np.arange(1, 11, dtype=np.float64) / 100.0
    big = np.arange(100, 5088, dtype=np.float64)
    return diagonal(np.concatenate([small, [30.0, 60.0], big]))


def diag_squares(n: int) -> CSR:
    """Examples 11 and 12: entries i^2/n for i = 1..n."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return diagonal(i * i / n)


def diag_clusters() -> CSR:
    """Eigenvalues in bunches well separated from the rest (the situation the
    stability discussion of section 3 describes): 1000 values evenly in
    [1, 2], then 300, 300.3, 300.6, 700, 701 and 1500; n = 1006."""
    return diagonal(np.concatenate([np.linspace(1.0, 2.0, 1000), [300.0, 300.3, 300.6, 700.0, 701.0, 1500.0]]))


def diag_wide() -> CSR:
    """A wide positive spectrum: 1000 values evenly in [0.01, 1], then 20
    values geometrically from 10 to 1e5; n = 1020."""
    return diagonal(np.concatenate([np.linspace(0.01, 1.0, 1000), np.geomspace(10.0, 1e5, 20)]))


def normal_vector(n: int, seed: int, count: int | None = None) -> np.ndarray:
    """N(0,1) draws of length n (or shape (count, n))."""
    rng = np.random.default_rng(seed)
    if count is None:
        return rng.standard_normal(n)
    return rng.standard_normal((count, n))


def rhs(n: int, seed: int = 1, count: int | None = None) -> np.ndarray:
    """Right-hand side(s): N(0,1) draws, each normalised to unit 2-norm."""
    b = normal_vector(n, seed, count)
    if count is None:
        return b / np.linalg.norm(b)
    return b / np.linalg.norm(b, axis=1, keepdims=True)


def start_vector(n: int, seed: int = 2) -> np.ndarray:
    """Random start vector for the polynomial's GMRES(d) run (not normalised)."""
    return normal_vector(n, seed)


def batched_convdiff_specs(count: int = 256, seed: int = 11, side_lo: int = 64, side_hi: int = 512,
                           coef_hi: float = 50.0):
    """Sizes and convection coefficients of the batched 2-D workload.

    Returns a list of (N, alpha, rhs_seed, start_seed) with N uniform in
    [side_lo, side_hi] and alpha uniform in [0, coef_hi).
    """
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=count)
    alphas = rng.uniform(0.0, coef_hi, size=count)
    return [(int(sides[i]), float(alphas[i]), 1000 + i, 5000 + i) for i in range(count)]
