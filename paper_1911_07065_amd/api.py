"""Python front of libppgmres: argument marshalling between torch tensors and the C ABI.

Every numerical step runs in the library (HIP kernels on the GPU, C++ for
the small host-side problems). Tensors passed to the device entry points
must live on a ROCm device; nothing here computes a result on the CPU.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import PPError, SetupInfo, SolveInfo, SolveOpts, StchOpts, check, lib, PP_BREAKDOWN, PP_NOCONV, PP_UNSTABLE, STATUS_NAMES

PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
DTYPE_OF_PREC = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}
PREC_OF_DTYPE = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}
KIND = {"p": 0, "phi": 1, "pi": 2}


def version() -> str:
    return lib.pp_version().decode()


N_CHAIN_VARIANTS = 34


def chain_variant_name(v: int) -> str:
    return lib.pp_chain_variant_name(int(v)).decode()


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _dev_tensor(x, dtype, device):
    t = torch.as_tensor(x, dtype=dtype, device=device)
    if t.device.type != "cuda":
        raise ValueError("device tensors are required")
    return t.contiguous()


class Matrix:
    """A square CSR matrix on the GPU (int32 indices, float64 values).

    The tensors are kept alive by this object; the library borrows them.
    """

    def __init__(self, rowptr, colind, val, device="cuda"):
        self.rowptr = _dev_tensor(rowptr, torch.int32, device)
        self.colind = _dev_tensor(colind, torch.int32, device)
        self.val = _dev_tensor(val, torch.float64, device)
        self.n = int(self.rowptr.numel() - 1)
        self.nnz = int(self.colind.numel())
        self.device = self.val.device
        h = ctypes.c_void_p()
        check(lib.pp_matrix_create(self.n, self.nnz, _ptr(self.rowptr), _ptr(self.colind), _ptr(self.val),
                                   _stream(self.device), ctypes.byref(h)), "pp_matrix_create")
        self.handle = h
        self._t = None
        self.scaling = None  # right scaling: None, "jacobi" or "custom"

    @classmethod
    def from_csr(cls, csr, device="cuda"):
        """From any object with rowptr/colind/val host arrays (e.g. workloads.CSR)."""
        return cls(csr.rowptr, csr.colind, csr.val, device=device)

    def set_values(self, val):
        val = _dev_tensor(val, torch.float64, self.device)
        if val.numel() != self.nnz:
            raise ValueError("value count does not match the pattern")
        self.val = val
        # a cached transpose (PPSolve.backward) keeps its pattern and tuning:
        # backward gathers the new values into it
        try:
            check(lib.pp_matrix_set_values(self.handle, _ptr(val), _stream(self.device)), "pp_matrix_set_values")
        except PPError:
            self.scaling = None  # a failed Jacobi scaling leaves the handle unscaled
            raise

    def right_scale(self, s=None):
        """Compose with the diagonal right preconditioner M^{-1} = diag(s) (eqs.
        1.3-1.4): the operator becomes A diag(s), polynomials built on this
        Matrix are polynomials in A M^{-1}, and solve() returns the solution of
        A x = b. s=None is Jacobi (s_i = 1/a_ii, recomputed by set_values)."""
        if s is not None:
            s = _dev_tensor(s, torch.float64, self.device)
            if s.numel() != self.n:
                raise ValueError("scaling length")
        self._t = None
        try:
            check(lib.pp_matrix_right_scale(self.handle, _ptr(s) if s is not None else None, _stream(self.device)),
                  "pp_matrix_right_scale")
        except PPError:
            self.scaling = None  # the handle reverts to the unscaled matrix
            raise
        self.scaling = "jacobi" if s is None else "custom"

    def block_jacobi(self, bs: int) -> "Matrix":
        """Compose with block-Jacobi (eqs. 1.3-1.4): M is the block diagonal of
        this matrix's current values in blocks of bs consecutive rows. Returns
        a new Matrix for B = A M^{-1}; polynomials built on it are polynomials
        in A M^{-1}, and solve() on it returns the solution of A x = b. The
        blocks of M^{-1} are in `.minv` (block k row-major at k*bs*bs)."""
        bs = int(bs)
        st = _stream(self.device)
        nnz_b = ctypes.c_int64()
        check(lib.pp_block_jacobi_nnz(self.handle, bs, st, ctypes.byref(nnz_b)), "pp_block_jacobi_nnz")
        nb = (self.n + bs - 1) // bs
        rp = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(max(nnz_b.value, 1), dtype=torch.int32, device=self.device)
        va = torch.empty(max(nnz_b.value, 1), dtype=torch.float64, device=self.device)
        mi = torch.empty(nb * bs * bs, dtype=torch.float64, device=self.device)
        check(lib.pp_block_jacobi(self.handle, bs, _ptr(rp), _ptr(ci), _ptr(va), _ptr(mi), st), "pp_block_jacobi")
        B = Matrix(rp, ci[: nnz_b.value], va[: nnz_b.value], device=self.device)
        check(lib.pp_matrix_right_blocks(B.handle, bs, _ptr(mi), st), "pp_matrix_right_blocks")
        B.minv, B.block_size = mi, bs
        return B

    def scale(self) -> torch.Tensor:
        """The right scaling s of a scaled Matrix."""
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        check(lib.pp_matrix_scale(self.handle, _ptr(out), _stream(self.device)), "pp_matrix_scale")
        return out

    def tune(self, prec: str = "fp32"):
        """Autotune the chain kernel for one precision; returns (variant name, remap, us per launch)."""
        v, r, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        check(lib.pp_matrix_tune(self.handle, PREC[prec], _stream(self.device), ctypes.byref(v), ctypes.byref(r),
                                 ctypes.byref(us)), "pp_matrix_tune")
        return lib.pp_chain_variant_name(v.value).decode(), r.value, us.value

    def variant(self, prec: str = "fp32"):
        """Chain variant in use for a precision without tuning: (name or None, remap, tuned us per launch)."""
        v, r, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        check(lib.pp_matrix_variant(self.handle, PREC[prec], ctypes.byref(v), ctypes.byref(r), ctypes.byref(us)),
              "pp_matrix_variant")
        name = None if v.value < 0 else lib.pp_chain_variant_name(v.value).decode()
        return name, r.value, us.value

    def set_pair_steps(self, on: bool, prec: str = "fp32"):
        """Run two real-root chain steps per launch (box stencils only), or not."""
        check(lib.pp_matrix_set_pair_steps(self.handle, PREC[prec], 1 if on else 0), "pp_matrix_set_pair_steps")

    def pair_steps(self, prec: str = "fp32"):
        """(in use, box dims or None, tuned us per two-step launch)."""
        mode, us = ctypes.c_int(), ctypes.c_double()
        box = (ctypes.c_int * 3)()
        check(lib.pp_matrix_pair_steps(self.handle, PREC[prec], ctypes.byref(mode), box, ctypes.byref(us)),
              "pp_matrix_pair_steps")
        dims = tuple(box) if box[0] else None
        return bool(mode.value), dims, us.value

    def set_march(self, steps: int, prec: str = "fp32", cz: int = 0, depth: int = 0):
        """Up to `steps` (2..4) chain steps per launch of the marching kernel
        on a box stencil (0: off); cz planes per chunk (0: default); depth
        planes of loads in flight per workgroup (0: 1)."""
        check(lib.pp_matrix_set_march(self.handle, PREC[prec], int(steps), int(cz), int(depth)),
              "pp_matrix_set_march")

    def march(self, prec: str = "fp32"):
        """(steps, cz, us per launch) of the marching kernel in use (steps 0: off)."""
        g, cz, us, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        check(lib.pp_matrix_march(self.handle, PREC[prec], ctypes.byref(g), ctypes.byref(cz), ctypes.byref(us),
                                  ctypes.byref(c)), "pp_matrix_march")
        return g.value, cz.value, us.value

    def set_march_shape(self, shape: int, prec: str = "fp32"):
        """Two-step launches on whole grid lines (shape 1) or marching planes (0)."""
        check(lib.pp_matrix_set_march_shape(self.handle, PREC[prec], int(shape)), "pp_matrix_set_march_shape")

    def march_shape(self, prec: str = "fp32") -> int:
        """1 while two-step launches run on whole grid lines, else 0."""
        v = ctypes.c_int()
        check(lib.pp_matrix_march_shape(self.handle, PREC[prec], ctypes.byref(v)), "pp_matrix_march_shape")
        return v.value

    def constant_stencil(self) -> bool:
        """True when every row is one interior row's box stencil truncated at the box."""
        g, c = ctypes.c_int(), ctypes.c_int()
        check(lib.pp_matrix_march(self.handle, 0, ctypes.byref(g), None, None, ctypes.byref(c)), "pp_matrix_march")
        return bool(c.value)

    def set_variant(self, prec: str, variant: int, remap: int = 1):
        """Force chain variant `variant` (0..30; 15 = persistent cooperative kernel) for a precision."""
        check(lib.pp_matrix_set_variant(self.handle, PREC[prec], int(variant), int(remap)), "pp_matrix_set_variant")

    def transpose_pattern(self):
        """(rowptr_t, colind_t, perm) of A^T with val_t = val[perm]."""
        rp = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        pm = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        check(lib.pp_matrix_transpose(self.handle, _ptr(rp), _ptr(ci), _ptr(pm), _stream(self.device)),
              "pp_matrix_transpose")
        return rp, ci[: self.nnz], pm[: self.nnz]

    def transpose(self) -> "Matrix":
        """A^T as a new Matrix (pattern built once, values gathered on the GPU)."""
        rp, ci, pm = self.transpose_pattern()
        vt = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        check(lib.pp_gather(self.nnz, _ptr(self.val), _ptr(pm), _ptr(vt), _stream(self.device)), "pp_gather")
        At = Matrix(rp, ci, vt, device=self.device)
        At.perm = pm
        if getattr(self, "scaling", None) == "jacobi":
            At.right_scale(None)  # diag(A^T) = diag(A)
        return At

    def adjoint_values(self, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        """dval[k] = -lam[row k] * x[col k]."""
        out = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        check(lib.pp_adjoint_values(self.handle, _ptr(lam.contiguous()), _ptr(x.contiguous()), _ptr(out),
                                    _stream(self.device)), "pp_adjoint_values")
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is None or not h.value or lib is None:
            return
        try:
            torch.cuda.synchronize(self.device)
            lib.pp_matrix_destroy(h)
        except Exception:  # interpreter shutdown
            pass
        self.handle = None


@dataclass
class Poly:
    """Handle of a preconditioning polynomial (library-owned root list)."""

    handle: ctypes.c_void_p
    d: int
    d_eff: int
    n_added: int
    breakdown: bool = False
    setup_info: dict | None = None
    stch: float | None = None  # stability check value (setup_checked only)
    composite_degree: int | None = None  # double polynomials: degree of phi2(phi1(z))
    unstable: bool = False     # setup_checked: no degree tried passed the check

    def roots(self, which: str = "final") -> np.ndarray:
        """Root list: "final" (applied order, with added roots), "theta" (raw
        harmonic Ritz values), "leja" (original roots in Leja order) or, for a
        double polynomial, "inner" (the final roots of phi1)."""
        w = {"final": 0, "theta": 1, "leja": 2, "inner": 3}[which]
        ln = ctypes.c_int()
        check(lib.pp_poly_roots(self.handle, w, 0, None, None, ctypes.byref(ln), None, None), "pp_poly_roots")
        re = np.zeros(ln.value)
        im = np.zeros(ln.value)
        check(lib.pp_poly_roots(self.handle, w, ln.value, re.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                im.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(ln), None, None),
              "pp_poly_roots")
        return re + 1j * im

    def units(self):
        """(kind, re, im) units of the final root list (kind 1 = conjugate pair)."""
        r = self.roots()
        out, i = [], 0
        while i < r.size:
            if r[i].imag == 0:
                out.append((0, float(r[i].real), 0.0))
                i += 1
            else:
                out.append((1, float(r[i].real), float(r[i].imag)))
                i += 2
        return out

    def __del__(self):
        if self.handle is None or not self.handle.value or lib is None:
            return
        try:
            lib.pp_poly_destroy(self.handle)
        except Exception:  # interpreter shutdown
            pass
        self.handle = None


def _poly_from_handle(h, setup_info=None, breakdown=False) -> Poly:
    de, do, na = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib.pp_poly_roots(h, 0, 0, None, None, ctypes.byref(de), ctypes.byref(do), ctypes.byref(na)),
          "pp_poly_roots")
    return Poly(h, do.value, de.value, na.value, breakdown, setup_info)


def setup(A: Matrix, v0, d: int, add_roots: bool = True, basis: str = "fp64") -> Poly:
    """Polynomial of degree d from one GMRES(d) cycle on A started at v0
    (Algorithm 4 step 1). basis: "fp64", or "fp32" to store the cycle's
    Krylov vectors in binary32 (FP64 dot products and Hessenberg)."""
    v0 = _dev_tensor(v0, torch.float64, A.device)
    if v0.numel() != A.n:
        raise ValueError("start vector length")
    h = ctypes.c_void_p()
    info = SetupInfo()
    if basis == "fp64":
        st = check(lib.pp_gmres_setup(A.handle, _ptr(v0), int(d), int(bool(add_roots)), _stream(A.device),
                                      ctypes.byref(h), ctypes.byref(info)), "pp_gmres_setup")
    elif basis == "fp32":
        st = check(lib.pp_gmres_setup_basis(A.handle, _ptr(v0), int(d), int(bool(add_roots)), PREC["fp32"],
                                            _stream(A.device), ctypes.byref(h), ctypes.byref(info)),
                   "pp_gmres_setup_basis")
    else:
        raise ValueError("basis must be 'fp64' or 'fp32'")
    si = {k: getattr(info, k) for k, _ in SetupInfo._fields_}
    return _poly_from_handle(h, si, breakdown=(st == PP_BREAKDOWN) or bool(info.breakdown))


def setup_double(A: Matrix, p1: Poly, v0, d2: int, add_roots: bool = True) -> Poly:
    """Double polynomial (section 6): phi2 from GMRES(d2) with the operator
    phi1(A) started at v0; the result is the composite phi2(phi1(A)) with
    p(A) = p1(A) p2(phi1(A)). Its roots("final"/"theta"/"leja") are phi2's,
    roots("inner") phi1's; .composite_degree = d_eff(phi1) * d_eff(phi2)."""
    v0 = _dev_tensor(v0, torch.float64, A.device)
    if v0.numel() != A.n:
        raise ValueError("start vector length")
    h = ctypes.c_void_p()
    info = SetupInfo()
    st = check(lib.pp_gmres_setup_double(A.handle, p1.handle, _ptr(v0), int(d2), int(bool(add_roots)),
                                         _stream(A.device), ctypes.byref(h), ctypes.byref(info)),
               "pp_gmres_setup_double")
    si = {k: getattr(info, k) for k, _ in SetupInfo._fields_}
    poly = _poly_from_handle(h, si, breakdown=(st == PP_BREAKDOWN) or bool(info.breakdown))
    poly.composite_degree = p1.d_eff * poly.d_eff if p1.composite_degree is None else \
        p1.composite_degree * poly.d_eff
    return poly


def setup_checked(A: Matrix, v0, d: int, b, tol: float = 1e-8, d_step: int = 0, d_min: int = 1,
                  add_roots: bool = True) -> Poly:
    """Setup followed by the stability check of section 3.5, the degree lowered
    by d_step (down to d_min) while StCh > tol ||b||. The returned Poly has
    .stch and .unstable (True when no degree tried passed; it is then the one
    with the smallest StCh)."""
    v0 = _dev_tensor(v0, torch.float64, A.device)
    b = _dev_tensor(b, torch.float64, A.device)
    if v0.numel() != A.n or b.numel() != A.n:
        raise ValueError("vector length")
    h = ctypes.c_void_p()
    info = SetupInfo()
    opts = StchOpts(_ptr(b), float(tol), int(d_step), int(d_min))
    sc = ctypes.c_double()
    st = check(lib.pp_gmres_setup_checked(A.handle, _ptr(v0), int(d), int(bool(add_roots)), ctypes.byref(opts),
                                          _stream(A.device), ctypes.byref(h), ctypes.byref(info), ctypes.byref(sc)),
               "pp_gmres_setup_checked")
    si = {k: getattr(info, k) for k, _ in SetupInfo._fields_}
    poly = _poly_from_handle(h, si, breakdown=(st == PP_BREAKDOWN) or bool(info.breakdown))
    poly.stch = sc.value
    poly.unstable = st == PP_UNSTABLE
    return poly


def poly_from_roots(roots, add_roots: bool = False, keep_order: bool = False) -> Poly:
    """Polynomial with given roots: Leja-ordered (optionally with added roots),
    or applied exactly in the given order with keep_order=True."""
    r = np.asarray(roots, dtype=np.complex128)
    re = np.ascontiguousarray(r.real)
    im = np.ascontiguousarray(r.imag)
    flags = (1 if add_roots else 0) | (2 if keep_order else 0)
    h = ctypes.c_void_p()
    check(lib.pp_poly_from_roots(r.size, re.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 im.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), flags,
                                 ctypes.byref(h)), "pp_poly_from_roots")
    return _poly_from_handle(h)


def apply(poly: Poly, A: Matrix, v: torch.Tensor, kind: str = "p", out: torch.Tensor | None = None) -> torch.Tensor:
    """p(A)v, phi(A)v or pi(A)v; the precision follows v's dtype (float64, float32 or bfloat16)."""
    if v.dtype not in PREC_OF_DTYPE:
        raise TypeError("v must be float64, float32 or bfloat16")
    v = v.contiguous()
    if v.numel() != A.n or v.device != A.device:
        raise ValueError("v must be a length-n tensor on the matrix's device")
    if out is None:
        out = torch.empty_like(v)
    check(lib.pp_apply(poly.handle, A.handle, KIND[kind], PREC_OF_DTYPE[v.dtype], _ptr(v), _ptr(out),
                       _stream(A.device)), "pp_apply")
    return out


def chain_bytes(poly: Poly, A: Matrix, kind: str = "phi", prec: str = "fp32"):
    """(bytes, launches) of one apply(poly, A, v, kind) in precision prec as the
    library runs it now (tuned variant, two-step fusion): the device-memory
    bytes the launches must move by their definition (pp_chain_bytes)."""
    b, l = ctypes.c_int64(), ctypes.c_int64()
    check(lib.pp_chain_bytes(poly.handle, A.handle, KIND[kind], PREC[prec], _stream(A.device), ctypes.byref(b),
                             ctypes.byref(l)), "pp_chain_bytes")
    return b.value, l.value


def solve_workspace_bytes(poly: Poly | None, A: Matrix, m: int = 50, inner: str = "fp32",
                          new_poly_degree: int = 0):
    """(total, additional) device bytes of pp_solve's workspace for these options
    on this handle (pp_solve_workspace_bytes)."""
    opts = SolveOpts(int(m), 1, 1e-8, PREC[inner], 0, 0.0, None, 0, int(new_poly_degree), 1, 0, 0, 1)
    t, a = ctypes.c_int64(), ctypes.c_int64()
    check(lib.pp_solve_workspace_bytes(poly.handle if poly is not None else None, A.handle, ctypes.byref(opts),
                                       ctypes.byref(t), ctypes.byref(a)), "pp_solve_workspace_bytes")
    return t.value, a.value


def launch_floor(launches: int, blocks: int, threads: int = 256, device="cuda"):
    """Queue `launches` empty kernels of `blocks` workgroups of `threads` threads on
    the current stream (time them with events to measure a kernel boundary's cost)."""
    check(lib.pp_launch_floor(int(launches), int(blocks), int(threads), _stream(device)), "pp_launch_floor")


def solve(poly: Poly | None, A: Matrix, b, tol: float = 1e-8, m: int = 50, max_cycles: int = 1000,
          inner: str = "fp32", stall_cycles: int = 5, x: torch.Tensor | None = None, inner_eta: float = 0.0,
          new_poly_degree: int = 0, new_poly_add: bool = True, lookahead: bool = True):
    """x solving A x = b by PP-GMRES(m) with FP64 refinement. Returns (x, info dict);
    info["history"] holds the true relative residual before each cycle and at the end.
    new_poly_degree > 0: a new polynomial of that degree from the current residual
    at every cycle (section 5.2, ChPoly); poly may then be None. lookahead: queue the
    next Arnoldi step's phi(A) before reading the current step's Hessenberg column
    (same iterates; see pp_solve_opts)."""
    b = _dev_tensor(b, torch.float64, A.device)
    if b.numel() != A.n:
        raise ValueError("right-hand side length")
    if x is None:
        x = torch.empty_like(b)
    hist = np.zeros(max(int(max_cycles), 0) + 2)
    opts = SolveOpts(int(m), int(max_cycles), float(tol), PREC[inner], int(stall_cycles), float(inner_eta),
                     hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), hist.size, int(new_poly_degree),
                     int(bool(new_poly_add)), 0, 0, int(bool(lookahead)))
    info = SolveInfo()
    st = check(lib.pp_solve(poly.handle if poly is not None else None, A.handle, _ptr(b), _ptr(x), ctypes.byref(opts), _stream(A.device),
                            ctypes.byref(info)), "pp_solve")
    out = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
    out["status_name"] = STATUS_NAMES.get(st, str(st))
    out["converged"] = st != PP_NOCONV
    out["history"] = hist[: min(hist.size, out["cycles"] + 1)].tolist()
    return x, out


def stability_check(poly: Poly, A: Matrix, b) -> float:
    """StCh = ||(b - A p(A) b) - pi(A) b|| (section 3.5), FP64 on the GPU."""
    b = _dev_tensor(b, torch.float64, A.device)
    out = ctypes.c_double()
    check(lib.pp_stability_check(poly.handle, A.handle, _ptr(b), _stream(A.device), ctypes.byref(out)),
          "pp_stability_check")
    return out.value


# ---------------------------------------------------------------------------
# differentiation: x = A(vals)^{-1} b with the adjoint solved by the same roots
# ---------------------------------------------------------------------------

class PPSolve(torch.autograd.Function):
    """x = A^{-1} b with A's stored values as a differentiable input.

    forward(vals, b, A, poly, opts): A is a Matrix whose pattern is used
    (its values are replaced by vals), poly the polynomial (for A; its
    roots serve A^T too since p(A)^T = p(A^T)), opts a dict of solve
    options. backward solves A^T lam = dL/dx with the same roots on the
    transposed pattern and returns dL/dvals[k] = -lam[row k] x[col k] and
    dL/db = lam.
    """

    @staticmethod
    def forward(ctx, vals, b, A, poly, opts):
        A.set_values(vals.detach())
        x, info = solve(poly, A, b.detach(), **opts)
        if not info["converged"]:
            raise RuntimeError(f"PP-GMRES did not converge in forward: {info}")
        ctx.A, ctx.poly, ctx.opts = A, poly, opts
        ctx.save_for_backward(vals.detach(), x)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, g):
        vals, x = ctx.saved_tensors
        A = ctx.A
        At = getattr(A, "_t", None)
        if At is None:
            At = A.transpose()
            A._t = At
        else:
            vt = torch.empty_like(vals)
            check(lib.pp_gather(A.nnz, _ptr(vals.contiguous()), _ptr(At.perm), _ptr(vt), _stream(A.device)),
                  "pp_gather")
            At.set_values(vt)
        lam, info = solve(ctx.poly, At, g.contiguous(), **ctx.opts)
        if not info["converged"]:
            raise RuntimeError(f"PP-GMRES did not converge in backward: {info}")
        dvals = A.adjoint_values(lam, x)
        return dvals, lam, None, None, None


def pp_solve_fn(vals, b, A: Matrix, poly: Poly, **opts):
    """Differentiable x = A(vals)^{-1} b (see PPSolve)."""
    return PPSolve.apply(vals, b, A, poly, opts)


# ---------------------------------------------------------------------------
# host-only building blocks (no device work; deterministic)
# ---------------------------------------------------------------------------

def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def leja_order(re, im) -> np.ndarray:
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    perm = np.zeros(re.size, dtype=np.int32)
    check(lib.pp_leja_order(re.size, _dp(re), _dp(im), _ip(perm)), "pp_leja_order")
    return perm.astype(np.int64)


def add_roots(re, im, add: bool = True):
    """Algorithm 2 steps 2-3 on Leja-ordered roots: dict of pof (mantissa, exponent), n_add, roots."""
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    d = re.size
    n_add = np.zeros(d, dtype=np.int32)
    mant = np.zeros(d)
    expo = np.zeros(d, dtype=np.int32)
    de = ctypes.c_int()
    check(lib.pp_add_roots(d, _dp(re), _dp(im), int(add), 0, None, None, ctypes.byref(de), _ip(n_add), _dp(mant),
                           _ip(expo)), "pp_add_roots")
    ro = np.zeros(de.value)
    io = np.zeros(de.value)
    check(lib.pp_add_roots(d, _dp(re), _dp(im), int(add), de.value, _dp(ro), _dp(io), ctypes.byref(de), None, None,
                           None), "pp_add_roots")
    return {"n_add": n_add, "pof_mant": mant, "pof_exp": expo, "roots": ro + 1j * io, "d_eff": de.value}


def harmonic_ritz(hbar: np.ndarray, breakdown: bool = False) -> np.ndarray:
    hbar = np.asarray(hbar, dtype=np.float64)
    k = hbar.shape[1]
    h = np.asfortranarray(hbar)
    re = np.zeros(k)
    im = np.zeros(k)
    check(lib.pp_harmonic_ritz(k, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(breakdown), _dp(re), _dp(im)),
          "pp_harmonic_ritz")
    return re + 1j * im


def hessenberg_eig(h: np.ndarray) -> np.ndarray:
    h = np.asfortranarray(np.asarray(h, dtype=np.float64))
    k = h.shape[0]
    re = np.zeros(k)
    im = np.zeros(k)
    check(lib.pp_hessenberg_eig(k, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), k, _dp(re), _dp(im)),
          "pp_hessenberg_eig")
    return re + 1j * im


# ---------------------------------------------------------------------------
# batched systems
# ---------------------------------------------------------------------------

class Batch:
    """Many independent systems solved in lockstep (block-diagonal CSR on the GPU).

    csrs: list of host CSR objects (rowptr/colind/val arrays, e.g. workloads.CSR).
    Vectors of the batch are concatenated over systems; with R right-hand
    sides they are interleaved (see interleave / deinterleave).
    """

    def __init__(self, csrs, device="cuda"):
        sizes = np.array([c.n for c in csrs], dtype=np.int64)
        self.row_off = np.zeros(len(csrs) + 1, dtype=np.int64)
        np.cumsum(sizes, out=self.row_off[1:])
        nnzs = np.array([int(c.rowptr[-1]) for c in csrs], dtype=np.int64)
        nnz_off = np.zeros(len(csrs) + 1, dtype=np.int64)
        np.cumsum(nnzs, out=nnz_off[1:])
        rp = np.empty(int(self.row_off[-1]) + 1, dtype=np.int64)
        rp[0] = 0
        cols, vals = [], []
        for s, c in enumerate(csrs):
            r0 = int(self.row_off[s])
            rp[r0 + 1: r0 + 1 + c.n] = np.asarray(c.rowptr[1:], dtype=np.int64) + nnz_off[s]
            cols.append(np.asarray(c.colind, dtype=np.int64) + r0)
            vals.append(np.asarray(c.val, dtype=np.float64))
        self.nsys = len(csrs)
        self.n = int(self.row_off[-1])
        self.nnz = int(nnz_off[-1])
        rowptr = _dev_tensor(rp.astype(np.int32), torch.int32, device)
        colind = _dev_tensor(np.concatenate(cols).astype(np.int32), torch.int32, device)
        val = _dev_tensor(np.concatenate(vals), torch.float64, device)
        self.device = val.device
        h = ctypes.c_void_p()
        ro = np.ascontiguousarray(self.row_off)
        check(lib.pp_batch_create(self.nsys, ro.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), self.nnz,
                                  _ptr(rowptr), _ptr(colind), _ptr(val), _stream(self.device), ctypes.byref(h)),
              "pp_batch_create")
        torch.cuda.synchronize(self.device)
        self.handle = h

    def interleave(self, vecs):
        """(R, n) host/device rows -> device vector of n*R values, entry (i, r) at i*R + r."""
        t = torch.as_tensor(vecs, dtype=torch.float64, device=self.device)
        if t.dim() == 1:
            t = t[None, :]
        return t.t().contiguous().reshape(-1)

    @staticmethod
    def deinterleave(x, R):
        return x.reshape(-1, R).t()

    def setup(self, v0, d: int, add_roots: bool = True):
        """One polynomial per system from GMRES(d) on each block (lockstep)."""
        v0 = _dev_tensor(v0, torch.float64, self.device)
        if v0.numel() != self.n:
            raise ValueError("start vector length")
        hs = (ctypes.c_void_p * self.nsys)()
        infos = (SetupInfo * self.nsys)()
        st = check(lib.pp_batch_setup(self.handle, _ptr(v0), int(d), int(bool(add_roots)), _stream(self.device), hs,
                                      infos), "pp_batch_setup")
        out = []
        for s in range(self.nsys):
            si = {k: getattr(infos[s], k) for k, _ in SetupInfo._fields_}
            out.append(_poly_from_handle(ctypes.c_void_p(hs[s]), si, breakdown=bool(infos[s].breakdown)))
        return out

    def solve(self, polys, b, R: int, tol: float = 1e-8, m: int = 50, max_cycles: int = 1000, inner: str = "fp32",
              stall_cycles: int = 5, inner_eta: float = 0.0, graphs: bool = True, graph_steps: int = 5):
        """x for every (system, rhs) pair; b interleaved (n*R). Returns (x, list of info dicts per pair).
        graphs: capture each restart cycle's device work, in segments of graph_steps Arnoldi
        steps (0: the whole cycle), into HIP graphs once per precision and replay them in
        later cycles (the same results as eager launches); between segments the host skips
        the rest of a cycle once every pair has stopped."""
        b = _dev_tensor(b, torch.float64, self.device)
        if b.numel() != self.n * R:
            raise ValueError("right-hand side length")
        x = torch.empty_like(b)
        hs = (ctypes.c_void_p * self.nsys)(*[p.handle.value for p in polys])
        hist = np.zeros(max(int(max_cycles), 0) + 2)
        opts = SolveOpts(int(m), int(max_cycles), float(tol), PREC[inner], int(stall_cycles), float(inner_eta),
                         hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), hist.size, 0, 1, int(bool(graphs)),
                         int(graph_steps))
        P = self.nsys * R
        infos = (SolveInfo * P)()
        check(lib.pp_batch_solve(self.handle, hs, int(R), _ptr(b), _ptr(x), ctypes.byref(opts), _stream(self.device),
                                 infos), "pp_batch_solve")
        out = []
        for p in range(P):
            d = {k: getattr(infos[p], k) for k, _ in SolveInfo._fields_}
            d["converged"] = d["status"] != PP_NOCONV
            out.append(d)
        return x, out

    def set_orth(self, mode: str):
        """Orthogonalisation of the batched cycles: "delayed" (two basis
        sweeps per step, the least squares one step behind) or "cgs2"."""
        if mode not in ("delayed", "cgs2"):
            raise ValueError("orth must be 'delayed' or 'cgs2'")
        check(lib.pp_batch_set_orth(self.handle, 1 if mode == "delayed" else 0), "pp_batch_set_orth")

    def orth(self) -> str:
        f = ctypes.c_int()
        check(lib.pp_batch_orth(self.handle, ctypes.byref(f)), "pp_batch_orth")
        return "delayed" if f.value else "cgs2"

    BATCH_FORMATS = ("sell", "pattern", "box")

    def format(self) -> str:
        """Storage the batch's sparse products read: "sell" (sliced-ELL),
        "pattern" (one byte per row naming its tuple in its system's table) or
        "box" (constant-coefficient 5-point stencils: each system's interior
        row only)."""
        f = ctypes.c_int()
        check(lib.pp_batch_format(self.handle, ctypes.byref(f)), "pp_batch_format")
        return self.BATCH_FORMATS[f.value]

    def set_format(self, name: str):
        check(lib.pp_batch_set_format(self.handle, self.BATCH_FORMATS.index(name)), "pp_batch_set_format")

    def tune(self, R: int, prec: str = "fp32"):
        """Run the batched autotuner for (prec, R) now; returns chain_config(R, prec)."""
        check(lib.pp_batch_tune(self.handle, PREC[prec], int(R), _stream(self.device)), "pp_batch_tune")
        return self.chain_config(R, prec)

    def set_chain_config(self, R: int, prec: str, fmt: str, spw: int = 1, remap: int = 1):
        """Force the chain kernel's shape for (prec, R) instead of tuning."""
        check(lib.pp_batch_set_chain_config(self.handle, PREC[prec], int(R), self.BATCH_FORMATS.index(fmt), int(spw),
                                            int(remap)), "pp_batch_set_chain_config")

    def chain_config(self, R: int, prec: str = "fp32"):
        """(format name, slices per wave, XCD order, tuned us per step) of the chain kernel in use."""
        f, spw, rm, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        check(lib.pp_batch_chain_config(self.handle, PREC[prec], int(R), ctypes.byref(f), ctypes.byref(spw),
                                        ctypes.byref(rm), ctypes.byref(us)), "pp_batch_chain_config")
        return self.BATCH_FORMATS[f.value], spw.value, rm.value, us.value

    def set_values(self, val):
        """New values (device or host float64[nnz], the concatenated systems'
        entries in CSR order); drops the pattern-coded copy."""
        v = _dev_tensor(val, torch.float64, self.device)
        if v.numel() != self.nnz:
            raise ValueError("values length")
        check(lib.pp_batch_set_values(self.handle, _ptr(v), _stream(self.device)), "pp_batch_set_values")
        torch.cuda.synchronize(self.device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is None or not h.value or lib is None:
            return
        try:
            torch.cuda.synchronize(self.device)
            lib.pp_batch_destroy(h)
        except Exception:
            pass
        self.handle = None
