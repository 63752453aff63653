"""MI355X-native polynomial-preconditioned GMRES (Loe & Morgan, arXiv 1911.07065).

The hot path (root-product chains, CSR sparse products, Gram-Schmidt) runs
in hand-written HIP kernels for gfx950 inside ``libppgmres.so``; the small
dense work (harmonic Ritz values, Leja ordering, added roots, Givens least
squares) runs in the same library's C++ host core. This package only
marshals arguments; PyTorch provides device memory and streams.

Public API (see ``api``): Matrix, Poly, setup, poly_from_roots, apply,
solve, stability_check, PPSolve, and the host helpers leja_order,
add_roots, harmonic_ritz, hessenberg_eig.
"""

__all__ = [
    "Matrix", "Poly", "setup", "setup_checked", "setup_double", "poly_from_roots", "apply", "solve", "stability_check", "PPSolve",
    "pp_solve_fn", "leja_order", "add_roots", "harmonic_ritz", "hessenberg_eig", "version", "Batch",
]


def __getattr__(name):
    if name in __all__:
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
