"""FP64 CPU oracle for polynomial-preconditioned GMRES (Loe & Morgan, arXiv 1911.07065).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, deliberately
unoptimised restatement of the paper's method in numpy/scipy float64. It is
used by the tests, by ``__graft_entry__.smoke()`` and by the CPU-baseline leg
of ``bench.py``; the product path (the HIP library and its Python binding)
never imports it, and it imports nothing from the product path. The two
share only the seeded input generators in ``workloads``.

Modules
-------
roots   : setup GMRES(d) cycle, harmonic Ritz values, modified Leja order,
          pof, added roots (section 2, Algorithm 2, Algorithm 4 step 1).
chains  : phi(A)v (Algorithm 1) and p(A)v (Algorithm 3, eq. (3.1)).
solver  : PP-GMRES(m) (Algorithm 4 step 2), stability check (section 3.5).
mixed   : float32 / bfloat16-storage emulation of the chains (no paper
          passage: used to state the bound for the mixed-precision form).
adjoint : gradient of a loss through x = A^{-1} b by a direct solve.

Parity status: every function is pinned by ``tests/test_oracle_*.py``
except the exact insertion positions of added roots (``roots.insert_roots``),
which the paper describes only in words ("parity unpinned": only the
properties the text states are checked).
"""

from .roots import (  # noqa: F401
    arnoldi,
    harmonic_ritz,
    leja_order,
    pof_values,
    n_add_from_pof,
    insert_roots,
    setup,
    Poly,
)
from .chains import apply_phi, apply_p, apply_pi  # noqa: F401
from .solver import pp_gmres, stability_check  # noqa: F401
