"""Seeded synthetic inputs (matrices in CSR form, right-hand sides, start vectors).

This package holds no arithmetic of the solver: it only builds test and
benchmark inputs. Both the CPU oracle and the GPU path read their inputs
from here, so that the two sides see bit-identical data.
"""

from .generators import (  # noqa: F401
    CSR,
    convdiff2d,
    convdiff2d_parts,
    convdiff2d_colscaled, convdiff2d_blockmixed,
    convdiff3d,
    convdiff3d_box,
    randsparse,
    biharmonic2d,
    diagonal,
    diag_example7,
    diag_squares,
    diag_clusters,
    diag_wide,
    normal_vector,
    rhs,
    start_vector,
    batched_convdiff_specs,
)
