"""FP64 CPU oracle for HICU's hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2004_08962_amd``) and imports nothing from it; the product path
never calls it.

What it computes, in plain NumPy float64 / complex128, following the paper
(Zhao, Potter, Ahmad, "High-dimensional fast convolutional framework (HICU)
for calibrationless MRI"):

* ``hankel``   — the multi-level Hankel lifting H(x) of the THEORY section
  (rows = valid-convolution outputs, columns = kernel taps over all coils),
  built explicitly, and its adjoint as a scatter-add.
* ``nullspace`` — the Gram H'H and its dense eigendecomposition; the
  nullspace basis Q spans the eigenvectors of the n-r smallest eigenvalues
  (the minimiser of Eq. 2 over Q, equivalent to the tail energy of Eq. 1).
* ``jl``       — the Johnson-Lindenstrauss compression of Algorithm 1 step
  "JL": i.i.d. normal P with variance 1/p drawn from a counter-based
  generator (Philox4x32-10 + Box-Muller), F = Q P.
* ``descent``  — objective ||H(x)F||_F^2, its gradient with hard data
  matching (zero at observed locations), the closed-form exact line search
  and the alternating minimisation of Algorithm 1.
* ``metrics``  — signal-to-error ratio as defined in the METHODS section.
* ``init``     — the time-averaged initial k-space of the 2-D+t study.
* ``rsvd``     — the paper's own nullspace route: randomized SVD of H(x)
  for the r principal right singular vectors V, then r Householder
  reflections for the basis Q orthogonal to V.
* Circular axes: the lifting and everything built on it take ``wrap``
  flags for the circular convolution along time of the 2-D+t study.

Parity status per function is listed in each module header.
"""
from .hankel import valid_extent, hankel_matrix, hankel_adjoint, forward, adjoint
from .nullspace import gram, nullspace
from .jl import philox4x32_10, philox_normals, jl_matrix
from .descent import objective_grad, line_search, descent_step, solve, objective
from .metrics import ser, rel_err
from .pointwise import grad_at_points, residual_at_points, gram_entries
from .init import time_average_init
from .rsvd import (sketch_size, sketch_matrix, rsvd_right, householder_complement,
                   nullspace_rsvd)

__all__ = [
    "valid_extent", "hankel_matrix", "hankel_adjoint", "forward", "adjoint", "gram",
    "nullspace", "philox4x32_10", "philox_normals", "jl_matrix", "objective_grad",
    "line_search", "descent_step", "solve", "objective", "ser", "rel_err",
    "grad_at_points", "residual_at_points", "gram_entries", "time_average_init",
    "sketch_size", "sketch_matrix", "rsvd_right", "householder_complement", "nullspace_rsvd",
]
