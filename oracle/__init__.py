"""FP64 CPU oracle for the alpha-circulant preconditioned Richardson method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) imports, links or executes anything in this package; only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` do.  The oracle shares no code with the HIP path: it never forms
the alpha-circulant preconditioner's diagonalisation, never transforms over the
time steps and never touches the eigenbasis of Q G^{-1}.

What it computes (Caklovic, Speck, Frank, arXiv 2103.12571):

* Radau-right collocation nodes and the integration matrix Q (Sec. 2.1, eq.
  (collocation); node polynomial P_{M-1}+P_M, Sec. 2.3).
* Periodic finite-difference operators, including central (order 2, 4, 6) and
  upwind (order 1..5) differences from their moment conditions (Sec. 5).
* The composite collocation solution of C u = w (with an optional source b(t)
  at the collocation times), by sequential step-by-step
  collocation solves (Sec. 2.1, eq. (seq_collocation_problem)) with three
  interchangeable spatial back-ends (dense, sparse LU, per-Fourier-mode), and
  by brute force on the assembled all-at-once matrix (eq. (globalsys)).
* The all-at-once residual w - C u, the preconditioner solve C_alpha^{-1} r
  (eq. (prec)) by a sparse direct solve, and the alpha schedule of Alg. 2.
* The adjoint system C^T lambda = g by a backward sequential sweep and the
  gradients of 1/2 ||u_{L,M} - u_target||^2 with respect to u0 and nu.
* Flexible GMRES on C u = w with C_alpha as right preconditioner (the Krylov
  alternative to Richardson that the paper points to).

Parity status of each function is stated in its docstring; every function is
pinned by a ``-m "not gpu"`` test against closed forms or values printed in
the paper, except where a docstring says "parity unpinned".
"""

from .collocation import radau_right_nodes, collocation_matrix, node_polynomial
from .operators import PeriodicStencil, stencil_for, fd_weights, central_d2, upwind_d1
from .sequential import sequential_solve
from .allatonce import (assemble_C, assemble_C_alpha, assemble_w, residual,
                        precond_solve, brute_force_solve)
from .adjoint import adjoint_solve, gradients
from .alpha import alpha_schedule
from .gmres import fgmres, gmres_solve

__all__ = [
    "fgmres", "gmres_solve",
    "radau_right_nodes", "collocation_matrix", "node_polynomial",
    "PeriodicStencil", "stencil_for", "fd_weights", "central_d2", "upwind_d1", "sequential_solve",
    "assemble_C", "assemble_C_alpha", "assemble_w", "residual",
    "precond_solve", "brute_force_solve", "adjoint_solve", "gradients",
    "alpha_schedule",
]
