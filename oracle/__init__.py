"""Oracle for the Nested Neumann (NN) iteration — TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct CPU implementation of what the
HIP library computes, written from the paper (Engsig, Yang, Mehouachi,
"Generalization of higher order methods for fast iterative matrix inversion
via GPU acceleration", arXiv 2212.02406):

* ``nn_fp64``  — ``nn_ref``, the NN iteration in FP64 / complex128 NumPy, step by step, from
                 the Theorem of Sec. II-D (the method Algorithm 1 runs), with the stopping and
                 status rules this project adopts where the paper is silent.
* ``exact``    — the same iteration and the paper's closed forms (Corollaries
                 1, 2, 4, 6) in exact rational arithmetic (``fractions``), for
                 tiny integer matrices.
* ``nn_fp64.nn_factorized_solve_ref`` — the factorised series of Corollary 6
                 applied to a right-hand side (A x = B without forming X).
* ``nn_fp64.nn_cns_solve_ref`` — the Chebyshev-Neumann series: NN nests as
                 the preconditioner of a Neumann series applied to B.
* ``nn_sparse.nn_sparse_solve_ref`` — the sparse form (Algorithm 2): the
                 Neumann series in P = I - phi W applied to phi B for CSR W.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in here.  The product path (the HIP
library and its Python binding) never does, and shares no code with it: the
two meet only in the seeded input generators, which hold none of the method's
arithmetic.

Pinning: every function here is checked by ``tests/test_oracle_*.py`` against
what the paper and the mathematics fix (exact rational closed forms,
Gauss-Jordan inverses, spectral closed forms, diagonal/identity special cases,
the order of convergence).  Nothing in this package is "parity unpinned".
"""

from .nn_fp64 import (  # noqa: F401
    OK, NOT_CONVERGED, STAGNATED, ERR_ARG, ERR_DIVERGED, ERR_NONFINITE,
    X0_TRANSPOSE, X0_SCALED_IDENTITY, X0_GIVEN, X0_TRANSPOSE_FROB, X0_POWER_IDENTITY,
    X0_POWER_TRANSPOSE, X0_JACOBI, splitmix64, power_vector, theta2,
    norm_1, norm_inf, initial_guess, residual, rms_of, nn_step, nn_ref,
    nn_solve_ref, nn_factorized_solve_ref, nn_cns_solve_ref,
)
from .nn_sparse import nn_sparse_solve_ref, sparse_preconditioner  # noqa: F401,E402
