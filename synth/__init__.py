"""Seeded synthetic problem data shared by the oracle, the tests and the benchmark.

This package draws random one- and two-body integrals and fixes the spectral shift.
It contains none of the solver's arithmetic: no operator application, no
preconditioner, no truncation.  Both the CPU oracle and the GPU library receive
exactly the arrays produced here.
"""
from .integrals import (  # noqa: F401
    Problem,
    make_problem,
    random_dense,
    random_decayed,
    sym8,
    v_from_chemist,
    shift_lower_bound,
)
from .mps import rho_table, random_block_mps, layout  # noqa: F401,E402
from .learned import N_FEAT, WIDTH, N_PARAMS, init_params, sample_determinants  # noqa: F401,E402
