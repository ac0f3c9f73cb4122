"""CPU oracle for grouped Trotter evolution -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it (own parser, own grouping, own schedule, own FP64
rotation loops in ``csrc/oracle.c``).
"""
from .oracle import (  # noqa: F401
    parse_pauli,
    Terms,
    build_terms,
    commutes,
    first_fit_groups,
    schedule,
    evolve,
    evolve_terms_dense,
    apply_on_coset,
    energy,
    term_expectations,
    fidelity,
    lib,
    build_lib,
    num_threads,
)
