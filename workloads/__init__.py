"""Seeded synthetic inputs (Hamiltonians and initial states) shared by the
oracle, the tests and the benchmark.

This package only *draws* inputs: Pauli strings, real coefficients and
initial state vectors.  It contains none of the method's arithmetic (no
commutation test, no grouping, no Clifford synthesis, no time evolution), so
that the CPU oracle and the GPU path can both consume it without sharing any
of the computation they are compared on.
"""
from .hamiltonians import (  # noqa: F401
    Model,
    tfim_chain,
    xxz_chain,
    random_klocal,
    jw_fermionic,
    tfim_fully_connected,
    syk_majorana,
    xxz_ensemble,
    neel_state,
    neel_index,
    basis_state,
    random_state,
    config,
)
