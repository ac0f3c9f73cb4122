"""MI355X (gfx950) engine for Trotter evolution by simultaneous diagonalisation
of commuting Pauli groups (Kawase & Fujii, arXiv:2206.11664).

The computation lives in ``libsdiag.so`` (C ABI: ``include/sd.h``); ``sd`` is a
thin ctypes binding with the same function names.
"""
from . import sd  # noqa: F401
from .sd import Plan, SdError  # noqa: F401

__all__ = ["sd", "Plan", "SdError"]
