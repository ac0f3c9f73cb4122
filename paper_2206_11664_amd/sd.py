"""Thin ctypes binding of ``libsdiag.so`` (the C ABI in ``include/sd.h``).

Functions keep the C names and only marshal arguments: torch device tensors
become raw pointers, the current HIP stream becomes a ``void*``.  Every step of
the computation runs in the library.  A missing library raises at import of
the first call -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdiag.so")

SD_OK, SD_ERR_ARG, SD_ERR_PARSE, SD_ERR_RANGE, SD_ERR_WORKSPACE, SD_ERR_HIP, \
    SD_ERR_INTERNAL, SD_ERR_STATE = range(8)
SD_C64, SD_C128 = 0, 1
SD_MODE_TILES, SD_MODE_PAPER_LAYERS, SD_MODE_TERMWISE = 0, 1, 2
GATE_NAMES = {0: "H", 1: "S", 2: "CNOT", 3: "CZ"}

# every symbol include/sd.h declares
EXPORTED = [
    "sd_hamiltonian_create", "sd_hamiltonian_create_masks", "sd_hamiltonian_terms",
    "sd_hamiltonian_destroy", "sd_plan_options_default", "sd_plan", "sd_plan_info_get",
    "sd_plan_export_group", "sd_plan_pass_count", "sd_plan_export_pass", "sd_plan_export_rounds",
    "sd_plan_destroy",
    "sd_bind_workspace", "sd_evolve", "sd_expectation", "sd_term_expectations", "sd_norm2", "sd_inner",
    "sd_inner_noalloc",
    "sd_ensemble_create", "sd_ensemble_workspace_bytes", "sd_ensemble_bind_workspace",
    "sd_ensemble_evolve", "sd_ensemble_destroy", "sd_sync", "sd_autotune_workspace_bytes",
    "sd_autotune_tiles", "sd_reduction_scratch_bytes", "sd_status_string",
    "sd_last_error", "sd_version",
]


class SdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class sd_plan_options(ctypes.Structure):
    _fields_ = [("skip_rule", ctypes.c_int32), ("tile_log2_c64", ctypes.c_int32),
                ("tile_log2_c128", ctypes.c_int32), ("coalesce_log2_c64", ctypes.c_int32),
                ("coalesce_log2_c128", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("coalesce_min_log2_c64", ctypes.c_int32), ("tile_shrink_c64", ctypes.c_int32),
                ("small_state_tiles", ctypes.c_int32)]


class sd_plan_info(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_terms", ctypes.c_int64),
                ("n_groups", ctypes.c_int32), ("max_group_terms", ctypes.c_int64),
                ("passes_c64", ctypes.c_int32), ("passes_c128", ctypes.c_int32),
                ("paper_model_passes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("plan_seconds", ctypes.c_double)]


class sd_group_view(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("term_ids", ctypes.POINTER(ctypes.c_int64)),
                ("zmask", ctypes.POINTER(ctypes.c_uint64)), ("sign", ctypes.POINTER(ctypes.c_int8)),
                ("n_gates", ctypes.c_int32), ("gates", ctypes.POINTER(ctypes.c_int32)),
                ("n_independent", ctypes.c_int32),
                ("independent", ctypes.POINTER(ctypes.c_int64))]


class sd_pass_view(ctypes.Structure):
    _fields_ = [("group", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("term_ids", ctypes.POINTER(ctypes.c_int64)), ("rho", ctypes.c_int32),
                ("tile_log2", ctypes.c_int32), ("basis", ctypes.POINTER(ctypes.c_uint64)),
                ("coalesce_log2", ctypes.c_int32), ("free_mask", ctypes.c_uint64),
                ("pivot_vec", ctypes.POINTER(ctypes.c_uint64)),
                ("pivot_coord", ctypes.POINTER(ctypes.c_uint32)),
                ("cz_s", ctypes.POINTER(ctypes.c_uint32)),
                ("zeta", ctypes.POINTER(ctypes.c_uint32)),
                ("ztile", ctypes.POINTER(ctypes.c_uint64)),
                ("coef", ctypes.POINTER(ctypes.c_double)), ("z_sign", ctypes.c_uint32)]


class sd_round_view(ctypes.Structure):
    _fields_ = [("n_rounds", ctypes.c_int32), ("lam_round", ctypes.c_int32),
                ("reg", (ctypes.c_int32 * 4) * 4), ("regpost", (ctypes.c_int32 * 4) * 4),
                ("xl", (ctypes.c_int32 * 2) * 4), ("nx", ctypes.c_int32 * 4),
                ("bmask", ctypes.c_uint32 * 4), ("iflag", ctypes.c_uint32 * 4),
                ("dflag", ctypes.c_uint32 * 4), ("later", ctypes.c_uint32 * 4),
                ("bucket", ctypes.POINTER(ctypes.c_int32)),
                ("n_lanes", ctypes.c_int32), ("io_coalesced", ctypes.c_int32),
                ("lanes", ctypes.POINTER(ctypes.c_uint32) * 4),
                ("lanes_post", ctypes.POINTER(ctypes.c_uint32) * 4),
                ("swz", ctypes.c_uint32 * 4), ("staged", ctypes.c_int32),
                ("czmask", ctypes.c_uint32 * 4), ("shift0", ctypes.c_int32)]


_lib = None
vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2206_11664_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    i32, i64, u64p, dp = ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64), \
        ctypes.POINTER(ctypes.c_double)
    sig = {
        "sd_hamiltonian_create": (st, [i32, i64, ctypes.POINTER(ctypes.c_char_p), dp, ctypes.POINTER(vp)]),
        "sd_hamiltonian_create_masks": (st, [i32, i64, u64p, u64p, dp, ctypes.POINTER(vp)]),
        "sd_hamiltonian_terms": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                      ctypes.POINTER(u64p), ctypes.POINTER(u64p),
                                      ctypes.POINTER(dp), ctypes.POINTER(ctypes.POINTER(i64))]),
        "sd_hamiltonian_destroy": (None, [vp]),
        "sd_plan_options_default": (None, [ctypes.POINTER(sd_plan_options)]),
        "sd_plan": (st, [vp, ctypes.POINTER(sd_plan_options), ctypes.POINTER(vp)]),
        "sd_plan_info_get": (st, [vp, ctypes.POINTER(sd_plan_info)]),
        "sd_plan_export_group": (st, [vp, i32, ctypes.POINTER(sd_group_view)]),
        "sd_plan_pass_count": (st, [vp, ctypes.c_int, ctypes.POINTER(i32)]),
        "sd_plan_export_pass": (st, [vp, ctypes.c_int, i32, ctypes.POINTER(sd_pass_view)]),
        "sd_plan_export_rounds": (st, [vp, ctypes.c_int, i32, ctypes.POINTER(sd_round_view)]),
        "sd_plan_destroy": (None, [vp]),
        "sd_bind_workspace": (st, [vp, vp, ctypes.c_size_t, vp]),
        "sd_evolve": (st, [vp, vp, ctypes.c_int, ctypes.c_double, i64, i32, vp]),
        "sd_expectation": (st, [vp, vp, ctypes.c_int, dp, vp]),
        "sd_term_expectations": (st, [vp, vp, ctypes.c_int, dp, vp]),
        "sd_reduction_scratch_bytes": (i64, []),
        "sd_norm2": (st, [vp, ctypes.c_int, i32, dp, vp, ctypes.c_size_t, vp]),
        "sd_inner": (st, [vp, vp, ctypes.c_int, i32, dp, vp, ctypes.c_size_t, vp]),
        "sd_inner_noalloc": (st, [vp, vp, ctypes.c_int, i32, dp, vp]),
        "sd_ensemble_create": (st, [ctypes.POINTER(vp), i32, ctypes.c_int, ctypes.POINTER(vp)]),
        "sd_ensemble_workspace_bytes": (st, [vp, ctypes.POINTER(i64)]),
        "sd_ensemble_bind_workspace": (st, [vp, vp, ctypes.c_size_t, vp]),
        "sd_ensemble_evolve": (st, [vp, ctypes.POINTER(vp), ctypes.c_double, i64, i32, vp]),
        "sd_ensemble_destroy": (None, [vp]),
        "sd_sync": (st, [vp]),
        "sd_autotune_workspace_bytes": (st, [vp, ctypes.POINTER(sd_plan_options), ctypes.c_int,
                                             ctypes.POINTER(i32), i32, ctypes.POINTER(i64)]),
        "sd_autotune_tiles": (st, [vp, ctypes.POINTER(sd_plan_options), ctypes.c_int, vp, ctypes.c_double,
                                   i32, i32, ctypes.POINTER(i32), i32, vp, ctypes.c_size_t,
                                   ctypes.POINTER(sd_plan_options), dp, vp]),
        "sd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "sd_last_error": (ctypes.c_char_p, []),
        "sd_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != SD_OK:
        L = lib()
        raise SdError(status, f"{L.sd_status_string(status).decode()} -- {L.sd_last_error().decode()}")


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _dtype_of(t) -> int:
    import torch
    if t.dtype == torch.complex64:
        return SD_C64
    if t.dtype == torch.complex128:
        return SD_C128
    raise TypeError(f"state dtype {t.dtype} is not complex64/complex128")


def _dev_ptr(t) -> int:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return int(t.data_ptr())


# ---------------------------------------------------------------------------
# Hamiltonian
# ---------------------------------------------------------------------------
def sd_hamiltonian_create(n_qubits: int, paulis: Sequence[str], coeffs) -> int:
    m = len(paulis)
    arr = (ctypes.c_char_p * max(m, 1))(*[p.encode() for p in paulis])
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    out = vp()
    _check(lib().sd_hamiltonian_create(n_qubits, m, arr,
                                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.byref(out)))
    return out.value


def sd_hamiltonian_create_masks(n_qubits: int, xmask, zmask, coeffs) -> int:
    x = np.ascontiguousarray(xmask, dtype=np.uint64)
    z = np.ascontiguousarray(zmask, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    out = vp()
    u64p = ctypes.POINTER(ctypes.c_uint64)
    _check(lib().sd_hamiltonian_create_masks(n_qubits, len(c), x.ctypes.data_as(u64p),
                                             z.ctypes.data_as(u64p),
                                             c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             ctypes.byref(out)))
    return out.value


def sd_hamiltonian_terms(h: int):
    n = ctypes.c_int32()
    m = ctypes.c_int64()
    x = ctypes.POINTER(ctypes.c_uint64)()
    z = ctypes.POINTER(ctypes.c_uint64)()
    c = ctypes.POINTER(ctypes.c_double)()
    s = ctypes.POINTER(ctypes.c_int64)()
    _check(lib().sd_hamiltonian_terms(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(x),
                                      ctypes.byref(z), ctypes.byref(c), ctypes.byref(s)))
    k = m.value
    return (n.value, np.ctypeslib.as_array(x, (k,)).copy() if k else np.zeros(0, np.uint64),
            np.ctypeslib.as_array(z, (k,)).copy() if k else np.zeros(0, np.uint64),
            np.ctypeslib.as_array(c, (k,)).copy() if k else np.zeros(0),
            np.ctypeslib.as_array(s, (k,)).copy() if k else np.zeros(0, np.int64))


def sd_hamiltonian_destroy(h: int):
    if h:
        lib().sd_hamiltonian_destroy(h)


# ---------------------------------------------------------------------------
# plan
# ---------------------------------------------------------------------------
def sd_plan_options_default() -> sd_plan_options:
    o = sd_plan_options()
    lib().sd_plan_options_default(ctypes.byref(o))
    return o


def sd_plan(h: int, opts: Optional[sd_plan_options] = None) -> int:
    out = vp()
    _check(lib().sd_plan(h, ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
    return out.value


def sd_plan_info_get(p: int) -> sd_plan_info:
    info = sd_plan_info()
    _check(lib().sd_plan_info_get(p, ctypes.byref(info)))
    return info


@dataclass
class GroupExport:
    term_ids: np.ndarray
    zmask: np.ndarray
    sign: np.ndarray
    gates: List[tuple]
    independent: np.ndarray


def sd_plan_export_group(p: int, g: int) -> GroupExport:
    v = sd_group_view()
    _check(lib().sd_plan_export_group(p, g, ctypes.byref(v)))
    k = v.n_terms
    gates_flat = np.ctypeslib.as_array(v.gates, (3 * v.n_gates,)).copy() if v.n_gates else []
    gates = [(GATE_NAMES[int(gates_flat[3 * i])], int(gates_flat[3 * i + 1]),
              int(gates_flat[3 * i + 2])) for i in range(v.n_gates)]
    return GroupExport(np.ctypeslib.as_array(v.term_ids, (k,)).copy(),
                       np.ctypeslib.as_array(v.zmask, (k,)).copy(),
                       np.ctypeslib.as_array(v.sign, (k,)).copy(), gates,
                       np.ctypeslib.as_array(v.independent, (v.n_independent,)).copy()
                       if v.n_independent else np.zeros(0, np.int64))


def sd_plan_pass_count(p: int, dtype: int) -> int:
    c = ctypes.c_int32()
    _check(lib().sd_plan_pass_count(p, dtype, ctypes.byref(c)))
    return c.value


def sd_plan_export_pass(p: int, dtype: int, i: int) -> dict:
    v = sd_pass_view()
    _check(lib().sd_plan_export_pass(p, dtype, i, ctypes.byref(v)))
    def arr(ptr, k):
        return np.ctypeslib.as_array(ptr, (k,)).copy() if k else np.zeros(0)
    D, m, r = v.tile_log2, v.n_terms, v.rho
    return {"group": v.group, "term_ids": arr(v.term_ids, m), "rho": r, "tile_log2": D,
            "basis": arr(v.basis, D), "coalesce_log2": v.coalesce_log2,
            "free_mask": int(v.free_mask), "pivot_vec": arr(v.pivot_vec, D),
            "pivot_coord": arr(v.pivot_coord, D), "cz_s": arr(v.cz_s, r),
            "zeta": arr(v.zeta, m), "ztile": arr(v.ztile, m), "coef": arr(v.coef, m),
            "z_sign": int(v.z_sign)}


def sd_plan_export_rounds(p: int, dtype: int, i: int) -> dict:
    v = sd_round_view()
    _check(lib().sd_plan_export_rounds(p, dtype, i, ctypes.byref(v)))
    nrounds = max(v.n_rounds, 1)
    return {"n_rounds": v.n_rounds, "lam_round": v.lam_round,
            "reg": [[v.reg[r][b] for b in range(4)] for r in range(4)],
            "regpost": [[v.regpost[r][b] for b in range(4)] for r in range(4)],
            "xl": [[v.xl[r][x] for x in range(2)] for r in range(4)],
            "nx": list(v.nx), "bmask": list(v.bmask), "iflag": list(v.iflag),
            "dflag": list(v.dflag), "later": list(v.later),
            "bucket": [v.bucket[w] for w in range(17)] if v.bucket else [0] * 17,
            "io_coalesced": v.io_coalesced,
            "lanes": [[v.lanes[r][i] for i in range(v.n_lanes)] if r < nrounds and v.n_lanes else []
                      for r in range(4)],
            "lanes_post": [[v.lanes_post[r][i] for i in range(v.n_lanes)]
                           if r < nrounds and v.n_lanes else [] for r in range(4)],
            "swz": list(v.swz), "staged": v.staged, "shift0": v.shift0,
            "czmask": list(v.czmask)}


def sd_plan_destroy(p: int):
    if p:
        lib().sd_plan_destroy(p)


# ---------------------------------------------------------------------------
# device
# ---------------------------------------------------------------------------
def sd_bind_workspace(p: int, workspace, stream=None):
    _check(lib().sd_bind_workspace(p, _dev_ptr(workspace), workspace.numel() * workspace.element_size(),
                                   _stream(stream)))


def sd_evolve(p: int, state, dt: float, steps: int, order: int = 1, stream=None):
    _check(lib().sd_evolve(p, _dev_ptr(state), _dtype_of(state), float(dt), int(steps), int(order),
                           _stream(stream)))


def sd_expectation(p: int, state, stream=None) -> float:
    e = ctypes.c_double()
    _check(lib().sd_expectation(p, _dev_ptr(state), _dtype_of(state), ctypes.byref(e),
                                _stream(stream)))
    return e.value


def sd_term_expectations(p: int, state, stream=None) -> np.ndarray:
    """<psi|P_k|psi> for every merged term k of the plan (sd_hamiltonian_terms order)."""
    info = sd_plan_info_get(p)
    out = np.zeros(int(info.n_terms), dtype=np.float64)
    _check(lib().sd_term_expectations(p, _dev_ptr(state), _dtype_of(state),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _stream(stream)))
    return out


_scratch = {}


def reduction_scratch(device):
    """A caller-owned scratch tensor for sd_norm2 / sd_inner on `device`
    (allocated by torch once per device and kept)."""
    import torch
    dev = torch.device(device)
    key = (dev.type, dev.index if dev.index is not None else torch.cuda.current_device())
    buf = _scratch.get(key)
    if buf is None:
        buf = torch.empty(int(lib().sd_reduction_scratch_bytes()), dtype=torch.uint8, device=dev)
        _scratch[key] = buf
    return buf


def sd_reduction_scratch_bytes() -> int:
    return int(lib().sd_reduction_scratch_bytes())


def sd_norm2(state, n_qubits: int, stream=None, scratch=None) -> float:
    buf = scratch if scratch is not None else reduction_scratch(state.device)
    out = ctypes.c_double()
    _check(lib().sd_norm2(_dev_ptr(state), _dtype_of(state), n_qubits, ctypes.byref(out),
                          _dev_ptr(buf), buf.numel() * buf.element_size(), _stream(stream)))
    return out.value


def sd_inner(a, b, n_qubits: int, stream=None, scratch=None) -> complex:
    buf = scratch if scratch is not None else reduction_scratch(a.device)
    out = (ctypes.c_double * 2)()
    _check(lib().sd_inner(_dev_ptr(a), _dev_ptr(b), _dtype_of(a), n_qubits, out,
                          _dev_ptr(buf), buf.numel() * buf.element_size(), _stream(stream)))
    return complex(out[0], out[1])


def sd_inner_noalloc(a, b, n_qubits: int, stream=None) -> complex:
    """sd_inner with the library's static device scratch (no caller memory)."""
    out = (ctypes.c_double * 2)()
    _check(lib().sd_inner_noalloc(_dev_ptr(a), _dev_ptr(b), _dtype_of(a), n_qubits, out,
                                  _stream(stream)))
    return complex(out[0], out[1])


def sd_ensemble_create(plans: Sequence[int], dtype: int) -> int:
    """plans: raw plan handles (``Plan.p``), each with a bound workspace."""
    arr = (vp * len(plans))(*plans)
    out = vp()
    _check(lib().sd_ensemble_create(arr, len(plans), dtype, ctypes.byref(out)))
    return out.value


def sd_ensemble_workspace_bytes(e: int) -> int:
    b = ctypes.c_int64()
    _check(lib().sd_ensemble_workspace_bytes(e, ctypes.byref(b)))
    return b.value


def sd_ensemble_bind_workspace(e: int, workspace, stream=None):
    _check(lib().sd_ensemble_bind_workspace(e, _dev_ptr(workspace),
                                            workspace.numel() * workspace.element_size(),
                                            _stream(stream)))


def sd_ensemble_evolve(e: int, states, dt: float, steps: int, order: int = 2, stream=None):
    arr = (vp * len(states))(*[_dev_ptr(s) for s in states])
    _check(lib().sd_ensemble_evolve(e, arr, float(dt), int(steps), int(order), _stream(stream)))


def sd_ensemble_destroy(e: int):
    if e:
        lib().sd_ensemble_destroy(e)


def sd_sync(stream=None):
    _check(lib().sd_sync(_stream(stream)))


def sd_autotune_workspace_bytes(h: int, dtype: int, candidates: Sequence[int],
                                base: Optional[sd_plan_options] = None) -> int:
    cand = (ctypes.c_int32 * len(candidates))(*[int(c) for c in candidates])
    b = ctypes.c_int64()
    _check(lib().sd_autotune_workspace_bytes(h, ctypes.byref(base) if base is not None else None,
                                             int(dtype), cand, len(candidates), ctypes.byref(b)))
    return b.value


def sd_autotune_tiles(h: int, dtype: int, state, dt: float, order: int, steps: int,
                      candidates: Sequence[int], base: Optional[sd_plan_options] = None,
                      stream=None, workspace=None):
    """Returns (options of the fastest candidate, per-step seconds of each).
    workspace: a device tensor of at least sd_autotune_workspace_bytes bytes
    (allocated here by torch when not given)."""
    import torch
    if workspace is None:
        nbytes = sd_autotune_workspace_bytes(h, dtype, candidates, base)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=state.device)
    cand = (ctypes.c_int32 * len(candidates))(*[int(c) for c in candidates])
    best = sd_plan_options()
    secs = np.zeros(len(candidates))
    _check(lib().sd_autotune_tiles(h, ctypes.byref(base) if base is not None else None, int(dtype),
                                   _dev_ptr(state), float(dt), int(order), int(steps), cand,
                                   len(candidates), _dev_ptr(workspace),
                                   workspace.numel() * workspace.element_size(), ctypes.byref(best),
                                   secs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   _stream(stream)))
    return best, secs


def sd_version() -> str:
    return lib().sd_version().decode()


# ---------------------------------------------------------------------------
# convenience owner objects (still marshalling only)
# ---------------------------------------------------------------------------
class Plan:
    """Owns a Hamiltonian handle, a plan handle and its device workspace."""

    def __init__(self, n: int, paulis: Sequence[str], coeffs, opts: Optional[sd_plan_options] = None,
                 device=None):
        self.n = n
        self.h = sd_hamiltonian_create(n, paulis, coeffs)
        self.p = sd_plan(self.h, opts)
        self.info = sd_plan_info_get(self.p)
        self.workspace = None
        self.device = device

    def bind(self, device="cuda"):
        import torch
        nbytes = int(self.info.workspace_bytes)
        # torch's caching allocator returns 256-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        sd_bind_workspace(self.p, self.workspace)
        return self

    def evolve(self, state, dt, steps, order=1, stream=None):
        sd_evolve(self.p, state, dt, steps, order, stream)

    def expectation(self, state, stream=None) -> float:
        return sd_expectation(self.p, state, stream)

    def term_expectations(self, state, stream=None) -> np.ndarray:
        return sd_term_expectations(self.p, state, stream)

    def group(self, g: int) -> GroupExport:
        return sd_plan_export_group(self.p, g)

    def passes(self, dtype: int) -> List[dict]:
        return [sd_plan_export_pass(self.p, dtype, i) for i in range(sd_plan_pass_count(self.p, dtype))]

    def close(self):
        sd_plan_destroy(self.p)
        sd_hamiltonian_destroy(self.h)
        self.p = self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
