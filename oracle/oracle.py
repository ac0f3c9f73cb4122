"""CPU oracle: term-by-term FP64 Trotter evolution in the planner's group order.

TEST INFRASTRUCTURE ONLY -- imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

What it computes (plain definitions, no Clifford, tableau or diagonal form):

* Terms: H = sum_j c_j P_j, c_j real, P_j in {I,X,Y,Z}^n (Sec. "Classical
  Simulation of Quantum Dynamics").
* Grouping: the paper partitions the terms into mutually commuting groups with
  a greedy method whose details it leaves open (Sec. "Partitioning
  Hamiltonian Terms").  Reading used here: first fit in input order -- a term
  joins the lowest-index group all of whose members commute with it, else it
  opens a new group.  Exact duplicate strings are merged first by summing
  their coefficients at the first occurrence.
* One Trotter step applies the groups in sequence (Eq. trotter_simul_diag);
  group 0 acts first.  Because the terms of a group commute, the group factor
  exp(-i tau sum_k c_k P_k) equals the product of the individual rotations
  exp(-i tau c_k P_k) exactly, so the oracle applies those one by one in input
  order (Eq. trotter_decomp restricted to one group).
* Second order (not specified by the paper, which only cites Suzuki): the
  symmetric Strang sequence -- groups 0..K-2 at dt/2, group K-1 at dt,
  groups K-2..0 at dt/2.  No half steps are merged across step boundaries.
* Fourth order: Suzuki's fractal composition of five second-order steps,
  S2(p dt) S2(p dt) S2((1-4p) dt) S2(p dt) S2(p dt), p = 1/(4 - 4^(1/3)),
  again without merging.
* e^{-i theta P} psi = cos(theta) psi - i sin(theta) P psi (P^2 = I), with
  P|x> = i^{#Y} (-1)^{popcount(x & zmask)} |x ^ xmask>, evaluated in FP64 in
  ``csrc/oracle.c``.
* Energy E = sum_j c_j <psi|P_j|psi>;  fidelity F = |<a|b>|^2 / (|a|^2 |b|^2).
* apply_on_coset: the same rotations on the amplitudes of one coset of the
  span of a commuting group's X masks (which the group maps onto itself), for
  sampled outputs of states too large for the full-state loops.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_lib(force: bool = True) -> str:
    """Compile the FP64 oracle loops with gcc (OpenMP over amplitudes)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_pauli_rotate.argtypes = [ctypes.c_int32, dp, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_double]
        L.or_apply_rotations.argtypes = [ctypes.c_int32, dp, ctypes.c_int64,
                                         u64p, u64p, dp]
        L.or_pauli_expect.argtypes = [ctypes.c_int32, dp, ctypes.c_uint64,
                                      ctypes.c_uint64, dp]
        L.or_inner.argtypes = [ctypes.c_int32, dp, dp, dp]
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------------------
# Pauli strings
# ---------------------------------------------------------------------------
def parse_pauli(s: str, n: int) -> Tuple[int, int]:
    """Return (xmask, zmask) of a Pauli string.

    Dense form: ``"XIZY"`` -- character i acts on qubit i.  Sparse form:
    ``"X0 Y3 Z7"`` -- letter followed by a 0-based qubit index.  Binary
    representation as in Sec. "Tableau Representation": X -> (x=1, z=0),
    Z -> (0, 1), Y -> (1, 1).
    """
    s = s.strip()
    x = z = 0
    if s and all(ch in "IXYZ" for ch in s):
        if len(s) != n:
            raise ValueError(f"dense Pauli string of length {len(s)} for n={n}")
        items = [(q, ch) for q, ch in enumerate(s)]
    else:
        items = []
        seen = set()
        for tok in s.split():
            ch, q = tok[0], int(tok[1:])
            if ch not in "IXYZ" or not (0 <= q < n) or q in seen:
                raise ValueError(f"bad sparse Pauli token {tok!r}")
            seen.add(q)
            items.append((q, ch))
    for q, ch in items:
        if ch in "XY":
            x |= 1 << q
        if ch in "ZY":
            z |= 1 << q
    return x, z


@dataclass
class Terms:
    n: int
    x: np.ndarray        # uint64 xmasks (after duplicate merge)
    z: np.ndarray        # uint64 zmasks
    c: np.ndarray        # float64 coefficients
    source: np.ndarray   # index of the first input entry of each merged term


def build_terms(n: int, paulis: Sequence[str], coeffs: Sequence[float]) -> Terms:
    """Parse and merge exact duplicates (coefficient sum at first occurrence)."""
    index = {}
    xs, zs, cs, src = [], [], [], []
    for i, (p, c) in enumerate(zip(paulis, coeffs)):
        key = parse_pauli(p, n)
        if key in index:
            cs[index[key]] += float(c)
            continue
        index[key] = len(xs)
        xs.append(key[0])
        zs.append(key[1])
        cs.append(float(c))
        src.append(i)
    return Terms(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
                 np.array(cs, dtype=np.float64), np.array(src, dtype=np.int64))


def commutes(xa: int, za: int, xb: int, zb: int) -> bool:
    """Two Pauli strings commute iff the number of qubits on which they
    anticommute (symplectic product x_a.z_b + x_b.z_a) is even."""
    return (bin(int(xa) & int(zb)).count("1") + bin(int(xb) & int(za)).count("1")) % 2 == 0


def first_fit_groups(t: Terms) -> List[List[int]]:
    """Greedy colouring of the anticommutation graph, vertices in term order."""
    groups: List[List[int]] = []
    xs = [int(v) for v in t.x]
    zs = [int(v) for v in t.z]
    for k in range(len(xs)):
        for g in groups:
            if all(commutes(xs[k], zs[k], xs[j], zs[j]) for j in g):
                g.append(k)
                break
        else:
            groups.append([k])
    return groups


def schedule(n_groups: int, order: int) -> List[Tuple[int, float]]:
    """(group, fraction of dt) in application order for one Trotter step."""
    if order == 1:
        return [(g, 1.0) for g in range(n_groups)]
    if order == 2:
        if n_groups == 1:
            return [(0, 1.0)]
        seq = [(g, 0.5) for g in range(n_groups - 1)]
        seq.append((n_groups - 1, 1.0))
        seq += [(g, 0.5) for g in range(n_groups - 2, -1, -1)]
        return seq
    if order == 4:
        # Suzuki's fourth-order fractal: S2(p) S2(p) S2(1 - 4p) S2(p) S2(p),
        # p = 1 / (4 - 4^(1/3)), each S2 the sequence above (no merging)
        p = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))
        s2 = schedule(n_groups, 2)
        return [(g, f * w) for w in (p, p, 1.0 - 4.0 * p, p, p) for g, f in s2]
    raise ValueError("order must be 1, 2 or 4")


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def evolve(n: int, paulis, coeffs, psi0: np.ndarray, dt: float, steps: int,
           order: int = 1, groups: List[List[int]] = None,
           terms: Terms = None) -> np.ndarray:
    """Grouped Trotter evolution, term by term, FP64.  Returns a new array."""
    t = terms if terms is not None else build_terms(n, paulis, coeffs)
    g = groups if groups is not None else first_fit_groups(t)
    seq = schedule(len(g), order)
    psi = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128)).copy()
    # flatten one step into a rotation list (first entry acts first)
    xs, zs, th = [], [], []
    for gi, frac in seq:
        for k in g[gi]:
            xs.append(int(t.x[k]))
            zs.append(int(t.z[k]))
            th.append(float(t.c[k]) * dt * frac)
    xs = np.array(xs, dtype=np.uint64)
    zs = np.array(zs, dtype=np.uint64)
    th = np.array(th, dtype=np.float64)
    L = lib()
    pv = psi.view(np.float64)
    for _ in range(steps):
        L.or_apply_rotations(n, _dp(pv), len(xs),
                             xs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                             zs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                             _dp(th))
    return psi


def evolve_terms_dense(n: int, xs, zs, thetas, psi0: np.ndarray) -> np.ndarray:
    """Apply exp(-i theta_k P_k) in the given order (first acts first)."""
    psi = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128)).copy()
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    zs = np.ascontiguousarray(zs, dtype=np.uint64)
    th = np.ascontiguousarray(thetas, dtype=np.float64)
    lib().or_apply_rotations(n, _dp(psi.view(np.float64)), len(xs),
                             xs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                             zs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                             _dp(th))
    return psi


def apply_on_coset(xs, zs, thetas, x0: int, span, amps) -> np.ndarray:
    """exp(-i theta_k P_k) applied in the given order (first acts first) to the
    amplitudes of a state on one coset C = {x0 ^ (XOR of span[i] over the set
    bits i of j)} of a subspace that holds every X mask; amps[j] is the
    amplitude at that index.  Each P_k maps C onto itself (x -> x ^ xmask_k),
    so the output on C depends on amps alone: the same rotation as the
    full-state loops, e^{-i theta P} = cos(theta) - i sin(theta) P with
    (P psi)[y] = i^{popcount(xmask & zmask)} (-1)^{popcount((y ^ xmask) & zmask)}
    psi[y ^ xmask], restricted to C.  FP64.  Used for sampled outputs of
    states too large for the full-state loops."""
    span = [int(v) for v in span]
    r = len(span)
    # echelon form of the span with each row's combination of span[i]
    rows = []
    for i, v in enumerate(span):
        comb = 1 << i
        for rv, rc in rows:
            if v ^ rv < v:
                v, comb = v ^ rv, comb ^ rc
        if v == 0:
            raise ValueError("span vectors must be independent")
        rows.append((v, comb))
        rows.sort(reverse=True)

    def coords(x: int) -> int:
        comb = 0
        for rv, rc in rows:
            if x ^ rv < x:
                x, comb = x ^ rv, comb ^ rc
        if x != 0:
            raise ValueError("X mask outside the span")
        return comb

    j = np.arange(1 << r, dtype=np.int64)
    phys = np.full(1 << r, np.uint64(x0), dtype=np.uint64)
    for i, v in enumerate(span):
        phys ^= ((j >> i) & 1).astype(np.uint64) * np.uint64(v)
    psi = np.asarray(amps, dtype=np.complex128).copy()
    for x, z, th in zip(xs, zs, thetas):
        x, z = int(x), int(z)
        a = coords(x)
        src = j ^ a
        ny = bin(x & z).count("1")
        par = np.bitwise_count(phys[src] & np.uint64(z)) & 1
        ppsi = (1j ** ny) * np.where(par == 1, -1.0, 1.0) * psi[src]
        psi = np.cos(th) * psi - 1j * np.sin(th) * ppsi
    return psi


def term_expectations(n: int, paulis, coeffs, psi: np.ndarray, terms: Terms = None) -> np.ndarray:
    """<psi|P_k|psi> of every merged term k (build_terms order), FP64, term by
    term over the full state (no grouping)."""
    t = terms if terms is not None else build_terms(n, paulis, coeffs)
    psi = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    out = np.zeros(2)
    vals = np.zeros(len(t.x))
    L = lib()
    for k in range(len(t.x)):
        L.or_pauli_expect(n, _dp(psi.view(np.float64)), int(t.x[k]), int(t.z[k]), _dp(out))
        vals[k] = out[0]
    return vals


def energy(n: int, paulis, coeffs, psi: np.ndarray, terms: Terms = None) -> float:
    t = terms if terms is not None else build_terms(n, paulis, coeffs)
    psi = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    out = np.zeros(2)
    e = 0.0
    L = lib()
    for k in range(len(t.x)):
        L.or_pauli_expect(n, _dp(psi.view(np.float64)), int(t.x[k]), int(t.z[k]),
                          _dp(out))
        e += float(t.c[k]) * out[0]
    return e


def fidelity(a: np.ndarray, b: np.ndarray) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ov = np.vdot(a, b)
    return float(abs(ov) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
