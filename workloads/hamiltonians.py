"""Seeded generators for the synthetic Pauli-sum Hamiltonians of the benchmark
configurations and for the paper's own experiment families.

Conventions (fixed here once, used everywhere):

* A Hamiltonian is ``H = sum_j c_j P_j`` with real ``c_j`` and ``P_j`` a tensor
  product of I, X, Y, Z (Sec. "Classical Simulation of Quantum Dynamics").
* A Pauli string is written densely, character ``i`` acting on qubit ``i``
  (0-based).  The paper lists qubit 1 first in its strings (e.g. X1 Y2 Z3),
  so its qubit 1 is our qubit 0.
* Qubit ``q`` is bit ``q`` of the amplitude index (the paper's basis
  |b_n ... b_1>, qubit 1 the least significant bit).
* Every random draw uses ``numpy.random.default_rng(seed)`` in the order the
  docstring states, so the terms (and therefore the greedy grouping, which
  depends on term order) are reproducible.

No function here evaluates anything about the method: the output is strings,
coefficients and state vectors.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Model:
    """A Pauli-sum Hamiltonian plus the run parameters of a workload."""
    name: str
    n: int
    paulis: List[str]
    coeffs: np.ndarray
    dt: float = 0.01
    steps: int = 1
    order: int = 1
    init: str = "zero"          # "zero" | "neel" | "random" | "basis"
    init_seed: Optional[int] = None
    init_index: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return len(self.paulis)

    def initial_state(self, dtype=np.complex128) -> np.ndarray:
        if self.init == "zero":
            return basis_state(self.n, 0, dtype)
        if self.init == "neel":
            return neel_state(self.n, dtype)
        if self.init == "basis":
            return basis_state(self.n, self.init_index, dtype)
        if self.init == "random":
            return random_state(self.n, self.init_seed, dtype)
        raise ValueError(self.init)


def _dense(n: int, ops: dict) -> str:
    s = ["I"] * n
    for q, p in ops.items():
        s[q] = p
    return "".join(s)


# ---------------------------------------------------------------------------
# initial states
# ---------------------------------------------------------------------------
def basis_state(n: int, index: int, dtype=np.complex128) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=dtype)
    psi[index] = 1.0
    return psi


def neel_index(n: int) -> int:
    """Neel pattern: qubit i holds (i mod 2), i.e. index 0b...1010."""
    return sum(1 << i for i in range(1, n, 2))


def neel_state(n: int, dtype=np.complex128) -> np.ndarray:
    return basis_state(n, neel_index(n), dtype)


def random_state(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex Gaussian vector, normalised in float64 (re draws, then im draws)."""
    rng = np.random.default_rng(seed)
    dim = 1 << n
    re = rng.standard_normal(dim)
    im = rng.standard_normal(dim)
    psi = re + 1j * im
    psi /= np.sqrt(np.vdot(psi, psi).real)
    return psi.astype(dtype)


# ---------------------------------------------------------------------------
# Hamiltonian families
# ---------------------------------------------------------------------------
def tfim_chain(n: int = 12, J: float = 1.0, h: float = 1.0) -> Model:
    """Open 1D transverse-field Ising chain: -J Z_i Z_{i+1} (i=0..n-2), then
    -h X_i (i=0..n-1).  Initial |0...0>, first order, dt 0.01, 100 steps."""
    paulis, coeffs = [], []
    for i in range(n - 1):
        paulis.append(_dense(n, {i: "Z", i + 1: "Z"}))
        coeffs.append(-J)
    for i in range(n):
        paulis.append(_dense(n, {i: "X"}))
        coeffs.append(-h)
    return Model("tfim_chain", n, paulis, np.array(coeffs), dt=0.01, steps=100,
                 order=1, init="zero")


def _xxz_terms(n: int, periodic: bool, h: np.ndarray, delta: float = 0.5):
    bonds = [(i, (i + 1) % n) for i in range(n)] if periodic else \
        [(i, i + 1) for i in range(n - 1)]
    paulis, coeffs = [], []
    for (i, j) in bonds:
        paulis.append(_dense(n, {i: "X", j: "X"}))
        coeffs.append(1.0)
    for (i, j) in bonds:
        paulis.append(_dense(n, {i: "Y", j: "Y"}))
        coeffs.append(1.0)
    for (i, j) in bonds:
        paulis.append(_dense(n, {i: "Z", j: "Z"}))
        coeffs.append(delta)
    for i in range(n):
        paulis.append(_dense(n, {i: "Z"}))
        coeffs.append(float(h[i]))
    return paulis, np.array(coeffs)


def xxz_chain(n: int = 26, seed: int = 2, periodic: bool = True,
              hmax: float = 1.0, dt: float = 0.05, steps: int = 1000) -> Model:
    """XXZ chain with random fields: sum_bonds (XX + YY + 0.5 ZZ) + sum_i h_i Z_i,
    h ~ U[-hmax, hmax] drawn from ``default_rng(seed)`` (n draws).  Terms are
    emitted all-XX, then all-YY, then all-ZZ, then the fields, which makes the
    first-fit grouping (XX)(YY)(ZZ+Z).  Neel initial state, second order."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(-hmax, hmax, size=n)
    paulis, coeffs = _xxz_terms(n, periodic, h)
    return Model("xxz_chain", n, paulis, coeffs, dt=dt, steps=steps, order=2,
                 init="neel", meta={"periodic": periodic, "h": h})


def random_klocal(n: int = 28, m: int = 2000, seed: int = 3,
                  init_seed: int = 30, dt: float = 0.01, steps: int = 200) -> Model:
    """Random sparse k-local Pauli Hamiltonian.  For each of ``m`` draws, in
    this order: weight w ~ U{2,3,4}; w distinct qubits (uniform, without
    replacement); one letter per qubit ~ U{X,Y,Z}; coefficient c ~ N(0,1).
    Exact duplicate strings are kept as separate entries here (the planner and
    the oracle each merge them).  Random complex-Gaussian initial state from
    ``init_seed``; first order."""
    rng = np.random.default_rng(seed)
    paulis, coeffs = [], []
    letters = "XYZ"
    for _ in range(m):
        w = int(rng.integers(2, 5))
        qs = rng.choice(n, size=w, replace=False)
        ls = rng.integers(0, 3, size=w)
        paulis.append(_dense(n, {int(q): letters[int(l)] for q, l in zip(qs, ls)}))
        coeffs.append(float(rng.standard_normal()))
    return Model("random_klocal", n, paulis, np.array(coeffs), dt=dt, steps=steps,
                 order=1, init="random", init_seed=init_seed)


def _jw_hop(n: int, i: int, j: int, a: str, b: str) -> dict:
    ops = {i: a, j: b}
    for k in range(i + 1, j):
        ops[k] = "Z"
    return ops


def jw_fermionic(n: int = 32, total: int = 10000, seed: int = 5,
                 dt: float = 0.02, steps: int = 100) -> Model:
    """Jordan-Wigner-shaped fermionic Hamiltonian.

    Emission order: every hopping i<j with endpoint letters (X,X), (Y,Y), (X,Y),
    (Y,X) and Z on i+1..j-1; every Z_i Z_j (i<j); every Z_i; then random
    double-excitation strings on four qubits i<j<k<l (two JW pairs (i,j) and
    (k,l), each with random X/Y endpoints) until ``total`` distinct strings.
    Coefficients: +-10^U[-4,0] (sign and exponent drawn per term after all
    strings are fixed).  Hartree-Fock-like initial state: qubits 0..n/2-1 set.
    """
    rng = np.random.default_rng(seed)
    paulis = []
    seen = set()

    def add(s):
        if s not in seen:
            seen.add(s)
            paulis.append(s)

    for i in range(n):
        for j in range(i + 1, n):
            for (a, b) in (("X", "X"), ("Y", "Y"), ("X", "Y"), ("Y", "X")):
                add(_dense(n, _jw_hop(n, i, j, a, b)))
    for i in range(n):
        for j in range(i + 1, n):
            add(_dense(n, {i: "Z", j: "Z"}))
    for i in range(n):
        add(_dense(n, {i: "Z"}))
    # (at most 16 C(n, 4) distinct double-excitation strings exist: ask for
    # no more than there are, or the draw below would never end)
    n_dbl = 16 * (n * (n - 1) * (n - 2) * (n - 3) // 24)
    if total > len(paulis) + n_dbl:
        raise ValueError(f"jw_fermionic: total={total} exceeds the {len(paulis) + n_dbl} "
                         f"distinct strings available at n={n}")
    while len(paulis) < total:
        q = sorted(int(v) for v in rng.choice(n, size=4, replace=False))
        ops = {}
        for (i, j) in ((q[0], q[1]), (q[2], q[3])):
            for k in range(i + 1, j):
                ops[k] = "Z" if ops.get(k, "I") == "I" else "I"
            ops[i] = "XY"[int(rng.integers(2))]
            ops[j] = "XY"[int(rng.integers(2))]
        ops = {k: v for k, v in ops.items() if v != "I"}
        add(_dense(n, ops))
    expo = rng.uniform(-4.0, 0.0, size=len(paulis))
    sign = np.where(rng.integers(0, 2, size=len(paulis)) == 1, 1.0, -1.0)
    coeffs = sign * np.power(10.0, expo)
    hf = sum(1 << i for i in range(n // 2))
    return Model("jw_fermionic", n, paulis, coeffs, dt=dt, steps=steps, order=2,
                 init="basis", init_index=hf)


def tfim_fully_connected(n: int, seed: int = 0, dt: float = 0.01) -> Model:
    """Fully connected TFIM of the paper's experiments: sum_{i<j} J_ij Z_i Z_j +
    sum_i h_i X_i with J, h ~ U[-1,1] (J in (i,j) lexicographic order, then h).
    m = n(n-1)/2 + n terms, two commuting groups."""
    rng = np.random.default_rng(seed)
    paulis, coeffs = [], []
    J = rng.uniform(-1, 1, size=n * (n - 1) // 2)
    h = rng.uniform(-1, 1, size=n)
    t = 0
    for i in range(n):
        for j in range(i + 1, n):
            paulis.append(_dense(n, {i: "Z", j: "Z"}))
            coeffs.append(float(J[t]))
            t += 1
    for i in range(n):
        paulis.append(_dense(n, {i: "X"}))
        coeffs.append(float(h[i]))
    return Model("tfim_fully_connected", n, paulis, np.array(coeffs), dt=dt,
                 steps=1, order=1, init="zero")


def _majorana(q: int, y: bool):
    """Jordan-Wigner Majorana on qubit q (0-based) as i^k X^x Z^z (per qubit,
    X^x_q Z^z_q): Z on the qubits below q, then X (k = 0) or Y = i X Z
    (k = 1) on qubit q."""
    below = (1 << q) - 1
    return (1 if y else 0, 1 << q, below | ((1 << q) if y else 0))


def syk_majorana(n: int, seed: int = 6, dt: float = 0.01) -> Model:
    """SYK Majorana model of the paper's second experiment on n qubits:
    H = sum_{a<b<c<d} g_abcd c_a c_b c_c c_d over the 2n Jordan-Wigner
    Majoranas c_{2q} = Z_0..Z_{q-1} X_q, c_{2q+1} = Z_0..Z_{q-1} Y_q.

    The paper draws J_ijkl complex Gaussian with J_ijkl = -J_jikl = -J_ijlk =
    J*_lkji and sums over all orderings; collecting the orderings of four
    distinct Majoranas onto c_a c_b c_c c_d (a < b < c < d) leaves one real
    coefficient per 4-subset, and the product is a Hermitian Pauli string up
    to a sign.  Reading used here: that real coefficient is drawn directly,
    g ~ N(0, 1) from default_rng(seed) in lexicographic (a, b, c, d) order;
    the sign of the product goes into the coefficient.  C(2n, 4) terms
    (367,290 at n = 28)."""
    import itertools
    rng = np.random.default_rng(seed)
    quads = list(itertools.combinations(range(2 * n), 4))
    g = rng.normal(size=len(quads))
    maj = [_majorana(a // 2, a % 2 == 1) for a in range(2 * n)]
    letters = {(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}
    paulis, coeffs = [], []
    for t, quad in enumerate(quads):
        k, x, z = 0, 0, 0
        for a in quad:
            k2, x2, z2 = maj[a]
            # (i^k X^x Z^z)(i^k2 X^x2 Z^z2) = i^{k+k2} (-1)^{z.x2} X^{x^x2} Z^{z^z2}
            k = (k + k2 + 2 * (bin(z & x2).count("1") & 1)) & 3
            x ^= x2
            z ^= z2
        # i^k X^x Z^z = i^{k - |x&z|} P with P the Hermitian string (Y = i X Z)
        e = (k - bin(x & z).count("1")) & 3
        assert e in (0, 2), "a product of four distinct Majoranas is Hermitian"
        paulis.append("".join(letters[((x >> q) & 1, (z >> q) & 1)] for q in range(n)))
        coeffs.append(float(g[t]) * (1.0 if e == 0 else -1.0))
    return Model("syk_majorana", n, paulis, np.array(coeffs), dt=dt, steps=1, order=1,
                 init="random", init_seed=seed + 100)


def xxz_ensemble(count: int = 256, seed: int = 4, nmin: int = 14, nmax: int = 20,
                 dt: float = 0.05, steps: int = 500) -> List[Model]:
    """Disorder ensemble of open XXZ chains of uneven size.  From
    ``default_rng(seed)``: all sizes n_i ~ U{nmin..nmax} first, then for each
    instance in turn its n_i fields h ~ U[-2, 2].  Neel initial states,
    second order."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for idx, n in enumerate(ns):
        n = int(n)
        h = rng.uniform(-2.0, 2.0, size=n)
        paulis, coeffs = _xxz_terms(n, False, h)
        out.append(Model(f"xxz_open_{idx}", n, paulis, coeffs, dt=dt, steps=steps,
                         order=2, init="neel", meta={"h": h}))
    return out


def config(idx: int, **kw):
    """The five benchmark workloads, 1-based: 1 TFIM chain n=12; 2 periodic XXZ
    n=26; 3 random k-local n=28; 4 XXZ ensemble (list of models); 5 JW n=32.
    Keyword arguments override sizes (e.g. ``n=``) for reduced parity runs."""
    if idx == 1:
        return tfim_chain(**kw)
    if idx == 2:
        return xxz_chain(**kw)
    if idx == 3:
        return random_klocal(**kw)
    if idx == 4:
        return xxz_ensemble(**kw)
    if idx == 5:
        return jw_fermionic(**kw)
    raise ValueError(idx)
