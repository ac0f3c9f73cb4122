"""Dense-matrix helpers for pinning the oracle and the planner on small n.

Independent of both: matrices are assembled from the paper's 2x2 Pauli and
Clifford matrices (Eqs. pauli_matrix and clifford_gates) with Kronecker
products, and exponentials come from scipy.linalg.expm.
"""
import numpy as np
import scipy.linalg

I2 = np.eye(2, dtype=complex)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)
H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
S = np.array([[1, 0], [0, 1j]], dtype=complex)
LETTER = {"I": I2, "X": X, "Y": Y, "Z": Z}


def kron_ops(n, ops):
    """ops: dict qubit -> 2x2.  Qubit 0 is the least significant index bit, so
    it is the rightmost Kronecker factor."""
    m = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        m = np.kron(m, ops.get(q, I2))
    return m


def pauli_matrix(s):
    n = len(s)
    return kron_ops(n, {q: LETTER[ch] for q, ch in enumerate(s)})


def hamiltonian(paulis, coeffs):
    return sum(c * pauli_matrix(p) for p, c in zip(paulis, coeffs))


def expm(a):
    return scipy.linalg.expm(a)


def single(n, q, g):
    return kron_ops(n, {q: g})


def cnot(n, c, t):
    dim = 1 << n
    m = np.zeros((dim, dim), dtype=complex)
    for x in range(dim):
        y = x ^ (1 << t) if (x >> c) & 1 else x
        m[y, x] = 1
    return m


def cz(n, a, b):
    d = np.ones(1 << n, dtype=complex)
    for x in range(1 << n):
        if (x >> a) & 1 and (x >> b) & 1:
            d[x] = -1
    return np.diag(d)


def gate_matrix(n, gate):
    kind, a, b = gate
    if kind == "H":
        return single(n, a, H)
    if kind == "S":
        return single(n, a, S)
    if kind == "CNOT":
        return cnot(n, a, b)
    if kind == "CZ":
        return cz(n, a, b)
    raise ValueError(kind)


def circuit_matrix(n, gates):
    """gates in application order (first acts first)."""
    u = np.eye(1 << n, dtype=complex)
    for g in gates:
        u = gate_matrix(n, g) @ u
    return u


def zstring(n, zmask):
    return kron_ops(n, {q: Z for q in range(n) if (zmask >> q) & 1})
