"""Seeded generator of one large commuting group with a chosen X-span rank,
for planner and kernel tests (test helper; no method arithmetic beyond the
Pauli product rule used to build the test input)."""
import numpy as np


def _letters(n, x, z):
    return "".join("IXZY"[((x >> q) & 1) | (((z >> q) & 1) << 1)] for q in range(n))


def commuting_group(rng, n, rho, n_terms, alternating=False, n_cnots=None):
    """n_terms mutually commuting Pauli strings whose X parts span rank rho.

    Built from generators X_{s_i} prod_j Z_{s_j}^{W_ij} (W symmetric over
    GF(2), zero diagonal when `alternating`) with extra Z factors on qubits
    outside the span, multiplied together at random and conjugated by a
    random CNOT network so that the X span is a general subspace."""
    span = rng.permutation(n)[:rho]
    rest = [q for q in range(n) if q not in set(span.tolist())]
    W = rng.integers(0, 2, size=(rho, rho))
    W = np.triu(W, 1)
    W = W + W.T
    if not alternating:
        W[np.diag_indices(rho)] = rng.integers(0, 2, size=rho)
    elif rho >= 2 and not W.any():
        W[0, 1] = W[1, 0] = 1
    gens = []
    for i in range(rho):
        x = 1 << int(span[i])
        z = 0
        for j in range(rho):
            if W[i, j]:
                z |= 1 << int(span[j])
        for q in rest:
            if rng.random() < 0.3:
                z |= 1 << q
        gens.append((x, z))
    terms = set()
    tries = 0
    while len(terms) < n_terms and tries < 100 * n_terms:
        tries += 1
        x = z = 0
        for i in range(rho):
            if rng.random() < 0.35:
                x ^= gens[i][0]
                z ^= gens[i][1]
        if rng.random() < 0.2:
            for q in rest:
                if rng.random() < 0.3:
                    z ^= 1 << q
        if x or z:
            terms.add((x, z))
    terms = sorted(terms)
    cn = 3 * n if n_cnots is None else n_cnots
    for _ in range(cn):
        c, t = rng.choice(n, size=2, replace=False)
        c, t = int(c), int(t)
        new = []
        for x, z in terms:
            x ^= ((x >> c) & 1) << t
            z ^= ((z >> t) & 1) << c
            new.append((x, z))
        terms = new
    paulis = [_letters(n, x, z) for x, z in terms]
    coeffs = rng.normal(size=len(paulis))
    return paulis, coeffs
