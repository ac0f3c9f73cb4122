"""Pins of the CPU oracle against facts fixed outside it: dense matrix
exponentials, closed forms, Trotter error orders, the paper's printed
examples and invariants.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle
import workloads
from tests import dense

pytestmark = pytest.mark.usefixtures("oracle_lib")


def rand_paulis(rng, n, m, wmax=None):
    out = []
    for _ in range(m):
        s = "".join("IXYZ"[int(rng.integers(4))] for _ in range(n))
        out.append(s)
    return out


# --- parsing: the paper's binary representation example -------------------
def test_parse_paper_example():
    # Sec. "Tableau Representation": X1 Y2 Z3 is represented by 110011,
    # i.e. x = (1,1,0) and z = (0,1,1) over qubits 1,2,3.
    x, z = oracle.parse_pauli("XYZ", 3)
    assert [(x >> q) & 1 for q in range(3)] == [1, 1, 0]
    assert [(z >> q) & 1 for q in range(3)] == [0, 1, 1]
    assert oracle.parse_pauli("X0 Y1 Z2", 3) == (x, z)


def test_parse_e4_strings():
    # Worked example (Eq. eg_diag_hami): binary forms printed in the text.
    printed = {"YIXI": "10101000", "IXIY": "01010001", "XZYZ": "10100111",
               "YZXZ": "10101101"}
    for s, bits in printed.items():
        x, z = oracle.parse_pauli(s, 4)
        got = "".join(str((x >> q) & 1) for q in range(4)) + \
            "".join(str((z >> q) & 1) for q in range(4))
        assert got == bits


def test_parse_rejects():
    for bad in ["XQ", "X0 X0", "X9"]:
        with pytest.raises(ValueError):
            oracle.parse_pauli(bad, 2)


# --- commutation vs dense matrices ----------------------------------------
def test_commutation_matches_dense():
    rng = np.random.default_rng(1)
    n = 4
    ps = rand_paulis(rng, n, 40)
    for a, b in itertools.combinations(ps, 2):
        A, B = dense.pauli_matrix(a), dense.pauli_matrix(b)
        dense_comm = np.allclose(A @ B, B @ A)
        xa, za = oracle.parse_pauli(a, n)
        xb, zb = oracle.parse_pauli(b, n)
        assert oracle.commutes(xa, za, xb, zb) == dense_comm


# --- single rotations vs expm ---------------------------------------------
@pytest.mark.parametrize("n", [1, 3, 5])
def test_rotation_matches_expm(n):
    rng = np.random.default_rng(10 + n)
    psi0 = workloads.random_state(n, 7)
    for s in rand_paulis(rng, n, 12):
        theta = float(rng.uniform(-2, 2))
        x, z = oracle.parse_pauli(s, n)
        got = oracle.evolve_terms_dense(n, [x], [z], [theta], psi0)
        ref = dense.expm(-1j * theta * dense.pauli_matrix(s)) @ psi0
        assert np.abs(got - ref).max() < 1e-13, s


# --- grouped Trotter step vs dense products --------------------------------
@pytest.mark.parametrize("order", [1, 2])
def test_trotter_step_matches_dense_groups(order):
    rng = np.random.default_rng(5 + order)
    n = 5
    ps = rand_paulis(rng, n, 14)
    cs = rng.normal(size=len(ps))
    t = oracle.build_terms(n, ps, cs)
    groups = oracle.first_fit_groups(t)
    assert len(groups) > 2
    dt, steps = 0.07, 3
    psi0 = workloads.random_state(n, 3)
    got = oracle.evolve(n, ps, cs, psi0, dt, steps, order)
    # dense: each group's exponential, composed in the Strang / sequential order
    hs = []
    for g in groups:
        hs.append(sum(t.c[k] * dense.pauli_matrix(_dense_str(n, t.x[k], t.z[k]))
                      for k in g))
    if order == 1:
        seq = [(g, 1.0) for g in range(len(groups))]
    else:
        K = len(groups)
        seq = [(g, .5) for g in range(K - 1)] + [(K - 1, 1.0)] + \
            [(g, .5) for g in range(K - 2, -1, -1)]
    U = np.eye(1 << n, dtype=complex)
    for g, f in seq:
        U = dense.expm(-1j * dt * f * hs[g]) @ U
    ref = np.linalg.matrix_power(U, steps) @ psi0
    assert np.abs(got - ref).max() < 1e-12


def _dense_str(n, x, z):
    x, z = int(x), int(z)
    s = []
    for q in range(n):
        b = ((x >> q) & 1, (z >> q) & 1)
        s.append({(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}[b])
    return "".join(s)


def test_single_commuting_group_is_exact():
    # one commuting group => no Trotter error at any dt (Eq. trotter_simul_diag)
    ps = ["YIXI", "IXIY", "XZYZ", "YZXZ", "XIYI", "IYIX", "ZXZY", "ZYZX"]
    rng = np.random.default_rng(2)
    cs = rng.normal(size=len(ps))
    t = oracle.build_terms(4, ps, cs)
    assert len(oracle.first_fit_groups(t)) == 1
    psi0 = workloads.random_state(4, 4)
    T = 1.3
    for dt, steps in [(1.3, 1), (0.13, 10)]:
        got = oracle.evolve(4, ps, cs, psi0, dt, steps, 1)
        ref = dense.expm(-1j * T * dense.hamiltonian(ps, cs)) @ psi0
        assert np.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("order,slope,n0", [(1, 2.0, 40), (2, 4.0, 40), (4, 16.0, 8)])
def test_trotter_error_order(order, slope, n0):
    # global error ~ dt^order: halving dt divides it by 2^order
    m = workloads.tfim_chain(6)
    psi0 = m.initial_state()
    T = 0.8
    ref = dense.expm(-1j * T * dense.hamiltonian(m.paulis, m.coeffs)) @ psi0
    errs = []
    for steps in (n0, 2 * n0):
        got = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, T / steps, steps, order)
        errs.append(np.linalg.norm(got - ref))
    ratio = errs[0] / errs[1]
    assert abs(ratio - slope) < 0.15 * slope, (errs, ratio)


# --- closed forms -------------------------------------------------------------
def test_x_only_field_is_product_state():
    n = 6
    h = np.linspace(-1, 1, n)
    ps = ["I" * q + "X" + "I" * (n - q - 1) for q in range(n)]
    T = 0.9
    got = oracle.evolve(n, ps, h, workloads.basis_state(n, 0), T / 7, 7, 1)
    ref = np.array([1.0 + 0j])
    for q in range(n - 1, -1, -1):
        ref = np.kron(ref, np.array([np.cos(h[q] * T), -1j * np.sin(h[q] * T)]))
    assert np.abs(got - ref).max() < 1e-13


def test_all_z_is_diagonal_phase():
    n = 7
    rng = np.random.default_rng(8)
    ps = []
    for _ in range(20):
        ps.append("".join("IZ"[int(rng.integers(2))] for _ in range(n)))
    cs = rng.normal(size=len(ps))
    psi0 = workloads.random_state(n, 9)
    T = 2.1
    got = oracle.evolve(n, ps, cs, psi0, T / 3, 3, 2)
    t = oracle.build_terms(n, ps, cs)
    phase = np.zeros(1 << n)
    for x in range(1 << n):
        for k in range(len(t.c)):
            phase[x] += t.c[k] * (-1) ** bin(x & int(t.z[k])).count("1")
    ref = np.exp(-1j * T * phase) * psi0
    assert np.abs(got - ref).max() < 1e-12


# --- invariants ------------------------------------------------------------------
def test_norm_conserved_and_group_order_invariance():
    m = workloads.random_klocal(n=10, m=120, seed=11, init_seed=12)
    psi0 = m.initial_state()
    t = oracle.build_terms(m.n, m.paulis, m.coeffs)
    groups = oracle.first_fit_groups(t)
    a = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, 0.05, 4, 1, groups=groups, terms=t)
    assert abs(np.vdot(a, a).real - 1) < 1e-12
    rng = np.random.default_rng(0)
    shuffled = [list(rng.permutation(g)) for g in groups]
    b = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, 0.05, 4, 1, groups=shuffled, terms=t)
    assert np.abs(a - b).max() < 1e-13
    # a different group order is a different product formula
    c = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, 0.05, 4, 1, groups=groups[::-1], terms=t)
    assert np.abs(a - c).max() > 1e-6


def test_energy_matches_dense():
    rng = np.random.default_rng(4)
    n = 5
    ps = rand_paulis(rng, n, 10)
    cs = rng.normal(size=len(ps))
    psi = workloads.random_state(n, 5)
    e = oracle.energy(n, ps, cs, psi)
    ref = np.vdot(psi, dense.hamiltonian(ps, cs) @ psi).real
    assert abs(e - ref) < 1e-12


@pytest.mark.parametrize("n,seed", [(3, 11), (5, 12), (6, 13)])
def test_term_expectations_match_dense(n, seed):
    # <psi|P_k|psi> of every merged term against the dense Pauli matrix
    # (Kronecker products of the 2x2 matrices), for input lists with exact
    # duplicates (merged at the first occurrence), identity strings and
    # strings with several Y factors (the i^{#Y} phase: a real expectation
    # needs it); the results come back in merged-term order.
    rng = np.random.default_rng(seed)
    ps = rand_paulis(rng, n, 14)
    ps += [ps[3], "I" * n, ps[0], "Y" * n, ps[7]]
    cs = rng.normal(size=len(ps))
    psi = workloads.random_state(n, seed + 100)
    t = oracle.build_terms(n, ps, cs)
    got = oracle.term_expectations(n, ps, cs, psi)
    assert got.shape == (len(t.c),) and len(t.c) < len(ps)
    first = {}
    for i, p in enumerate(ps):
        first.setdefault(p, i)
    for k, src in enumerate(t.source):
        s = ps[int(src)]
        assert first[s] == int(src)
        want = np.vdot(psi, dense.pauli_matrix(s) @ psi)
        assert abs(want.imag) < 1e-12
        assert abs(got[k] - want.real) < 1e-13, (k, s, got[k], want)
    # identity term: <psi|psi> = 1
    k_id = [k for k, src in enumerate(t.source) if ps[int(src)] == "I" * n][0]
    assert abs(got[k_id] - 1.0) < 1e-13
    # the coefficient-weighted sum is the energy, and both match the dense
    # expectation of H (merged coefficients)
    e_dense = np.vdot(psi, dense.hamiltonian(ps, cs) @ psi).real
    assert abs(float(np.dot(t.c, got)) - e_dense) < 1e-12
    assert abs(oracle.energy(n, ps, cs, psi) - e_dense) < 1e-12
    # a basis state: every term with an X part has expectation 0, a Z string
    # has (-1)^{popcount(x & zmask)}
    x0 = int(rng.integers(1 << n))
    b = workloads.basis_state(n, x0)
    gb = oracle.term_expectations(n, ps, cs, b)
    for k in range(len(t.c)):
        want = 0.0 if int(t.x[k]) else (-1.0) ** bin(x0 & int(t.z[k])).count("1")
        assert gb[k] == want


def test_energy_conserved_by_single_group():
    ps = ["ZZII", "IZZI", "IIZZ", "ZIIZ"]
    cs = [0.3, -0.7, 1.1, 0.2]
    psi = workloads.random_state(4, 1)
    e0 = oracle.energy(4, ps, cs, psi)
    psi1 = oracle.evolve(4, ps, cs, psi, 0.3, 5, 1)
    assert abs(oracle.energy(4, ps, cs, psi1) - e0) < 1e-12


# --- grouping counts fixed by the paper / the workload definitions -----------
def test_grouping_counts():
    m1 = workloads.tfim_chain(12)
    g1 = oracle.first_fit_groups(oracle.build_terms(m1.n, m1.paulis, m1.coeffs))
    assert [len(g) for g in g1] == [11, 12]
    m2 = workloads.xxz_chain(26)
    g2 = oracle.first_fit_groups(oracle.build_terms(m2.n, m2.paulis, m2.coeffs))
    assert [len(g) for g in g2] == [26, 26, 52]
    # fully connected TFIM: two groups (paper, Sec. "Transverse Field Ising Model")
    m3 = workloads.tfim_fully_connected(10)
    g3 = oracle.first_fit_groups(oracle.build_terms(m3.n, m3.paulis, m3.coeffs))
    assert len(g3) == 2 and len(m3.paulis) == 10 * 9 // 2 + 10


def test_tfim_term_count_n30():
    # the paper quotes 465 terms at 30 qubits
    assert workloads.tfim_fully_connected(30).m == 465


def test_duplicate_merge():
    t = oracle.build_terms(2, ["XZ", "ZZ", "XZ"], [1.0, 2.0, 0.5])
    assert len(t.c) == 2 and t.c[0] == 1.5 and list(t.source) == [0, 1]


def test_fidelity():
    a = workloads.random_state(5, 1)
    assert abs(oracle.fidelity(a, 2j * a) - 1) < 1e-14
    b = workloads.random_state(5, 2)
    assert oracle.fidelity(a, b) < 0.5


# --- sampled outputs on a coset: pinned to the full-state rotation loops ----
@pytest.mark.parametrize("seed,rho,extra", [(1, 4, 0), (2, 6, 1), (3, 7, 2)])
def test_apply_on_coset_matches_full_state(seed, rho, extra):
    # a commuting group with Y, Z and X factors; the coset basis is given as
    # random combinations of the X span (plus `extra` further vectors, a
    # larger invariant subspace), so the coordinates of each X mask are not
    # read off directly
    from tests import groups
    rng = np.random.default_rng(seed)
    n = 10
    ps, cs = groups.commuting_group(rng, n, rho, 14)
    t = oracle.build_terms(n, ps, cs)
    xs = [int(v) for v in t.x]
    zs = [int(v) for v in t.z]
    thetas = list(0.37 * t.c)
    basis = []

    def indep(v, vs):
        rows = []
        for w in vs + [v]:
            for r in rows:
                w = min(w, w ^ r)
            if w == 0:
                return False
            rows.append(w)
        return True

    for v in xs:
        if v and indep(v, basis):
            basis.append(v)
    while len(basis) < rho + extra:
        v = int(rng.integers(1, 1 << n))
        if indep(v, basis):
            basis.append(v)
    # random invertible recombination of the basis
    mixed = list(basis)
    for _ in range(20):
        i, j = rng.choice(len(mixed), 2, replace=False)
        mixed[i] ^= mixed[j]
    psi = workloads.random_state(n, seed)
    full = oracle.evolve_terms_dense(n, xs, zs, thetas, psi)
    for x0 in rng.integers(0, 1 << n, size=4):
        idx = np.zeros(1 << len(mixed), dtype=np.int64)
        for jj in range(1 << len(mixed)):
            v = int(x0)
            for i, b in enumerate(mixed):
                if (jj >> i) & 1:
                    v ^= b
            idx[jj] = v
        got = oracle.apply_on_coset(xs, zs, thetas, int(x0), mixed, psi[idx])
        assert np.abs(got - full[idx]).max() < 1e-13


# --- the SYK workload (the paper's second experiment) -----------------------
def test_syk_majorana_terms_match_dense_products():
    # Jordan-Wigner Majoranas built as dense matrices: they anticommute and
    # square to one, and every generated term equals g_abcd c_a c_b c_c c_d
    import math
    n = 3
    c = []
    for q in range(n):
        zs = {p: dense.Z for p in range(q)}
        c.append(dense.kron_ops(n, {**zs, q: dense.X}))
        c.append(dense.kron_ops(n, {**zs, q: dense.Y}))
    eye = np.eye(1 << n)
    for a in range(2 * n):
        for b in range(2 * n):
            assert np.allclose(c[a] @ c[b] + c[b] @ c[a], 2 * eye * (a == b))
    m = workloads.syk_majorana(n, seed=6)
    assert m.m == math.comb(2 * n, 4)
    g = np.random.default_rng(6).normal(size=m.m)
    for t, quad in enumerate(itertools.combinations(range(2 * n), 4)):
        prod = c[quad[0]] @ c[quad[1]] @ c[quad[2]] @ c[quad[3]]
        assert np.allclose(m.coeffs[t] * dense.pauli_matrix(m.paulis[t]), g[t] * prod)
    assert workloads.syk_majorana(6).m == math.comb(12, 4)


def test_fourth_order_schedule_is_symmetric_and_sums_to_dt():
    # Suzuki's fractal: every group's fractions add up to one step, and the
    # sequence reads the same backwards (a symmetric product formula)
    for K in (1, 2, 5):
        seq = oracle.schedule(K, 4)
        for g in range(K):
            assert abs(sum(f for h, f in seq if h == g) - 1.0) < 1e-14
        assert [h for h, _ in seq] == [h for h, _ in reversed(seq)]
        assert all(abs(a[1] - b[1]) < 1e-15 for a, b in zip(seq, reversed(seq)))


def test_trotter_energy_error_is_bounded_and_of_the_right_order():
    # a product formula of order p conserves a Hamiltonian within O(dt^p) of
    # H, so <H> oscillates within O(dt^p) of its start instead of drifting:
    # halving dt shrinks the largest deviation ~2x (order 1) and ~4x
    # (order 2), and the second half of a long run stays near the first
    # (open XXZ chain, three groups, T = 20)
    m = workloads.xxz_chain(n=8)
    psi0 = workloads.random_state(8, 3)
    e0 = oracle.energy(8, m.paulis, m.coeffs, psi0)
    for order, lo, hi in ((1, 1.6, 2.5), (2, 3.2, 5.0)):
        dev = {}
        for dt in (0.1, 0.05):
            k = int(round(0.5 / dt))
            psi = psi0.copy()
            d = []
            for _ in range(40):
                psi = oracle.evolve(8, m.paulis, m.coeffs, psi, dt, k, order)
                d.append(abs(oracle.energy(8, m.paulis, m.coeffs, psi) - e0))
            dev[dt] = np.array(d)
            assert dev[dt][20:].max() <= 1.8 * dev[dt][:20].max(), (order, dt)
        ratio = dev[0.1].max() / dev[0.05].max()
        assert lo < ratio < hi, (order, ratio)
