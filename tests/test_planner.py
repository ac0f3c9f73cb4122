"""Host-side planner tests through the C ABI (no GPU calls): parsing, grouping
bit-exact against the oracle, the paper's worked examples, brute-force
checks that every synthesised Clifford diagonalises its group, and two
emulations against the oracle: of the compiled tile programs as described,
and of the register-round kernel algorithm that runs them on the GPU."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from paper_2206_11664_amd import sd
from tests import dense, groups, round_emulator, tile_emulator

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _libs(oracle_lib):
    sd.lib()


def plan_for(n, paulis, coeffs, **opt):
    o = sd.sd_plan_options_default()
    if any(k.startswith("tile_log2") for k in opt):
        o.small_state_tiles = 0  # (a test asking for a tile size gets that size)
    for k, v in opt.items():
        setattr(o, k, v)
    h = sd.sd_hamiltonian_create(n, paulis, coeffs)
    p = sd.sd_plan(h, o)
    return h, p


def groups_of(p):
    info = sd.sd_plan_info_get(p)
    return [list(sd.sd_plan_export_group(p, g).term_ids) for g in range(info.n_groups)]


def pauli_str(n, x, z):
    return "".join({(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}[((x >> q) & 1, (z >> q) & 1)]
                   for q in range(n))


# --- parsing ---------------------------------------------------------------------
def test_masks_bit_exact_vs_oracle():
    for m in (workloads.tfim_chain(12), workloads.xxz_chain(26),
              workloads.random_klocal(n=28), workloads.jw_fermionic(n=12, total=400)):
        h = sd.sd_hamiltonian_create(m.n, m.paulis, m.coeffs)
        n, x, z, c, src = sd.sd_hamiltonian_terms(h)
        t = oracle.build_terms(m.n, m.paulis, m.coeffs)
        assert n == m.n
        assert np.array_equal(x, t.x) and np.array_equal(z, t.z)
        assert np.array_equal(src, t.source)
        assert np.allclose(c, t.c, rtol=0, atol=1e-15)
        sd.sd_hamiltonian_destroy(h)


def test_sparse_and_dense_forms_agree():
    h1 = sd.sd_hamiltonian_create(5, ["X0 Y3 Z4", "Z1"], [1.0, 2.0])
    h2 = sd.sd_hamiltonian_create(5, ["XIIYZ", "IZIII"], [1.0, 2.0])
    a, b = sd.sd_hamiltonian_terms(h1), sd.sd_hamiltonian_terms(h2)
    assert all(np.array_equal(u, v) for u, v in zip(a[1:], b[1:]))


@pytest.mark.parametrize("bad,status", [(["XQ"], sd.SD_ERR_PARSE), (["X0 X0"], sd.SD_ERR_PARSE),
                                        (["X7"], sd.SD_ERR_RANGE), (["XXX"], sd.SD_ERR_PARSE)])
def test_parse_errors(bad, status):
    with pytest.raises(sd.SdError) as e:
        sd.sd_hamiltonian_create(2, bad, [1.0])
    assert e.value.status == status


def test_argument_errors():
    with pytest.raises(sd.SdError) as e:
        sd.sd_hamiltonian_create(64, ["X0"], [1.0])
    assert e.value.status == sd.SD_ERR_RANGE
    with pytest.raises(sd.SdError) as e:
        sd.sd_hamiltonian_create(2, ["X0"], [float("nan")])
    assert e.value.status == sd.SD_ERR_ARG
    with pytest.raises(sd.SdError) as e:
        sd.sd_hamiltonian_create_masks(2, [4], [0], [1.0])
    assert e.value.status == sd.SD_ERR_RANGE
    o = sd.sd_plan_options_default()
    o.tile_log2_c64 = 20
    h = sd.sd_hamiltonian_create(2, ["XX"], [1.0])
    with pytest.raises(sd.SdError) as e:
        sd.sd_plan(h, o)
    assert e.value.status == sd.SD_ERR_RANGE


# --- grouping ------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["tfim", "xxz", "klocal", "jw", "tfim_fc"])
def test_grouping_bit_exact_vs_oracle(which):
    m = {"tfim": lambda: workloads.tfim_chain(12),
         "xxz": lambda: workloads.xxz_chain(26),
         "klocal": lambda: workloads.random_klocal(n=28),
         "jw": lambda: workloads.jw_fermionic(n=16, total=1500),
         "tfim_fc": lambda: workloads.tfim_fully_connected(20)}[which]()
    h, p = plan_for(m.n, m.paulis, m.coeffs)
    got = groups_of(p)
    want = oracle.first_fit_groups(oracle.build_terms(m.n, m.paulis, m.coeffs))
    assert got == want
    sd.sd_plan_destroy(p)
    sd.sd_hamiltonian_destroy(h)


# --- the paper's worked examples -----------------------------------------------------
def test_e5_independent_set():
    g = json.load(open(os.path.join(GOLD, "e5_independent_set.json")))
    h, p = plan_for(g["n"], g["terms"], [1.0] * len(g["terms"]))
    assert len(groups_of(p)) == 1
    ex = sd.sd_plan_export_group(p, 0)
    assert [int(i) + 1 for i in ex.independent] == g["independent_rows_1based"]


def _zstr_to_mask(s):
    sign = -1 if s[0] == "-" else 1
    body = s[1:]
    mask = 0
    for tok in body.split("Z")[1:]:
        mask |= 1 << (int(tok) - 1)
    return sign, mask


def test_e4_circuit_and_diagonal_form():
    g = json.load(open(os.path.join(GOLD, "e4_diagonalization.json")))
    h, p = plan_for(g["n"], g["terms"], [1.0] * len(g["terms"]))
    assert len(groups_of(p)) == 1
    ex = sd.sd_plan_export_group(p, 0)
    assert list(ex.independent) == g["independent_terms"]
    gates = ex.gates
    c = g["circuit_paper_1based"]
    # layers in application order: H (step i), CNOT, CZ/S, H (step iv)
    kinds = [k for k, _, _ in gates]
    nh1 = len(c["H_first"])
    assert sorted(a + 1 for k, a, _ in gates[:nh1] if k == "H") == c["H_first"]
    rest = gates[nh1:]
    cn = [(a + 1, b + 1) for k, a, b in rest if k == "CNOT"]
    assert cn == [tuple(v) for v in c["CNOT"]]
    cz = sorted((a + 1, b + 1) for k, a, b in rest if k == "CZ")
    assert cz == sorted(tuple(v) for v in c["CZ"])
    s = sorted(a + 1 for k, a, _ in rest if k == "S")
    assert s == c["S"]
    tail = [a + 1 for k, a, _ in gates[-4:]]
    assert all(k == "H" for k in kinds[-4:]) and sorted(tail) == c["H_last"]
    assert len(gates) == nh1 + len(c["CNOT"]) + len(c["CZ"]) + len(c["S"]) + 4
    for k, want in enumerate(g["diagonal_paper"]):
        sign, mask = _zstr_to_mask(want)
        assert int(ex.zmask[k]) == mask, (k, want)
        assert (-1) ** int(ex.sign[k]) == sign, (k, want)


# --- brute force: every synthesised circuit diagonalises its group --------------------
def random_commuting_hamiltonian(rng, n, m):
    out = []
    while len(out) < m:
        s = "".join("IXYZ"[int(rng.integers(4))] for _ in range(n))
        out.append(s)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_paper_circuits_diagonalise_dense(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 7))
    ps = random_commuting_hamiltonian(rng, n, 30)
    cs = rng.normal(size=len(ps))
    h, p = plan_for(n, ps, cs)
    t = oracle.build_terms(n, ps, cs)
    for gi, g in enumerate(groups_of(p)):
        ex = sd.sd_plan_export_group(p, gi)
        C = dense.circuit_matrix(n, ex.gates)
        for j, k in enumerate(g):
            P = dense.pauli_matrix(pauli_str(n, int(t.x[k]), int(t.z[k])))
            want = (-1) ** int(ex.sign[j]) * dense.zstring(n, int(ex.zmask[j]))
            assert np.allclose(C @ P @ C.conj().T, want, atol=1e-12), (gi, j)


def test_paper_circuits_diagonalise_large_groups():
    # n = 28 random k-local groups: propagate each Pauli through the gate list
    # with the single- and two-qubit conjugation tables, qubit by qubit.
    m = workloads.random_klocal(n=28)
    h, p = plan_for(m.n, m.paulis, m.coeffs)
    n, x, z, c, _ = sd.sd_hamiltonian_terms(h)
    for gi, g in enumerate(groups_of(p)):
        ex = sd.sd_plan_export_group(p, gi)
        for j, k in enumerate(g):
            ph, xx, zz = _propagate(int(x[k]), int(z[k]), ex.gates)
            assert xx == 0 and zz == int(ex.zmask[j])
            assert ph == (2 if ex.sign[j] else 0)


def _propagate(x, z, gates):
    """U P U^dagger gate by gate, with P = i^{phase} prod_q sigma(x_q, z_q)
    (sigma(1,1) = Y).  Single-qubit images: H: X->Z, Z->X, Y->-Y;  S: X->Y,
    Y->-X, Z->Z.  CNOT(c,t): X_c->X_c X_t, Z_t->Z_c Z_t, X_t, Z_c fixed.
    CZ(a,b): X_a->X_a Z_b, X_b->Z_a X_b.  Products are multiplied out with the
    single-qubit Pauli multiplication table."""
    # represent as dict qubit -> letter, plus phase (power of i)
    n = 64
    P = {q: _letter((x >> q) & 1, (z >> q) & 1) for q in range(n) if ((x | z) >> q) & 1}
    phase = 0
    for kind, a, b in gates:
        if kind in ("H", "S"):
            l = P.get(a, "I")
            img = {"H": {"X": (0, "Z"), "Z": (0, "X"), "Y": (2, "Y")},
                   "S": {"X": (0, "Y"), "Y": (2, "X"), "Z": (0, "Z")}}[kind].get(l)
            if img:
                phase += img[0]
                P[a] = img[1]
        else:
            la, lb = P.get(a, "I"), P.get(b, "I")
            # images of the generators on (a, b)
            if kind == "CNOT":
                gen = {"Xa": ("X", "X"), "Za": ("Z", "I"), "Xb": ("I", "X"), "Zb": ("Z", "Z")}
            else:
                gen = {"Xa": ("X", "Z"), "Za": ("Z", "I"), "Xb": ("Z", "X"), "Zb": ("I", "Z")}
            # decompose la (x) lb = i^{#Y} X^xa Z^za X^xb Z^zb (order X_a Z_a X_b Z_b)
            xa, za = _bits(la)
            xb, zb = _bits(lb)
            ph = (xa & za) + (xb & zb)
            cur = ("I", "I")
            for use, gname in ((xa, "Xa"), (za, "Za"), (xb, "Xb"), (zb, "Zb")):
                if use:
                    g = gen[gname]
                    p1, r1 = _mul(cur[0], g[0])
                    p2, r2 = _mul(cur[1], g[1])
                    ph += p1 + p2
                    cur = (r1, r2)
            phase += ph
            P[a], P[b] = cur
    xx = zz = 0
    for q, l in P.items():
        bx, bz = _bits(l)
        xx |= bx << q
        zz |= bz << q
    # P = i^{phase} prod sigma; a Z-string has no Y, so nothing to convert
    return phase % 4, xx, zz


def _letter(bx, bz):
    return {(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}[(bx, bz)]


def _bits(l):
    return {"I": (0, 0), "X": (1, 0), "Z": (0, 1), "Y": (1, 1)}[l]


def _mul(a, b):
    """a*b = i^k c for single-qubit Paulis."""
    if a == "I":
        return 0, b
    if b == "I":
        return 0, a
    if a == b:
        return 0, "I"
    cyc = {("X", "Y"): "Z", ("Y", "Z"): "X", ("Z", "X"): "Y"}
    if (a, b) in cyc:
        return 1, cyc[(a, b)]
    return 3, cyc[(b, a)]


def test_tableau_tables_by_dense_conjugation():
    # the paper's single- and two-qubit conjugation tables, checked with matrices
    H, S = dense.H, dense.S
    X, Y, Z = dense.X, dense.Y, dense.Z
    assert np.allclose(H @ X @ H.conj().T, Z) and np.allclose(H @ Y @ H.conj().T, -Y)
    assert np.allclose(S @ X @ S.conj().T, Y) and np.allclose(S @ Y @ S.conj().T, -X)
    CN = dense.cnot(2, 0, 1)
    k = dense.kron_ops
    assert np.allclose(CN @ k(2, {1: Z}) @ CN.T, k(2, {0: Z, 1: Z}))   # I1 Z2 -> Z1 Z2
    assert np.allclose(CN @ k(2, {0: Y, 1: Y}) @ CN.T, -k(2, {0: X, 1: Z}))
    # and the propagation helper used above agrees on every 2-qubit Pauli
    for l1 in "IXYZ":
        for l2 in "IXYZ":
            for gate in (("CNOT", 0, 1), ("CZ", 0, 1), ("H", 0, -1), ("S", 1, -1)):
                x = (l1 in "XY") | ((l2 in "XY") << 1)
                z = (l1 in "ZY") | ((l2 in "ZY") << 1)
                ph, xx, zz = _propagate(x, z, [gate])
                U = dense.gate_matrix(2, gate)
                P = dense.pauli_matrix(l1 + l2)
                want = (1j) ** ph * dense.pauli_matrix(pauli_str(2, xx, zz))
                assert np.allclose(U @ P @ U.conj().T, want)


# --- tile programs vs the oracle (emulated on the CPU) ---------------------------------
@pytest.mark.parametrize("case", ["klocal", "xxz", "tfim", "jw", "rand"])
@pytest.mark.parametrize("dtype", [sd.SD_C64, sd.SD_C128])
def test_tile_program_emulation_matches_oracle(case, dtype):
    rng = np.random.default_rng(7)
    if case == "klocal":
        m = workloads.random_klocal(n=9, m=60, seed=5, init_seed=6)
        opts = dict(tile_log2_c64=6, tile_log2_c128=6, coalesce_log2_c64=2, coalesce_log2_c128=1)
    elif case == "xxz":
        m = workloads.xxz_chain(n=8, steps=3)
        opts = dict(tile_log2_c64=6, tile_log2_c128=7)
    elif case == "tfim":
        m = workloads.tfim_chain(7)
        opts = {}
    elif case == "jw":
        m = workloads.jw_fermionic(n=8, total=120)
        opts = dict(tile_log2_c64=7, tile_log2_c128=6)
    else:
        m = workloads.random_klocal(n=8, m=40, seed=9, init_seed=1)
        m.paulis = random_commuting_hamiltonian(rng, 8, 40)
        opts = dict(tile_log2_c64=6, tile_log2_c128=6)
    h, p = plan_for(m.n, m.paulis, m.coeffs, **opts)
    info = sd.sd_plan_info_get(p)
    passes = [sd.sd_plan_export_pass(p, dtype, i) for i in range(sd.sd_plan_pass_count(p, dtype))]
    psi0 = workloads.random_state(m.n, 3)
    order = 2 if case == "xxz" else 1
    got = tile_emulator.evolve(psi0, m.n, passes, [q["group"] for q in passes], info.n_groups,
                               0.11, 3, order)
    want = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, 0.11, 3, order)
    assert np.abs(got - want).max() < 1e-12


# --- the register-round kernel algorithm (emulated on the CPU) -------------------------
def _export_all(p, dtype):
    cnt = sd.sd_plan_pass_count(p, dtype)
    return ([sd.sd_plan_export_pass(p, dtype, i) for i in range(cnt)],
            [sd.sd_plan_export_rounds(p, dtype, i) for i in range(cnt)])


def _check_round_structure(ps, rv):
    """Chunks hold consecutive span coordinates (register slots first, then
    the exchanged lane coordinates), a CZ inside a chunk only between its
    register slots (exported as the round's sign mask); fillers are never
    span coordinates of a later chunk; the only S sits in register slot 0 of
    the Lambda round; round 0's leading lanes are the lowest address bits."""
    rho, B = ps["rho"], [int(v) for v in ps["cz_s"]]
    D = ps["tile_log2"]
    nr = rv["n_rounds"]
    if rho == 0:
        assert nr == 0
        return
    seen = []
    for r in range(nr):
        nb = bin(rv["bmask"][r]).count("1")
        nx = rv["nx"][r]
        assert rv["bmask"][r] == (1 << nb) - 1 and 1 <= nb <= 4 and 0 <= nx <= 2
        assert nx == 0 or nb == 4
        coords = [rv["reg"][r][l] for l in range(nb)] + [rv["xl"][r][x] for x in range(nx)]
        assert coords == list(range(len(seen), len(seen) + nb + nx))
        seen += coords
        cm = sum(1 << a for a in coords)
        regs = coords[:4]
        czm = 0
        for l1 in range(len(regs)):
            for l2 in range(l1 + 1, len(regs)):
                if (B[regs[l1]] >> regs[l2]) & 1:
                    for g in range(16):
                        if (g >> l1) & (g >> l2) & 1:
                            czm ^= 1 << g
        assert rv["czmask"][r] == czm
        for l, a in enumerate(coords):
            if l >= 4:
                assert B[a] & cm & ~(1 << a) == 0, "CZ inside a chunk outside its register slots"
            assert ((rv["iflag"][r] >> l) & 1) == ((B[a] >> a) & 1)
            assert ((rv["dflag"][r] >> l) & 1) == ((ps["z_sign"] >> a) & 1)
            if (B[a] >> a) & 1:
                assert r == nr - 1 and l == 0
        assert rv["later"][r] == sum(1 << b for b in range(len(seen), rho))
        for l in range(nb, 4):
            assert not (rv["later"][r] >> rv["reg"][r][l]) & 1
        post = list(rv["reg"][r])
        for x in range(nx):
            post[2 + x] = rv["xl"][r][x]
        assert rv["regpost"][r] == post
        # lane vectors: with the register slots they span the tile
        vecs = [1 << q for q in rv["reg"][r]] + list(rv["lanes"][r])
        assert _rank(vecs) == D
        assert rv["lanes"][r][4:4 + nx] == [1 << rv["xl"][r][x] for x in range(nx)]
    assert seen == list(range(rho)) and rv["lam_round"] == nr - 1
    bk = rv["bucket"]
    assert bk[0] == 0 and bk[16] == len(ps["coef"]) and all(bk[w] <= bk[w + 1] for w in range(16))
    k = rv["io_coalesced"]
    assert rv["lanes"][0][:k] == [int(v) for v in ps["pivot_coord"][:k]]
    c = min(ps["coalesce_log2"], 4)
    assert (k == c) != bool(rv["staged"])
    # round 0 writes its outputs without the lanes' components along its own
    # coordinates; every layout spans the tile
    nb0 = bin(rv["bmask"][0]).count("1")
    c0 = sum(1 << a for a in range(nb0 + rv["nx"][0]))
    assert rv["lanes_post"][0][:k] == [v & ~c0 for v in rv["lanes"][0][:k]]
    assert bool(rv["shift0"]) == any(v & c0 for v in rv["lanes"][0][:k])
    for r in range(nr):
        assert _rank([1 << q for q in rv["regpost"][r]] + list(rv["lanes_post"][r])) == D


def _rank(vs):
    basis = []
    for v in vs:
        for b in basis:
            v = min(v, v ^ b)
        if v:
            basis.append(v)
    return len(basis)


@pytest.mark.parametrize("seed,rho,alt", [(1, 9, False), (2, 9, True), (3, 8, True), (4, 6, True),
                                          (5, 3, True), (6, 12, False), (7, 11, True),
                                          (8, 13, False), (9, 13, True)])
def test_register_rounds_large_group_matches_oracle(seed, rho, alt):
    # one commuting group of X-span rank rho (alternating: its CZ/S form has no
    # S, so the planner has to split CZ pairs across chunks)
    rng = np.random.default_rng(seed)
    n = 14
    ps, cs = groups.commuting_group(rng, n, rho, 40, alternating=alt)
    h, p = plan_for(n, ps, cs, tile_log2_c64=13, tile_log2_c128=13, coalesce_log2_c64=0,
                    coalesce_log2_c128=0)
    info = sd.sd_plan_info_get(p)
    assert info.n_groups == 1
    passes, rounds = _export_all(p, sd.SD_C64)
    assert [q["rho"] for q in passes] == [rho]
    # canonical form: exactly one S when the form is not alternating, none
    # when it is
    n_s = sum((int(b) >> i) & 1 for i, b in enumerate(passes[0]["cz_s"]))
    assert n_s == (0 if alt else 1)
    for q, r in zip(passes, rounds):
        _check_round_structure(q, r)
    psi0 = workloads.random_state(n, 3)
    got = round_emulator.evolve(psi0, n, passes, rounds, info.n_groups, 0.07, 1, 1)
    want = oracle.evolve(n, ps, cs, psi0, 0.07, 1, 1)
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("case", ["klocal", "xxz", "jw", "wide", "n16"])
@pytest.mark.parametrize("dtype", [sd.SD_C64, sd.SD_C128])
def test_register_rounds_models_match_oracle(case, dtype):
    if case == "klocal":
        m, D = workloads.random_klocal(n=12, m=80, seed=5, init_seed=6), 10
    elif case == "xxz":
        m, D = workloads.xxz_chain(n=11, steps=3), 10
    elif case == "jw":
        m, D = workloads.jw_fermionic(n=11, total=150), 10
    elif case == "wide":
        m, D = workloads.random_klocal(n=15, m=300, seed=11, init_seed=2), 13
    else:
        m, D = workloads.random_klocal(n=16, m=400, seed=3, init_seed=30), 13
    h, p = plan_for(m.n, m.paulis, m.coeffs, tile_log2_c64=D, tile_log2_c128=D)
    info = sd.sd_plan_info_get(p)
    passes, rounds = _export_all(p, dtype)
    for q, r in zip(passes, rounds):
        _check_round_structure(q, r)
    if case == "n16":
        # passes whose round-0 lanes are shifted (direct I/O with the layout
        # and sign correction)
        assert any(r["shift0"] and not r["staged"] and r["n_rounds"] >= 2 for r in rounds)
    if case in ("klocal", "jw", "wide", "n16"):
        # rounds with a CZ between register slots of their chunk
        assert any(any(r["czmask"]) for r in rounds)
    psi0 = workloads.random_state(m.n, 3)
    got = round_emulator.evolve(psi0, m.n, passes, rounds, info.n_groups, 0.11, 1, 2)
    want = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, 0.11, 1, 2)
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("which", ["klocal28", "jw32", "xxz26"])
def test_register_round_structure_full_size(which):
    # every pass of the benchmark-size plans satisfies the round invariants
    m = {"klocal28": lambda: workloads.random_klocal(n=28),
         "jw32": lambda: workloads.jw_fermionic(n=32),
         "xxz26": lambda: workloads.xxz_chain(n=26)}[which]()
    h, p = plan_for(m.n, m.paulis, m.coeffs)
    for dtype in (sd.SD_C64, sd.SD_C128):
        passes, rounds = _export_all(p, dtype)
        for q, r in zip(passes, rounds):
            if q["tile_log2"] >= 10:
                _check_round_structure(q, r)



# plans with a shifted round 0 whose chunk also holds a CZ between register
# slots (the shift then also moves round 0's outputs, by M d(t))
SHIFT_CZ_CASES = [(12, 3, 300, 10, sd.SD_C64), (12, 19, 150, 10, sd.SD_C128),
                  (14, 14, 300, 13, sd.SD_C64)]


@pytest.mark.parametrize("n,seed,m,D,dtype", SHIFT_CZ_CASES)
def test_register_rounds_shift_with_cz_matches_oracle(n, seed, m, D, dtype):
    w = workloads.random_klocal(n=n, m=m, seed=seed, init_seed=2)
    h, p = plan_for(w.n, w.paulis, w.coeffs, tile_log2_c64=D, tile_log2_c128=D)
    info = sd.sd_plan_info_get(p)
    passes, rounds = _export_all(p, dtype)
    for q, r in zip(passes, rounds):
        _check_round_structure(q, r)
    assert any(r["shift0"] and not r["staged"] and r["czmask"][0] for r in rounds)
    psi0 = workloads.random_state(w.n, 3)
    got = round_emulator.evolve(psi0, w.n, passes, rounds, info.n_groups, 0.11, 1, 2)
    want = oracle.evolve(w.n, w.paulis, w.coeffs, psi0, 0.11, 1, 2)
    assert np.abs(got - want).max() < 1e-13


# --- sub-group splits ---------------------------------------------------------------
def _gf2_rank(vecs):
    basis = []  # reduced rows, distinct leading bits
    for v in vecs:
        v = int(v)
        for b in basis:
            v = min(v, v ^ b)
        if v:
            basis.append(v)
    return len(basis)


@pytest.mark.parametrize("which", ["klocal28", "jw32", "syk12", "tfim20", "klocal_small_tiles"]
                         + [f"fuzz{i}" for i in range(6)])
def test_subgroup_splits_partition_groups(which):
    # every group's passes (in plan order) hold each of the group's terms
    # exactly once; each pass's span is the rank of its terms' X parts and its
    # tile (those X parts and the low address bits) fits 2^tile_log2
    opt = {}
    if which == "klocal28":
        m = workloads.random_klocal(n=28)
    elif which == "jw32":
        m = workloads.jw_fermionic(n=32)
    elif which == "syk12":
        m = workloads.syk_majorana(12)
    elif which == "tfim20":
        m = workloads.tfim_fully_connected(20)
    elif which == "klocal_small_tiles":
        m = workloads.random_klocal(n=14, m=400, seed=11, init_seed=12)
        opt = dict(tile_log2_c64=10, tile_log2_c128=10, coalesce_log2_c64=3, coalesce_log2_c128=2)
    else:
        # tiny tiles: groups split into many sub-groups, so the split's local
        # moves (dissolving sub-groups, moving single terms) run often
        i = int(which[4:])
        m = workloads.random_klocal(n=10 + i, m=150 + 40 * i, seed=100 + i, init_seed=1)
        opt = dict(tile_log2_c64=6 + i % 3, tile_log2_c128=6 + i % 3,
                   coalesce_log2_c64=i % 3, coalesce_log2_c128=i % 2)
    h, p = plan_for(m.n, m.paulis, m.coeffs, **opt)
    _, xs, _, _, _ = sd.sd_hamiltonian_terms(h)
    info = sd.sd_plan_info_get(p)
    groups = groups_of(p)
    for dtype in (sd.SD_C64, sd.SD_C128):
        seen = [[] for _ in range(info.n_groups)]
        for i in range(sd.sd_plan_pass_count(p, dtype)):
            q = sd.sd_plan_export_pass(p, dtype, i)
            ids = [int(t) for t in q["term_ids"]]
            assert ids, "empty pass"
            seen[q["group"]].append(ids)
            x = [int(xs[t]) for t in ids]
            assert q["rho"] == _gf2_rank(x)
            low = [1 << b for b in range(q["coalesce_log2"])]
            assert _gf2_rank(x + low) <= q["tile_log2"]
        for g in range(info.n_groups):
            got = [t for ids in seen[g] for t in ids]
            assert sorted(got) == sorted(int(t) for t in groups[g]), f"group {g}"
        # (passes of a group are consecutive: group ids never decrease)
        order = [sd.sd_plan_export_pass(p, dtype, i)["group"] for i in range(sd.sd_plan_pass_count(p, dtype))]
        assert order == sorted(order)
    sd.sd_plan_destroy(p)
    sd.sd_hamiltonian_destroy(h)


def test_benchmark_split_cost_guard():
    # the n = 28 benchmark's complex64 plan: pass and register-round counts
    # (a regression guard on the sub-group split and the chunk packing)
    m = workloads.random_klocal(n=28)
    h, p = plan_for(m.n, m.paulis, m.coeffs)
    npass = sd.sd_plan_pass_count(p, sd.SD_C64)
    rounds = sum(sd.sd_plan_export_rounds(p, sd.SD_C64, i)["n_rounds"] for i in range(npass))
    assert npass <= 158 and rounds <= 277, (npass, rounds)
    sd.sd_plan_destroy(p)
    sd.sd_hamiltonian_destroy(h)


def test_jw_generator_rejects_impossible_totals():
    # asking for more distinct strings than exist raises instead of drawing forever
    with pytest.raises(ValueError):
        workloads.jw_fermionic(n=12)
    assert len(workloads.jw_fermionic(n=12, total=2000).paulis) == 2000


def _pass_tiles(p, dtype):
    return [sd.sd_plan_export_pass(p, dtype, i)["tile_log2"] for i in range(sd.sd_plan_pass_count(p, dtype))]


def test_small_state_tiles():
    # a state of fewer than 256 tiles of the requested size takes the
    # smallest tile (>= 2^10) that needs no more passes; a large state keeps
    # the requested size; the option off keeps it too
    m = workloads.tfim_fully_connected(14)
    for dtype in (sd.SD_C64, sd.SD_C128):
        h, p = plan_for(m.n, m.paulis, m.coeffs)
        h0, p0 = plan_for(m.n, m.paulis, m.coeffs, small_state_tiles=0)
        t, t0 = _pass_tiles(p, dtype), _pass_tiles(p0, dtype)
        assert len(t) == len(t0)
        assert max(t) < max(t0) and min(t) >= 10
        # the smallest such size: one below it needs more passes
        if max(t) > 10:
            h1, p1 = plan_for(m.n, m.paulis, m.coeffs, small_state_tiles=0,
                              **{("tile_log2_c64" if dtype == sd.SD_C64 else "tile_log2_c128"): max(t) - 1})
            assert len(_pass_tiles(p1, dtype)) > len(t)
            sd.sd_plan_destroy(p1)
            sd.sd_hamiltonian_destroy(h1)
        for q in (p, p0):
            sd.sd_plan_destroy(q)
        for g in (h, h0):
            sd.sd_hamiltonian_destroy(g)
    big = workloads.random_klocal(n=22, m=300, seed=3, init_seed=2)
    h, p = plan_for(big.n, big.paulis, big.coeffs)
    h0, p0 = plan_for(big.n, big.paulis, big.coeffs, small_state_tiles=0)
    for dtype in (sd.SD_C64, sd.SD_C128):
        assert _pass_tiles(p, dtype) == _pass_tiles(p0, dtype)
    for q in (p, p0):
        sd.sd_plan_destroy(q)
    for g in (h, h0):
        sd.sd_hamiltonian_destroy(g)


def test_shrink_never_adds_passes():
    # complex64 tile shrinking (smallest tile per pass, and each group split
    # again for tiles one or two coordinates smaller while that needs no more
    # passes) never needs more passes than one tile size for the whole plan;
    # at n = 28 the benchmark keeps its 139 passes and moves most of them off
    # 2^13 tiles
    cases = [(workloads.random_klocal(28), 139), (workloads.xxz_chain(26), None),
             (workloads.random_klocal(n=20, m=600, seed=7, init_seed=2), None),
             (workloads.jw_fermionic(n=16, total=900), None)]
    for m, want in cases:
        h, p = plan_for(m.n, m.paulis, m.coeffs)
        h0, p0 = plan_for(m.n, m.paulis, m.coeffs, tile_shrink_c64=0)
        t, t0 = _pass_tiles(p, sd.SD_C64), _pass_tiles(p0, sd.SD_C64)
        assert len(t) <= len(t0), (m.name, len(t), len(t0))
        if want is not None:
            assert len(t) == want and sum(1 for d in t if d < 13) > len(t) // 2, (len(t), t.count(13))
        for q in (p, p0):
            sd.sd_plan_destroy(q)
        for g in (h, h0):
            sd.sd_hamiltonian_destroy(g)
