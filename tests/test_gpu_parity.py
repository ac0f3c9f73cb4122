"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Bars (from the workload definitions): complex128 L2 error <= 1e-10; complex64
L2 error <= 1e-5 and fidelity >= 1 - 1e-6 (the complex64 bar is stated for
1000 steps; shorter runs must meet it too).
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import groups

torch = pytest.importorskip("torch")
from paper_2206_11664_amd import sd  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {sd.SD_C128: 1e-10, sd.SD_C64: 1e-5}
TDT = {sd.SD_C128: torch.complex128, sd.SD_C64: torch.complex64}


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sd.lib()


def gpu_evolve(m, psi0, dtype, dt, steps, order, opts=None, plan=None):
    print(f"[gpu] {m.name} n={m.n} dtype={dtype} steps={steps} order={order}", flush=True)
    if plan is None:
        o = sd.sd_plan_options_default()
        if any(k.startswith("tile_log2") for k in (opts or {})):
            o.small_state_tiles = 0  # (a test asking for a tile size gets that size)
        for k, v in (opts or {}).items():
            setattr(o, k, v)
        plan = sd.Plan(m.n, m.paulis, m.coeffs, o).bind()
    psi = torch.from_numpy(np.asarray(psi0, dtype=np.complex128)).to(TDT[dtype]).cuda()
    plan.evolve(psi, dt, steps, order)
    torch.cuda.synchronize()
    return psi.cpu().numpy().astype(np.complex128), plan


def l2(a, b):
    return float(np.linalg.norm(a - b))


def check(m, dtype, dt, steps, order, opts=None, psi0=None):
    psi0 = m.initial_state() if psi0 is None else psi0
    got, plan = gpu_evolve(m, psi0, dtype, dt, steps, order, opts)
    want = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, dt, steps, order)
    err = l2(got, want)
    assert err <= TOL[dtype], (m.name, dtype, err)
    if dtype == sd.SD_C64:
        assert oracle.fidelity(got, want) >= 1 - 1e-6
    return plan, got, want


@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_config1_tfim_chain_full(dtype):
    m = workloads.tfim_chain(12)
    check(m, dtype, m.dt, m.steps, m.order)


@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_xxz_periodic_order2(dtype):
    m = workloads.xxz_chain(n=14, steps=40)
    check(m, dtype, m.dt, m.steps, 2)


@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_random_klocal_reduced(dtype):
    m = workloads.random_klocal(n=16, m=400, seed=3, init_seed=30)
    check(m, dtype, 0.01, 10, 1)


@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_fourth_order_suzuki(dtype):
    # Suzuki's fourth-order fractal of Strang steps, against the oracle's own
    # schedule (several groups, and a single group)
    m = workloads.random_klocal(n=12, m=120, seed=31, init_seed=32)
    check(m, dtype, 0.07, 3, 4)
    m1 = workloads.xxz_chain(n=10, steps=2)
    m1.paulis = m1.paulis[: len(m1.paulis) // 4]
    m1.coeffs = m1.coeffs[: len(m1.paulis)]
    check(m1, dtype, 0.05, 2, 4)


@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_jw_fermionic_reduced(dtype):
    m = workloads.jw_fermionic(n=12, total=700)
    check(m, dtype, 0.02, 5, 2, psi0=workloads.random_state(12, 5))


@pytest.mark.parametrize("tile", [6, 8, 10, 13])
def test_tile_sizes_and_split_groups(tile):
    # small tiles force many tiles per pass and sub-group splits
    m = workloads.random_klocal(n=15, m=200, seed=8, init_seed=2)
    opts = dict(tile_log2_c64=tile, tile_log2_c128=tile)
    check(m, sd.SD_C128, 0.03, 3, 1, opts)
    check(m, sd.SD_C64, 0.03, 3, 1, opts)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_tiny_systems(n):
    rng = np.random.default_rng(n)
    ps = ["".join("IXYZ"[int(rng.integers(4))] for _ in range(n)) for _ in range(6)]
    m = workloads.Model("tiny", n, ps, rng.normal(size=6))
    psi0 = workloads.random_state(n, 1)
    for dt in (sd.SD_C128, sd.SD_C64):
        check(m, dt, 0.2, 4, 2, psi0=psi0)


def test_diagonal_only_and_identity_terms():
    n = 11
    ps = ["I" * n] + ["".join("IZ"[(q * 7 + k) % 3 == 0] for q in range(n)) for k in range(30)]
    m = workloads.Model("allz", n, ps, np.linspace(-1, 1, len(ps)))
    check(m, sd.SD_C128, 0.3, 3, 1, psi0=workloads.random_state(n, 2))


def test_empty_hamiltonian_is_identity():
    n = 6
    plan = sd.Plan(n, [], []).bind()
    psi0 = workloads.random_state(n, 4)
    psi = torch.from_numpy(psi0).cuda()
    plan.evolve(psi, 0.1, 5, 1)
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), psi0)


def test_expectation_matches_oracle():
    m = workloads.random_klocal(n=14, m=300, seed=4, init_seed=9)
    psi0 = m.initial_state()
    plan = sd.Plan(m.n, m.paulis, m.coeffs).bind()
    want = oracle.energy(m.n, m.paulis, m.coeffs, psi0)
    for dtype, tol in ((sd.SD_C128, 1e-10), (sd.SD_C64, 1e-5)):
        psi = torch.from_numpy(psi0).to(TDT[dtype]).cuda()
        e = plan.expectation(psi)
        assert abs(e - want) <= tol * max(1.0, abs(want)), (dtype, e, want)


def test_norm_and_inner():
    n = 17
    a = workloads.random_state(n, 1)
    b = workloads.random_state(n, 2)
    for dtype in (sd.SD_C128, sd.SD_C64):
        ta = torch.from_numpy(a).to(TDT[dtype]).cuda()
        tb = torch.from_numpy(b).to(TDT[dtype]).cuda()
        ref_a = ta.cpu().numpy().astype(np.complex128)
        ref_b = tb.cpu().numpy().astype(np.complex128)
        assert abs(sd.sd_norm2(ta, n) - np.vdot(ref_a, ref_a).real) < 1e-12
        ov = sd.sd_inner(ta, tb, n)
        assert abs(ov - np.vdot(ref_a, ref_b)) < 1e-12


def test_split_runs_are_bit_identical():
    m = workloads.random_klocal(n=15, m=250, seed=6, init_seed=7)
    plan = sd.Plan(m.n, m.paulis, m.coeffs).bind()
    psi0 = torch.from_numpy(m.initial_state()).to(torch.complex64).cuda()
    a = psi0.clone()
    plan.evolve(a, 0.02, 10, 1)
    b = psi0.clone()
    plan.evolve(b, 0.02, 5, 1)
    plan.evolve(b, 0.02, 5, 1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_c64_long_run_fidelity():
    # 1000 second-order steps, the complex64 bar's own length
    m = workloads.xxz_chain(n=12, steps=1000)
    check(m, sd.SD_C64, 0.05, 1000, 2)


def _random_state_torch(n, seed):
    g = torch.Generator().manual_seed(seed)
    re = torch.randn(1 << n, dtype=torch.float64, generator=g)
    im = torch.randn(1 << n, dtype=torch.float64, generator=g)
    psi = torch.complex(re, im)
    del re, im
    psi /= torch.linalg.vector_norm(psi)
    return psi


def test_full_size_n28_properties():
    # the benchmark workload at full size: time reversibility of the symmetric
    # second-order product, norm conservation, c64 against c128
    m = workloads.random_klocal(n=28)
    plan = sd.Plan(m.n, m.paulis, m.coeffs).bind()
    print("[gpu] n28 reversibility", flush=True)
    d128 = _random_state_torch(28, 11).cuda()
    a = d128.clone()
    plan.evolve(a, 0.01, 2, 2)
    plan.evolve(a, -0.01, 2, 2)
    torch.cuda.synchronize()
    assert float(torch.linalg.vector_norm(a - d128)) < 1e-10
    del a
    b = d128.clone()
    plan.evolve(b, 0.01, 2, 1)
    c = d128.to(torch.complex64)
    plan.evolve(c, 0.01, 2, 1)
    torch.cuda.synchronize()
    assert abs(sd.sd_norm2(b, 28) - 1) < 1e-12
    assert abs(sd.sd_norm2(c, 28) - 1) < 1e-5
    assert float(torch.linalg.vector_norm(c.to(torch.complex128) - b)) < 1e-5


def test_full_size_n28_widest_group_vs_oracle():
    # one application of the benchmark's widest commuting group (largest X
    # span, several tile passes) at n = 28, same tile configuration as the
    # benchmark, against the oracle on the full 2^28 vector
    m = workloads.random_klocal(n=28)
    full = sd.Plan(m.n, m.paulis, m.coeffs)
    passes = full.passes(sd.SD_C64)
    g = max(range(full.info.n_groups),
            key=lambda gi: sum(p["rho"] for p in passes if p["group"] == gi))
    ids = full.group(g).term_ids
    t = oracle.build_terms(m.n, m.paulis, m.coeffs)
    letters = {(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}
    ps = ["".join(letters[((int(t.x[k]) >> q) & 1, (int(t.z[k]) >> q) & 1)] for q in range(28))
          for k in ids]
    cs = [float(t.c[k]) for k in ids]
    sub = workloads.Model("group", 28, ps, np.array(cs))
    plan = sd.Plan(28, ps, cs).bind()
    assert plan.info.n_groups == 1
    print(f"[gpu] n28 group {g}: {len(ids)} terms, passes "
          f"{[p['rho'] for p in plan.passes(sd.SD_C64)]}", flush=True)
    psi0 = _random_state_torch(28, 5)
    want = oracle.evolve(28, sub.paulis, sub.coeffs, psi0.numpy(), 0.37, 1, 1)
    for dtype in (sd.SD_C128, sd.SD_C64):
        d = psi0.to(TDT[dtype]).cuda()
        plan.evolve(d, 0.37, 1, 1)
        got = d.cpu().numpy().astype(np.complex128)
        del d
        err = l2(got, want)
        print(f"[gpu] n28 group dtype={dtype} L2={err:.3e}", flush=True)
        assert err <= (1e-10 if dtype == sd.SD_C128 else 1e-6)


@pytest.mark.parametrize("shrink", [1, 0])
@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_ensemble_of_uneven_instances(dtype, shrink):
    # uneven sizes; n = 8 runs below the multi-instance kernel's tile minimum.
    # Plans with one tile size per plan (complex128 always, complex64 without
    # tile shrinking) and plans with several: the ensemble must equal each
    # instance's own sd_evolve bit for bit.
    models = workloads.xxz_ensemble(count=5, seed=4, nmin=8, nmax=15, steps=20)
    models[0] = workloads.xxz_ensemble(count=1, seed=9, nmin=8, nmax=8, steps=20)[0]
    print(f"[gpu] ensemble sizes {[m.n for m in models]} dtype={dtype} shrink={shrink}", flush=True)
    o = sd.sd_plan_options_default()
    o.tile_shrink_c64 = shrink
    plans = [sd.Plan(m.n, m.paulis, m.coeffs, o).bind() for m in models]
    ens = sd.sd_ensemble_create([p.p for p in plans], dtype)
    ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
    sd.sd_ensemble_bind_workspace(ens, ws)
    states = [torch.from_numpy(m.initial_state()).to(TDT[dtype]).cuda() for m in models]
    singles = [s.clone() for s in states]
    sd.sd_ensemble_evolve(ens, states, 0.05, 12, 2)
    sd.sd_ensemble_evolve(ens, states, 0.05, 8, 2)   # graph replay path
    for p, s in zip(plans, singles):
        # (the same calls: a call joins the G_0 halves of its own steps)
        p.evolve(s, 0.05, 12, 2)
        p.evolve(s, 0.05, 8, 2)
    torch.cuda.synchronize()
    for m, s, s1 in zip(models, states, singles):
        got = s.cpu().numpy().astype(np.complex128)
        assert torch.equal(s, s1), m.n
        want = oracle.evolve(m.n, m.paulis, m.coeffs, m.initial_state(), 0.05, 20, 2)
        assert l2(got, want) <= TOL[dtype], (m.n, l2(got, want))
    sd.sd_ensemble_destroy(ens)


@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_ensemble_of_small_instances_only(dtype):
    # every instance below the multi-instance kernel's tile minimum: the step
    # graphs hold only single-instance pass launches; a second call with the
    # same arguments replays them, a third with another dt captures again
    models = workloads.xxz_ensemble(count=3, seed=11, nmin=6, nmax=9, steps=10)
    print(f"[gpu] small-only ensemble sizes {[m.n for m in models]} dtype={dtype}", flush=True)
    plans = [sd.Plan(m.n, m.paulis, m.coeffs).bind() for m in models]
    ens = sd.sd_ensemble_create([p.p for p in plans], dtype)
    ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
    sd.sd_ensemble_bind_workspace(ens, ws)
    psi0 = [workloads.random_state(m.n, 80 + i) for i, m in enumerate(models)]
    states = [torch.from_numpy(a).to(TDT[dtype]).cuda() for a in psi0]
    singles = [s.clone() for s in states]
    calls = [(0.05, 4), (0.05, 3), (0.03, 2)]
    for dt, k in calls:
        sd.sd_ensemble_evolve(ens, states, dt, k, 2)
    for p, s in zip(plans, singles):
        for dt, k in calls:
            p.evolve(s, dt, k, 2)
    torch.cuda.synchronize()
    for i, (m, s, s1) in enumerate(zip(models, states, singles)):
        assert torch.equal(s, s1), m.n
        want = psi0[i]
        for dt, k in calls:
            want = oracle.evolve(m.n, m.paulis, m.coeffs, want, dt, k, 2)
        err = l2(s.cpu().numpy().astype(np.complex128), want)
        print(f"[gpu]   instance {i} n={m.n}: L2 {err:.3e}", flush=True)
        assert err <= TOL[dtype], (m.n, err)
    sd.sd_ensemble_destroy(ens)


def test_ensemble_with_a_state_above_4gib():
    # complex128 n = 29 (8 GiB: the multi-instance kernel's 32-bit offsets do
    # not reach it, so it takes single-instance pass launches inside the step
    # graphs) beside an n = 12 instance: both equal their own sd_evolve bit
    # for bit, on a second call that replays the graphs too
    big = workloads.random_klocal(n=29, m=60, seed=12, init_seed=13)
    small = workloads.random_klocal(n=12, m=80, seed=14, init_seed=15)
    plans = [sd.Plan(m.n, m.paulis, m.coeffs).bind() for m in (big, small)]
    print(f"[gpu] ensemble with n=29 complex128: passes {[p.info.passes_c128 for p in plans]}", flush=True)
    ens = sd.sd_ensemble_create([p.p for p in plans], sd.SD_C128)
    ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
    sd.sd_ensemble_bind_workspace(ens, ws)
    states = [torch.zeros(1 << 29, dtype=torch.complex128, device="cuda"),
              torch.from_numpy(workloads.random_state(12, 16)).cuda()]
    states[0][5] = 0.6
    states[0][(1 << 29) - 3] = 0.8
    singles = [s.clone() for s in states]
    for _ in range(2):
        sd.sd_ensemble_evolve(ens, states, 0.05, 2, 2)
    for p, st in zip(plans, singles):
        for _ in range(2):
            p.evolve(st, 0.05, 2, 2)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(states, singles)):
        assert torch.equal(a, b), i
    n2 = sd.sd_norm2(states[0], 29)
    print(f"[gpu] ensemble with n=29: bit-identical to sd_evolve, norm drift {n2 - 1:.2e}", flush=True)
    assert abs(n2 - 1) <= 1e-12
    sd.sd_ensemble_destroy(ens)
    del states, singles, ws
    for p in plans:
        p.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shrink", [1, 0])
def test_ensemble_after_plan_rebind(shrink):
    # a member plan rebound to a new workspace (the old one released) between
    # two ensemble calls: the second call must use the new workspace, not the
    # step captured with the old one (plans with one or several tile sizes)
    models = workloads.xxz_ensemble(count=3, seed=14, nmin=12, nmax=14, steps=10)
    print(f"[gpu] ensemble rebind sizes {[m.n for m in models]} shrink={shrink}", flush=True)
    o = sd.sd_plan_options_default()
    o.tile_shrink_c64 = shrink
    plans = [sd.Plan(m.n, m.paulis, m.coeffs, o).bind() for m in models]
    ens = sd.sd_ensemble_create([p.p for p in plans], sd.SD_C64)
    ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
    sd.sd_ensemble_bind_workspace(ens, ws)
    states = [torch.from_numpy(m.initial_state()).to(torch.complex64).cuda() for m in models]
    singles = [s.clone() for s in states]
    sd.sd_ensemble_evolve(ens, states, 0.05, 4, 2)
    torch.cuda.synchronize()
    old = plans[1].workspace
    plans[1].bind()                  # new workspace tensor, same contents
    # the old memory now holds the tables of another valid plan of the same
    # shape (the same strings, other coefficients): a step captured with the
    # old workspace would run that plan instead
    m1 = models[1]
    other = sd.Plan(m1.n, m1.paulis, np.asarray(m1.coeffs) * 1.5, o)
    assert other.info.workspace_bytes == plans[1].info.workspace_bytes
    sd.sd_bind_workspace(other.p, old)
    sd.sd_ensemble_evolve(ens, states, 0.05, 6, 2)
    for p, s in zip(plans, singles):
        p.evolve(s, 0.05, 4, 2)
        p.evolve(s, 0.05, 6, 2)
    torch.cuda.synchronize()
    for m, s, s1 in zip(models, states, singles):
        assert torch.equal(s, s1), m.n
    sd.sd_ensemble_destroy(ens)
    other.close()


@pytest.mark.skip(reason="the persistent one-launch ensemble step is switched off: a version with "
                         "per-instance counters of finished tiles and waits on them ran without finishing "
                         "on MI355X (killed after 180 s without output, twice, in the 5-instance complex128 "
                         "ensemble below); the cause was not shown, so the step is not built")
def test_ensemble_persistent_step():
    # kept as the record of the case: 5 XXZ instances n = [8, 15, 15, 12, 15],
    # complex128, 20 second-order steps, the persistent step against each
    # instance's own sd_evolve
    raise AssertionError("not built")


@pytest.mark.parametrize("mode", [sd.SD_MODE_PAPER_LAYERS, sd.SD_MODE_TERMWISE])
@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
@pytest.mark.parametrize("order", [2, 4])
def test_reference_modes(mode, dtype, order):
    # the paper's layer-by-layer circuit execution and the term-by-term
    # baseline give the same state as the oracle (and as the tiles)
    m = workloads.random_klocal(n=12, m=120, seed=21, init_seed=22)
    check(m, dtype, 0.05, 3, order, dict(mode=mode))


# one large commuting group per case: X-span rank rho up to 13 (four register
# rounds), CZ/S forms with S, Z and cross-chunk CZ (alternating: no S, CZ
# pairs split across chunks), tiles of 2^10 and 2^13
@pytest.mark.parametrize("seed,rho,alt", [(1, 9, False), (2, 9, True), (4, 6, True), (5, 3, True),
                                          (8, 13, False), (9, 13, True), (7, 11, True)])
@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_large_commuting_group(seed, rho, alt, dtype):
    rng = np.random.default_rng(seed)
    n = 15
    ps, cs = groups.commuting_group(rng, n, rho, 60, alternating=alt)
    m = workloads.Model(f"group{seed}", n, ps, np.asarray(cs))
    psi0 = workloads.random_state(n, seed)
    for tile, coal in ((13, 0), (13, 4), (10, 2)):
        opts = dict(tile_log2_c64=tile, tile_log2_c128=tile, coalesce_log2_c64=coal,
                    coalesce_log2_c128=min(coal, 3))
        check(m, dtype, 0.09, 2, 2, opts=opts, psi0=psi0)


@pytest.mark.parametrize("seed,rho,alt", [(2, 9, True), (8, 13, False), (9, 13, True)])
def test_large_group_expectation(seed, rho, alt):
    rng = np.random.default_rng(seed)
    n = 15
    ps, cs = groups.commuting_group(rng, n, rho, 60, alternating=alt)
    psi0 = workloads.random_state(n, seed + 100)
    want = oracle.energy(n, ps, np.asarray(cs), psi0)
    plan = sd.Plan(n, ps, cs).bind()
    for dtype, tol in ((sd.SD_C128, 1e-10), (sd.SD_C64, 1e-5)):
        psi = torch.from_numpy(psi0).to(TDT[dtype]).cuda()
        e = plan.expectation(psi)
        assert abs(e - want) <= tol * max(1.0, abs(want)), (dtype, e, want)


def test_state_above_4gib_uses_wide_offsets():
    # complex128 at n = 29 is 8 GiB: in-state byte offsets need 64 bits there,
    # complex64 at n = 29 (4 GiB) still uses 32-bit offsets; both runs of the
    # benchmark-like workload must agree to the complex64 bar
    n = 29
    m = workloads.random_klocal(n=n, m=600, seed=8, init_seed=1)
    plan = sd.Plan(n, m.paulis, m.coeffs).bind()
    print("[gpu] n29 wide offsets", flush=True)
    g = torch.Generator(device="cuda").manual_seed(3)
    b = torch.randn(1 << n, dtype=torch.complex128, device="cuda", generator=g)
    b /= torch.linalg.vector_norm(b)
    c = b.to(torch.complex64)
    plan.evolve(b, 0.01, 1, 2)
    plan.evolve(c, 0.01, 1, 2)
    torch.cuda.synchronize()
    assert abs(sd.sd_norm2(b, n) - 1) < 1e-12
    diff = float(torch.linalg.vector_norm(c.to(torch.complex128) - b))
    print(f"[gpu] n29 c64 vs c128 L2={diff:.3e}", flush=True)
    assert diff < 1e-5


def _gpu_fidelity(a, b, n):
    ov = sd.sd_inner(a, b, n)
    return abs(ov) ** 2 / (sd.sd_norm2(a, n) * sd.sd_norm2(b, n))


def test_config2_xxz_n26_full_length():
    # periodic XXZ n = 26 from the Neel state, second order, dt = 0.05: one
    # step of the complex128 path against the oracle on the full vector, then
    # 1000 steps of both paths (the complex64 bar: L2 <= 1e-5 and fidelity
    # >= 1 - 1e-6 against the FP64 path)
    m = workloads.xxz_chain(n=26)
    plan = sd.Plan(m.n, m.paulis, m.coeffs).bind()
    print(f"[gpu] xxz26 groups {plan.info.n_groups} passes c64 {plan.info.passes_c64}", flush=True)
    psi0 = m.initial_state()
    want = oracle.evolve(m.n, m.paulis, m.coeffs, psi0, 0.05, 1, 2)
    d = torch.from_numpy(psi0).cuda()
    plan.evolve(d, 0.05, 1, 2)
    err = l2(d.cpu().numpy(), want)
    print(f"[gpu] xxz26 one step c128 L2={err:.3e}", flush=True)
    assert err <= 1e-10
    del want
    a128 = torch.from_numpy(psi0).cuda()
    a64 = a128.to(torch.complex64)
    plan.evolve(a128, 0.05, 1000, 2)
    plan.evolve(a64, 0.05, 1000, 2)
    torch.cuda.synchronize()
    b64 = a64.to(torch.complex128)
    fid = _gpu_fidelity(a128, b64, 26)
    err = float(torch.linalg.vector_norm(b64 - a128))
    drift = abs(sd.sd_norm2(a128, 26) - 1.0)
    print(f"[gpu] xxz26 1000 steps c64 vs c128: L2={err:.3e} 1-F={1 - fid:.3e} "
          f"c128 norm drift={drift:.2e}", flush=True)
    assert err <= 1e-5 and fid >= 1 - 1e-6 and drift <= 1e-10


def test_config4_full_ensemble():
    # 256 open XXZ chains, n ~ U{14..20}, 500 second-order steps at dt = 0.05
    # in one ensemble: complex64 against complex128 for every instance, and
    # the two smallest instances of both against the oracle
    models = workloads.xxz_ensemble()
    plans = [sd.Plan(m.n, m.paulis, m.coeffs).bind() for m in models]
    print(f"[gpu] ensemble of {len(models)}, amplitudes {sum(1 << m.n for m in models)}", flush=True)
    out = {}
    for dtype in (sd.SD_C128, sd.SD_C64):
        ens = sd.sd_ensemble_create([p.p for p in plans], dtype)
        ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
        sd.sd_ensemble_bind_workspace(ens, ws)
        states = [torch.from_numpy(m.initial_state()).to(TDT[dtype]).cuda() for m in models]
        sd.sd_ensemble_evolve(ens, states, 0.05, 500, 2)
        torch.cuda.synchronize()
        sd.sd_ensemble_destroy(ens)
        out[dtype] = states
    fids = [_gpu_fidelity(a, b.to(torch.complex128), m.n)
            for m, a, b in zip(models, out[sd.SD_C128], out[sd.SD_C64])]
    print(f"[gpu] ensemble c64 vs c128: mean 1-F {1 - np.mean(fids):.3e}, "
          f"max 1-F {1 - min(fids):.3e}", flush=True)
    assert min(fids) >= 1 - 1e-6
    for i in sorted(range(len(models)), key=lambda i: models[i].n)[:2]:
        m = models[i]
        want = oracle.evolve(m.n, m.paulis, m.coeffs, m.initial_state(), 0.05, 500, 2)
        e128 = l2(out[sd.SD_C128][i].cpu().numpy(), want)
        e64 = l2(out[sd.SD_C64][i].cpu().numpy().astype(np.complex128), want)
        print(f"[gpu] ensemble instance {i} n={m.n}: L2 c128 {e128:.3e} c64 {e64:.3e}", flush=True)
        assert e128 <= 1e-10 and e64 <= 1e-5



@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
@pytest.mark.parametrize("order", [1, 4])
def test_ensemble_of_mixed_workloads(order, dtype):
    # instances of different kinds in one ensemble (passes with a shifted
    # round 0, CZ inside a chunk, staged I/O, split groups, 2^10 tiles), a
    # change of dt between calls (the step graph is captured again): every
    # instance matches the oracle and its own sd_evolve
    specs = [(workloads.random_klocal(n=12, m=300, seed=3, init_seed=2),
              dict(tile_log2_c64=10, tile_log2_c128=10)),
             (workloads.random_klocal(n=14, m=300, seed=14, init_seed=2), {}),
             (workloads.random_klocal(n=13, m=120, seed=21, init_seed=4), {}),
             (workloads.jw_fermionic(n=12, total=700), {}),
             (workloads.tfim_chain(12), {})]
    plans = []
    for m, o in specs:
        opts = sd.sd_plan_options_default()
        for k, v in o.items():
            setattr(opts, k, v)
        plans.append(sd.Plan(m.n, m.paulis, m.coeffs, opts).bind())
    models = [m for m, _ in specs]
    print(f"[gpu] mixed ensemble order {order} dtype {dtype}: sizes {[m.n for m in models]}", flush=True)
    ens = sd.sd_ensemble_create([p.p for p in plans], dtype)
    ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
    sd.sd_ensemble_bind_workspace(ens, ws)
    psi0 = [workloads.random_state(m.n, 60 + i) for i, m in enumerate(models)]
    states = [torch.from_numpy(a).to(TDT[dtype]).cuda() for a in psi0]
    singles = [s.clone() for s in states]
    sd.sd_ensemble_evolve(ens, states, 0.03, 3, order)
    sd.sd_ensemble_evolve(ens, states, 0.02, 2, order)
    for p, s in zip(plans, singles):
        p.evolve(s, 0.03, 3, order)
        p.evolve(s, 0.02, 2, order)
    torch.cuda.synchronize()
    for i, (m, s, s1) in enumerate(zip(models, states, singles)):
        want = oracle.evolve(m.n, m.paulis, m.coeffs, psi0[i], 0.03, 3, order)
        want = oracle.evolve(m.n, m.paulis, m.coeffs, want, 0.02, 2, order)
        err = l2(s.cpu().numpy().astype(np.complex128), want)
        err1 = l2(s1.cpu().numpy().astype(np.complex128), want)
        diff = float((s - s1).abs().max())
        print(f"[gpu]   instance {i} n={m.n}: L2 ensemble {err:.3e} single {err1:.3e} "
              f"max|ensemble - single| {diff:.3e}", flush=True)
        assert err <= TOL[dtype] and err1 <= TOL[dtype], (i, m.n, err, err1)
        assert diff <= (1e-12 if dtype == sd.SD_C128 else 1e-6), (i, m.n, diff)
    sd.sd_ensemble_destroy(ens)


def _xspan_basis(xs):
    rows, basis = [], []
    for v in xs:
        w = int(v)
        for r in rows:
            w = min(w, w ^ r)
        if w:
            rows.append(w)
            basis.append(int(v))
    return basis


@pytest.mark.parametrize("dtype", [sd.SD_C64, sd.SD_C128])
def test_config5_jw_n32_sampled_cosets(dtype):
    # the Jordan-Wigner workload at its full size, n = 32 (32 GiB complex64,
    # 64 GiB complex128, 64-bit in-state offsets): one application of its
    # largest group with an X span of rank <= 14 on a random state; sampled
    # outputs (whole cosets of the X span, which the group maps onto itself)
    # against the oracle computed on those cosets alone
    n = 32
    m = workloads.jw_fermionic(n=n)
    full = sd.Plan(n, m.paulis, m.coeffs)
    t = oracle.build_terms(n, m.paulis, m.coeffs)
    best = None
    for g in range(full.info.n_groups):
        ids = list(full.group(g).term_ids)
        r = len(_xspan_basis([t.x[k] for k in ids]))
        if 8 <= r <= 14 and (best is None or len(ids) > len(best[1])):
            best = (g, ids, r)
    g, ids, r = best
    letters = {(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}
    ps = ["".join(letters[((int(t.x[k]) >> q) & 1, (int(t.z[k]) >> q) & 1)] for q in range(n))
          for k in ids]
    cs = [float(t.c[k]) for k in ids]
    plan = sd.Plan(n, ps, cs).bind()
    assert plan.info.n_groups == 1
    print(f"[gpu] jw32 group {g}: {len(ids)} terms, X rank {r}, dtype={dtype}, "
          f"passes {[p['rho'] for p in plan.passes(dtype)]}", flush=True)
    psi = torch.empty(1 << n, dtype=TDT[dtype], device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(32)
    flat = torch.view_as_real(psi).view(-1)
    chunk = 1 << 28
    for s in range(0, flat.numel(), chunk):
        flat[s:s + chunk].normal_(generator=gen)
    del flat
    span = _xspan_basis([t.x[k] for k in ids])
    rng = np.random.default_rng(33)
    x0s = [int(v) for v in rng.integers(0, 1 << n, size=6, dtype=np.uint64)]
    jj = np.arange(1 << len(span), dtype=np.int64)
    idx = []
    for x0 in x0s:
        v = np.full(jj.shape, x0, dtype=np.int64)
        for i, b in enumerate(span):
            v ^= ((jj >> i) & 1) * b
        idx.append(v)
    idx_t = torch.from_numpy(np.concatenate(idx)).cuda()
    before = psi[idx_t].cpu().numpy().astype(np.complex128)
    dt = 0.02
    plan.evolve(psi, dt, 1, 1)
    after = psi[idx_t].cpu().numpy().astype(np.complex128)
    torch.cuda.synchronize()
    del psi
    xs = [int(t.x[k]) for k in ids]
    zs = [int(t.z[k]) for k in ids]
    th = [float(t.c[k]) * dt for k in ids]
    L = 1 << len(span)
    worst = 0.0
    for c, x0 in enumerate(x0s):
        want = oracle.apply_on_coset(xs, zs, th, x0, span, before[c * L:(c + 1) * L])
        got = after[c * L:(c + 1) * L]
        worst = max(worst, float(np.linalg.norm(got - want) / np.linalg.norm(want)))
    print(f"[gpu] jw32 sampled cosets: worst relative L2 {worst:.3e}", flush=True)
    assert worst <= (1e-12 if dtype == sd.SD_C128 else 1e-6)


@pytest.mark.parametrize("n,steps", [(12, 5), (20, 1)])
@pytest.mark.parametrize("mode", [sd.SD_MODE_TILES, sd.SD_MODE_PAPER_LAYERS, sd.SD_MODE_TERMWISE])
@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_tfim_fully_connected_modes(n, steps, mode, dtype):
    # the paper's first experiment (fully connected TFIM, two groups): the
    # fused tiles, the layer-by-layer circuit and the term-by-term baseline,
    # each against the oracle
    m = workloads.tfim_fully_connected(n)
    psi0 = workloads.random_state(n, 12)
    check(m, dtype, m.dt, steps, 1, dict(mode=mode), psi0=psi0)


@pytest.mark.parametrize("n", [6, 8])
@pytest.mark.parametrize("mode", [sd.SD_MODE_TILES, sd.SD_MODE_PAPER_LAYERS, sd.SD_MODE_TERMWISE])
@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_syk_majorana_modes(n, mode, dtype):
    # the paper's second experiment (SYK Majorana model, C(2n, 4) terms in
    # many small groups): every execution mode against the oracle
    m = workloads.syk_majorana(n)
    check(m, dtype, m.dt, 2, 1, dict(mode=mode), psi0=m.initial_state())


@pytest.mark.parametrize("case", ["klocal", "tfim", "syk", "jw", "wide", "dense", "shifted"])
@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_term_expectations_match_oracle(case, dtype):
    # grouped measurement: <psi|P_k|psi> of every term from one transform per
    # (sub-)group, against the oracle term by term; their weighted sum is the
    # energy of sd_expectation
    m, opts = {
        "klocal": (workloads.random_klocal(n=12, m=150, seed=41, init_seed=42), {}),
        "tfim": (workloads.tfim_fully_connected(10), {}),
        "syk": (workloads.syk_majorana(6), {}),
        "jw": (workloads.jw_fermionic(n=11, total=150), dict(tile_log2_c64=10, tile_log2_c128=10)),
        "wide": (workloads.random_klocal(n=16, m=300, seed=43, init_seed=44), {}),
        # a diagonal pass of 120 terms (lanes hold the running sums of
        # terms k mod 64, a second register from term 64 on)
        "dense": (workloads.tfim_fully_connected(16), {}),
        # 2^10 tiles: shifted round 0 and a CZ between register slots
        "shifted": (workloads.random_klocal(n=12, m=300, seed=3, init_seed=2),
                    dict(tile_log2_c64=10, tile_log2_c128=10)),
    }[case]
    o = sd.sd_plan_options_default()
    for k, v in opts.items():
        setattr(o, k, v)
    plan = sd.Plan(m.n, m.paulis, m.coeffs, o).bind()
    psi = workloads.random_state(m.n, 45)
    d = torch.from_numpy(psi).to(TDT[dtype]).cuda()
    got = plan.term_expectations(d)
    ref_state = d.cpu().numpy().astype(np.complex128)
    want = oracle.term_expectations(m.n, m.paulis, m.coeffs, ref_state)
    t = oracle.build_terms(m.n, m.paulis, m.coeffs)
    err = float(np.abs(got - want).max())
    print(f"[gpu] term expectations {case} dtype={dtype} terms={len(want)} max err {err:.2e}", flush=True)
    assert err <= (1e-12 if dtype == sd.SD_C128 else 1e-6)
    assert abs(float(np.dot(t.c, got)) - plan.expectation(d)) <= 1e-9


@pytest.mark.parametrize("dtype", [sd.SD_C128, sd.SD_C64])
def test_term_expectations_sampled_n24(dtype):
    # n = 24 (passes of up to 3 rounds, the tile kernel's per-term sums over
    # 4096 tiles): 32 sampled terms against the oracle on the same state,
    # and the weighted sum of all of them against sd_expectation
    m = workloads.random_klocal(n=24, m=1500, seed=3, init_seed=2)
    plan = sd.Plan(m.n, m.paulis, m.coeffs).bind()
    psi = workloads.random_state(24, 46)
    d = torch.from_numpy(psi).to(TDT[dtype]).cuda()
    got = plan.term_expectations(d)
    ref_state = d.cpu().numpy().astype(np.complex128)
    t = oracle.build_terms(m.n, m.paulis, m.coeffs)
    ids = np.sort(np.random.default_rng(47).choice(len(t.x), size=32, replace=False))
    sub = oracle.Terms(t.n, t.x[ids], t.z[ids], t.c[ids], t.source[ids])
    want = oracle.term_expectations(m.n, None, None, ref_state, terms=sub)
    err = float(np.abs(got[ids] - want).max())
    e = plan.expectation(d)
    print(f"[gpu] term expectations n=24 dtype={dtype}: {len(t.x)} terms, sampled max err {err:.2e}, "
          f"sum c_k <P_k> - E {float(np.dot(t.c, got)) - e:.2e}", flush=True)
    assert err <= (1e-12 if dtype == sd.SD_C128 else 1e-6)
    assert abs(float(np.dot(t.c, got)) - e) <= 1e-9
    plan.close()


def test_term_expectations_time_series():
    # observables along a trajectory: after every step of an XXZ chain the
    # bond and field terms of H, from the evolving GPU state, against the
    # oracle's state
    m = workloads.xxz_chain(n=12, steps=5)
    plan = sd.Plan(m.n, m.paulis, m.coeffs).bind()
    psi = m.initial_state()
    d = torch.from_numpy(psi).cuda()
    t = oracle.build_terms(m.n, m.paulis, m.coeffs)
    for step in range(5):
        plan.evolve(d, 0.05, 1, 2)
        psi = oracle.evolve(m.n, m.paulis, m.coeffs, psi, 0.05, 1, 2, terms=t)
        got = plan.term_expectations(d)
        want = oracle.term_expectations(m.n, m.paulis, m.coeffs, psi, terms=t)
        assert np.abs(got - want).max() <= 1e-12, step


@pytest.mark.parametrize("n,seed,m,D,dtype", [(12, 3, 300, 10, sd.SD_C64), (12, 19, 150, 10, sd.SD_C128),
                                              (14, 14, 300, 13, sd.SD_C64)])
def test_shifted_round0_with_cz(n, seed, m, D, dtype):
    # plans with a shifted round 0 whose chunk holds a CZ between register
    # slots (its outputs move by M d(t) as well as taking the sign)
    w = workloads.random_klocal(n=n, m=m, seed=seed, init_seed=2)
    check(w, dtype, 0.11, 3, 2, dict(tile_log2_c64=D, tile_log2_c128=D))


def test_autotune_tiles():
    # the tile-size autotuner returns one of its candidates with per-step
    # times, and the plan it chooses evolves correctly; an ensemble built
    # with the size tuned on its largest instance matches the oracle
    m = workloads.random_klocal(n=16, m=200, seed=51, init_seed=52)
    h = sd.sd_hamiltonian_create(m.n, m.paulis, m.coeffs)
    scratch = torch.from_numpy(workloads.random_state(m.n, 53)).to(torch.complex64).cuda()
    cands = [10, 11, 12, 13]
    best, secs = sd.sd_autotune_tiles(h, sd.SD_C64, scratch, 0.05, 2, 1, cands)
    print(f"[gpu] autotune n=16 c64: {dict(zip(cands, secs))} -> {best.tile_log2_c64}", flush=True)
    assert best.tile_log2_c64 in cands and all(s > 0 for s in secs)
    assert best.tile_log2_c64 == cands[int(np.argmin(secs))]
    check(m, sd.SD_C64, 0.05, 2, 2, dict(tile_log2_c64=best.tile_log2_c64))
    sd.sd_hamiltonian_destroy(h)
    models = workloads.xxz_ensemble(count=6, seed=7, nmin=12, nmax=16, steps=10)
    big = max(models, key=lambda w: w.n)
    hb = sd.sd_hamiltonian_create(big.n, big.paulis, big.coeffs)
    sb = torch.from_numpy(big.initial_state()).cuda()
    bo, _ = sd.sd_autotune_tiles(hb, sd.SD_C128, sb, 0.05, 2, 1, [10, 11, 12])
    sd.sd_hamiltonian_destroy(hb)
    o = sd.sd_plan_options_default()
    o.tile_log2_c128 = bo.tile_log2_c128
    plans = [sd.Plan(w.n, w.paulis, w.coeffs, o).bind() for w in models]
    ens = sd.sd_ensemble_create([p.p for p in plans], sd.SD_C128)
    ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
    sd.sd_ensemble_bind_workspace(ens, ws)
    states = [torch.from_numpy(w.initial_state()).cuda() for w in models]
    sd.sd_ensemble_evolve(ens, states, 0.05, 10, 2)
    torch.cuda.synchronize()
    for w, s in zip(models, states):
        want = oracle.evolve(w.n, w.paulis, w.coeffs, w.initial_state(), 0.05, 10, 2)
        assert l2(s.cpu().numpy(), want) <= 1e-10, w.n
    sd.sd_ensemble_destroy(ens)
