"""Benchmark: Trotter steps/s of the grouped (simultaneously diagonalised)
evolution on one MI355X.

Workload: random sparse k-local Pauli Hamiltonian, n = 28 qubits, 2000 drawn
strings of weight 2-4 (1932 after merging duplicates), N(0,1) coefficients,
first-order Trotter, dt = 0.01, random complex-Gaussian initial state.  The
complex64 path (FP32 amplitudes, FP64 phase and butterflies) gives `value`;
the complex128 path is timed beside it and serves as the FP64 reference for
the fidelity figure.

Prints one JSON line on stdout; progress goes to stderr.  --experiment
tfim_sweep | syk_sweep runs the paper's two experiments instead (one line per
n); --experiment ensemble the 256-instance XXZ ensemble, xxz26 / jw32 the
XXZ chain at n = 26 and the Jordan-Wigner workload at n = 32, observables the
per-term expectation values of the benchmark Hamiltonian (one line each).
"""
import argparse
import collections
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
ROOFLINE_KERNEL = "sd::k_tile<float2, 0, uint32_t, GEN>"   # both GEN instantiations
COUNTERS = os.path.join(ROOT, "profiles", "k_tile_c64_n28_hbm_counters.txt")


def kernel_source_digest():
    """sha256 over the library's sources: the traffic figure in the counter
    summary is valid only for the sources it was measured with."""
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2206_11664_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".cpp", ".h")):
            h.update(name.encode())
            with open(os.path.join(src, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per k_tile launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's
    reading for a plain copy of known size), or None when the summary is
    missing or was taken with other kernel sources."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    with open(COUNTERS) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_groups(K, order):
    """Group applications of one Trotter step in a run of many steps, as
    (group, fraction of dt): order 1 the groups in order; order 2 (Strang)
    G_0..G_{K-2} at dt/2, G_{K-1} at dt, back down to G_0 at dt/2; order 4
    five Strang steps (Suzuki).  Applications of one group that follow each
    other are joined into one, inside a step and across the step boundary
    (the steady-state step of a call of many steps)."""
    if K <= 0:
        return []
    if order == 1 or K == 1:
        seq = [(g, 1.0) for g in range(K)]
    else:
        s2 = [(g, 0.5) for g in range(K - 1)] + [(K - 1, 1.0)] + [(g, 0.5) for g in range(K - 2, -1, -1)]
        if order == 2:
            seq = s2
        else:
            p = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))
            seq = [(g, f * w) for w in (p, p, 1.0 - 4.0 * p, p, p) for g, f in s2]
    m = []
    for g, f in seq:
        if m and m[-1][0] == g:
            m[-1] = (g, m[-1][1] + f)
        else:
            m.append((g, f))
    if len(m) >= 2 and m[0][0] == m[-1][0]:
        m = m[1:-1] + [(m[-1][0], m[-1][1] + m[0][1])]
    return m


def applications_per_step(K, order):
    """Group applications (C_g, Lambda_g, C_g^dagger) in one steady-state
    Trotter step: the unit of the algorithmic bytes, one read and one write
    of the state each.  Order 1: K; order 2 (Strang, the G_0 halves of
    consecutive steps joined): 2K - 2 for K > 1; order 4: 5 (2K - 2)."""
    return len(step_groups(K, order))


def passes_per_step(plan, dtype, order):
    """Tile passes (launches) of one steady-state step of a plan."""
    per_group = collections.Counter(ps["group"] for ps in plan.passes(dtype))
    return sum(per_group[g] for g, _ in step_groups(int(plan.info.n_groups), order))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def paper_sweep(args, torch, workloads, sd):
    """The paper's experiments on this GPU: one first-order Trotter step
    (dt = 0.01) for n = nmin..nmax of
      tfim_sweep: the fully connected TFIM, J_ij, h_i ~ U[-1,1], m = n(n-1)/2
        + n terms in two commuting groups;
      syk_sweep: the SYK Majorana model, C(2n, 4) four-Majorana terms.
    Timed per step: the term-by-term baseline (one rotation pass per term),
    the paper's grouped circuit executed layer by layer (one pass per gate
    layer, as the paper runs it) and the fused tile passes; speedups of both
    grouped forms over term by term beside the paper's cost-model line
    m/(n n_g).  complex128 and complex64 states."""
    stream = torch.cuda.current_stream()

    def step_time(plan, state, dt):
        # one step first (a warm-up, and the measurement when it is long)
        k = 1
        while True:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.evolve(state, dt, k, 1)
            e1.record(stream)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / 1e3
            if (k == 1 and sec > 0.5) or (k > 1 and sec > 0.05) or k >= 64:
                return sec / k
            k *= 4

    gen = workloads.tfim_fully_connected if args.experiment == "tfim_sweep" else workloads.syk_majorana
    modes = [x for x in args.modes.split(",") if x]
    for n in range(args.nmin, args.nmax + 1, args.nstep):
        m = gen(n)
        row = {"experiment": args.experiment, "n": n, "terms": len(m.paulis)}
        plans = {}
        for name, mode in (("tiles", sd.SD_MODE_TILES), ("paper_layers", sd.SD_MODE_PAPER_LAYERS),
                           ("termwise", sd.SD_MODE_TERMWISE)):
            if name != "tiles" and name not in modes:
                continue
            o = sd.sd_plan_options_default()
            o.mode = mode
            ps, cs = m.paulis, m.coeffs
            if name == "termwise" and 0 < args.termwise_sample < len(m.paulis):
                # one rotation pass per term, all alike: time the first terms
                # and scale to all of them
                ps, cs = m.paulis[:args.termwise_sample], m.coeffs[:args.termwise_sample]
            plans[name] = sd.Plan(n, ps, cs, o).bind("cuda")
        scale = {k: 1.0 for k in plans}
        if "termwise" in plans and 0 < args.termwise_sample < len(m.paulis):
            scale["termwise"] = len(m.paulis) / args.termwise_sample
            row["termwise_sampled_terms"] = args.termwise_sample
        info = plans["tiles"].info
        ng = int(info.n_groups)
        row["groups"] = ng
        row["plan_seconds"] = round(float(info.plan_seconds), 2)
        row["passes_c64"] = int(info.passes_c64)
        row["cost_model_speedup"] = round(len(m.paulis) / (n * ng), 3)
        if n <= 28:
            psi0 = torch.from_numpy(workloads.random_state(n, 1)).cuda()
        else:
            # (drawn on the GPU: the host copy would take 2^n x 16 bytes)
            psi0 = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
            g = torch.Generator(device="cuda").manual_seed(1)
            flat = torch.view_as_real(psi0).view(-1)
            for i in range(0, flat.numel(), 1 << 28):
                flat[i:i + (1 << 28)].normal_(generator=g)
            del flat
            psi0 /= sd.sd_norm2(psi0, n) ** 0.5
        for dname, tdt in (("c128", torch.complex128), ("c64", torch.complex64)):
            t = {}
            for name, plan in plans.items():
                st = psi0.to(tdt)
                t[name] = step_time(plan, st, m.dt) * scale[name]
                del st
            row[dname] = {"step_ms": {k: round(v * 1e3, 4) for k, v in t.items()}}
            if "termwise" in t:
                row[dname]["speedup_tiles_vs_termwise"] = round(t["termwise"] / t["tiles"], 2)
                if "paper_layers" in t:
                    row[dname]["speedup_paper_layers_vs_termwise"] = round(t["termwise"] / t["paper_layers"], 2)
        log(f"{args.experiment} n={n}: c128 {row['c128']['step_ms']} c64 {row['c64']['step_ms']}")
        print(json.dumps(row), flush=True)
        del psi0, plans


def ensemble_experiment(args, torch, workloads, sd):
    """The ensemble workload on this GPU: 256 open XXZ chains, n_i ~ U{14..20}
    (seed 4), Neel states, second order at dt = 0.05, evolved together by
    sd_ensemble_evolve (one multi-instance tile launch per pass level and
    tile size, one step replayed as a HIP graph).  Timed: --steps steps after
    --warmup, for complex64 and complex128; beside it the same instances
    evolved one after another with sd_evolve.  The tile size is autotuned on
    the whole ensemble first (--no-autotune: 2^13).  Algorithmic bytes: every group
    application of every instance reads and writes its state once,
    2 * 2^n_i * B bytes (4 applications per second-order step of the three
    XXZ groups, the G_0 halves of consecutive steps joined); the bytes of all
    passes (sub-groups) are given beside them.
    Accuracy: mean and worst 1 - F between the complex64 and complex128
    ensembles after the same steps."""
    import numpy as np
    stream = torch.cuda.current_stream()
    models = workloads.xxz_ensemble()
    dt, order = models[0].dt, models[0].order
    amps = sum(1 << m.n for m in models)

    def timed(fn, steps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    o = sd.sd_plan_options_default()
    o.tile_shrink_c64 = args.tile_shrink
    tune = {}
    # The tile size (LDS block) on this GPU: every candidate maximum tile size
    # timed on the whole ensemble (10 steps after 2), per precision; complex64
    # keeps only sizes that need no more passes than 2^13 (each pass rounds
    # every amplitude once).  Ties within 1% go to the larger tile.
    for name, dtype, tdt, attr in (() if args.no_autotune else
                                   (("c64", sd.SD_C64, torch.complex64, "tile_log2_c64"),
                                    ("c128", sd.SD_C128, torch.complex128, "tile_log2_c128"))):
        secs, npass = {}, {}
        for c in (12, 13):
            oc = sd.sd_plan_options_default()
            oc.tile_shrink_c64 = args.tile_shrink
            setattr(oc, attr, c)
            pl = [sd.Plan(m.n, m.paulis, m.coeffs, oc).bind("cuda") for m in models]
            npass[c] = sum(passes_per_step(p, dtype, order) for p in pl)
            ens = sd.sd_ensemble_create([p.p for p in pl], dtype)
            ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
            sd.sd_ensemble_bind_workspace(ens, ws)
            sts = [torch.from_numpy(m.initial_state()).to(tdt).cuda() for m in models]
            sd.sd_ensemble_evolve(ens, sts, dt, 2, order)
            secs[c] = timed(lambda k: sd.sd_ensemble_evolve(ens, sts, dt, k, order), 10) / 10
            sd.sd_ensemble_destroy(ens)
            del ws, sts, pl
        ok = [c for c in secs if dtype != sd.SD_C64 or npass[c] <= npass[13]]
        chosen = max(c for c in ok if secs[c] <= 1.01 * min(secs[x] for x in ok))
        setattr(o, attr, chosen)
        tune[name] = {"step_ms": {str(c): round(1e3 * t, 3) for c, t in secs.items()},
                      "instance_passes_per_step": {str(c): v for c, v in npass.items()}, "chosen": chosen}
        log(f"ensemble autotune {name}: {tune[name]}")
    log(f"ensemble: planning {len(models)} instances")
    t0 = time.time()
    plans = [sd.Plan(m.n, m.paulis, m.coeffs, o).bind("cuda") for m in models]
    plan_s = time.time() - t0

    res = {}
    finals = {}
    for name, dtype, tdt, B in (("c64", sd.SD_C64, torch.complex64, 8),
                                ("c128", sd.SD_C128, torch.complex128, 16)):
        log(f"ensemble {name}")
        ens = sd.sd_ensemble_create([p.p for p in plans], dtype)
        ws = torch.empty(sd.sd_ensemble_workspace_bytes(ens), dtype=torch.uint8, device="cuda")
        sd.sd_ensemble_bind_workspace(ens, ws)
        states = [torch.from_numpy(m.initial_state()).to(tdt).cuda() for m in models]
        run = lambda k: sd.sd_ensemble_evolve(ens, states, dt, k, order)
        if args.warmup:
            run(args.warmup)
        sec = timed(run, args.steps)
        launches = sum(passes_per_step(p, dtype, order) for p in plans)
        # algorithmic bytes: one read and one write of an instance's state per
        # group application (2K - 2 of them in a second-order step whose G_0
        # halves are joined with those of the neighbouring steps)
        step_bytes = sum(applications_per_step(int(p.info.n_groups), order) * 2 * (1 << m.n) * B
                         for p, m in zip(plans, models))
        pass_bytes = sum(passes_per_step(p, dtype, order) * 2 * (1 << m.n) * B for p, m in zip(plans, models))
        gbps = step_bytes * args.steps / sec / 1e9
        # the same instances one after another (warm-up of the same length)
        seq = [torch.from_numpy(m.initial_state()).to(tdt).cuda() for m in models]
        ks = max(1, args.steps // 4)

        def one_by_one(k):
            for p, st in zip(plans, seq):
                p.evolve(st, dt, k, order)
        one_by_one(1)
        sec_seq = timed(one_by_one, ks)
        res[name] = {"steps_per_s": round(args.steps / sec, 3),
                     "ms_per_step": round(1e3 * sec / args.steps, 4),
                     "instance_passes_per_step": launches,
                     "algorithmic_bytes_per_step": step_bytes,
                     "pass_bytes_per_step": pass_bytes,
                     "hbm_gbps_per_pass_bytes": round(pass_bytes * args.steps / sec / 1e9, 1),
                     "hbm_gbps_algorithmic": round(gbps, 1),
                     "frac_of_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4),
                     "one_by_one_steps_per_s": round(ks / sec_seq, 3),
                     "ensemble_speedup_vs_one_by_one": round((args.steps / sec) / (ks / sec_seq), 2)}
        finals[name] = states
        log(f"ensemble {name}: {res[name]}")
        sd.sd_ensemble_destroy(ens)
        del ws, seq
    fids = []
    for m, a, b in zip(models, finals["c64"], finals["c128"]):
        a2 = a.to(torch.complex128)
        ov = sd.sd_inner(b, a2, m.n)
        fids.append(abs(ov) ** 2 / (sd.sd_norm2(a2, m.n) * sd.sd_norm2(b, m.n)))
    out = {"experiment": "ensemble", "metric": "ensemble Trotter steps/s (256 instances together)",
           "unit": "steps/s", "steps": args.steps, "warmup": args.warmup,
           "config": {"workload": "xxz_open_ensemble_256", "instances": len(models),
                      "n_range": [min(m.n for m in models), max(m.n for m in models)],
                      "amplitudes": amps, "order": order, "dt": dt, "seed": 4},
           "plan_seconds": round(plan_s, 2), "tile_shrink_c64": args.tile_shrink,
           "tile_log2": {"c64": int(o.tile_log2_c64), "c128": int(o.tile_log2_c128)}, "autotune": tune, **res,
           "accuracy_c64_vs_c128": {"steps": args.warmup + args.steps,
                                    "mean_1_minus_F": float(1.0 - np.mean(fids)),
                                    "max_1_minus_F": float(1.0 - np.min(fids))}}
    print(json.dumps(out), flush=True)


def config_experiment(args, torch, workloads, sd):
    """Configurations 2 and 5 on this GPU, one JSON line each:
      xxz26: periodic XXZ chain with random fields, n = 26, K = 3 groups,
        second order, dt = 0.05 (Neel state);
      jw32: Jordan-Wigner-shaped fermionic Hamiltonian, n = 32, 10^4 terms,
        second order, dt = 0.02 (Hartree-Fock-like basis state; the state
        takes 32 GiB in complex64, 64 GiB in complex128).
    Timed: steps of the complex64 and complex128 paths (HIP events on the
    launch stream).  Algorithmic bytes: one read and one write of the state
    per group application, 2K - 2 applications per second-order step (the G_0
    halves of consecutive steps joined).
    Accuracy: complex64 against complex128 after the same steps from the same
    state (1000 steps for xxz26, one for jw32)."""
    stream = torch.cuda.current_stream()
    if args.experiment == "xxz26":
        m = workloads.xxz_chain(26)
        steps, warm, acc_steps = max(args.steps, 100), max(args.warmup, 2), 1000
    else:
        m = workloads.jw_fermionic(32)
        steps, warm, acc_steps = 1, 0, 1
    n, dt, order = m.n, m.dt, 2
    t0 = time.time()
    plan = sd.Plan(n, m.paulis, m.coeffs).bind("cuda")
    plan_s = time.time() - t0
    info = plan.info
    K = int(info.n_groups)
    apps = applications_per_step(K, order)
    log(f"{args.experiment}: {info.n_terms} terms, {K} groups, passes c64 {info.passes_c64} "
        f"c128 {info.passes_c128}, planned in {plan_s:.1f} s")

    def state(tdt):
        st = torch.zeros(1 << n, dtype=tdt, device="cuda")
        st[int(m.init_index) if m.init == "basis" else workloads.neel_index(n)] = 1.0
        return st

    def timed(st, k):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.evolve(st, dt, k, order)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    res = {}
    for name, tdt, B in (("c64", torch.complex64, 8), ("c128", torch.complex128, 16)):
        st = state(tdt)
        if warm:
            plan.evolve(st, dt, warm, order)
        sec = timed(st, steps)
        alg = apps * 2 * (1 << n) * B
        passes = int(info.passes_c64 if B == 8 else info.passes_c128)
        gbps = alg * steps / sec / 1e9
        res[name] = {"steps_per_s": round(steps / sec, 4), "ms_per_step": round(1e3 * sec / steps, 3),
                     "launches_per_step": passes_per_step(plan, sd.SD_C64 if B == 8 else sd.SD_C128, order),
                     "passes_per_order1_step": passes,
                     "algorithmic_bytes_per_step": alg, "hbm_gbps_algorithmic": round(gbps, 1),
                     "frac_of_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4)}
        log(f"{args.experiment} {name}: {res[name]}")
        del st
    # accuracy: the same steps from the same state in both precisions
    a = state(torch.complex64)
    b = state(torch.complex128)
    e0 = plan.expectation(b)
    done = 0
    while done < acc_steps:
        k = min(100, acc_steps - done)
        plan.evolve(a, dt, k, order)
        plan.evolve(b, dt, k, order)
        torch.cuda.synchronize()
        done += k
    l2sq, mx = 0.0, 0.0
    for i in range(0, a.numel(), 1 << 26):
        d = a[i:i + (1 << 26)].to(torch.complex128) - b[i:i + (1 << 26)]
        l2sq += float(torch.sum(d.real * d.real + d.imag * d.imag))
        mx = max(mx, float(d.abs().max()))
    na, nb = sd.sd_norm2(a, n), sd.sd_norm2(b, n)
    ov = 0j
    for i in range(0, a.numel(), 1 << 28):
        aa = a[i:i + (1 << 28)].to(torch.complex128)
        ov += complex(torch.vdot(b[i:i + (1 << 28)], aa))
    fid = abs(ov) ** 2 / (na * nb)
    ea, eb = plan.expectation(a), plan.expectation(b)
    out = {"experiment": args.experiment,
           "metric": "Trotter steps/s (grouped), c64 amplitudes + FP64 phase vs c128",
           "unit": "steps/s",
           "config": {"workload": "xxz_periodic_n26" if n == 26 else "jw_fermionic_n32",
                      "n_qubits": n, "terms": int(info.n_terms), "groups": K, "order": order,
                      "dt": dt, "initial_state": m.init},
           "plan_seconds": round(plan_s, 2), "timed_steps": steps, "warmup": warm,
           "group_applications_per_step": apps, **res,
           "c64_over_c128": round(res["c64"]["steps_per_s"] / res["c128"]["steps_per_s"], 3),
           "accuracy_c64_vs_c128": {"steps": acc_steps, "l2": l2sq ** 0.5, "max_abs": mx,
                                    "energy_initial": e0, "energy_drift_c64": ea - e0,
                                    "energy_drift_c128": eb - e0,
                                    "1_minus_fidelity": 1.0 - fid, "norm_drift_c64": na - 1.0,
                                    "norm_drift_c128": nb - 1.0}}
    print(json.dumps(out), flush=True)


def observables_experiment(args, torch, workloads, sd):
    """Grouped measurement on this GPU: <psi|P_k|psi> of every term of the
    n = 28 random k-local benchmark Hamiltonian (1932 terms) from one
    forward transform per (sub-)group pass, complex64 and complex128 states
    (a random state drawn on the GPU).  Timed (host clock around the
    synchronising call, median of --steps calls after one warm-up): the
    per-term call, the energy call and one first-order evolve step.  Read
    bytes: one read of the state per pass.  Check: sum_k c_k <P_k> against
    the energy call (a different reduction of the same passes)."""
    import numpy as np
    n = args.n
    m = workloads.random_klocal(n=n)
    plan = sd.Plan(n, m.paulis, m.coeffs).bind("cuda")
    info = plan.info
    coef = np.asarray(sd.sd_hamiltonian_terms(plan.h)[3], dtype=np.float64)   # merged-term c_k
    res = {}
    for name, tdt, B, passes in (("c64", torch.complex64, 8, int(info.passes_c64)),
                                 ("c128", torch.complex128, 16, int(info.passes_c128))):
        st = torch.empty(1 << n, dtype=tdt, device="cuda")
        gen = torch.Generator(device="cuda").manual_seed(7)
        flat = torch.view_as_real(st).view(-1)
        for i in range(0, flat.numel(), 1 << 28):
            flat[i:i + (1 << 28)].normal_(generator=gen)
        del flat
        st /= sd.sd_norm2(st, n) ** 0.5
        vals = plan.term_expectations(st)
        e = plan.expectation(st)
        tt, te = [], []
        for _ in range(max(3, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vals = plan.term_expectations(st)
            t1 = time.perf_counter()
            e = plan.expectation(st)
            te.append(time.perf_counter() - t1)
            tt.append(t1 - t0)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        plan.evolve(st, m.dt, 1, 1)
        ev1.record()
        torch.cuda.synchronize()
        sec = float(np.median(tt))
        rd = passes * (1 << n) * B
        res[name] = {"term_expectations_ms": round(1e3 * sec, 2),
                     "expectation_ms": round(1e3 * float(np.median(te)), 2),
                     "evolve_step_ms": round(ev0.elapsed_time(ev1), 2),
                     "terms_per_s": round(len(vals) / sec, 1), "passes": passes,
                     "read_bytes": rd, "read_gbps": round(rd / sec / 1e9, 1),
                     "sum_c_k_P_k_minus_energy": float(np.dot(coef, vals) - e)}
        log(f"observables {name}: {res[name]}")
        del st
    out = {"experiment": "observables", "metric": "per-term expectation values of H (grouped measurement)",
           "unit": "terms/s", "config": {"workload": f"random_klocal_n{n}", "n_qubits": n,
                                         "terms": int(info.n_terms), "groups": int(info.n_groups)},
           "calls_timed": max(3, args.steps), **res}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference-modes", action="store_true")
    ap.add_argument("--cpu-sample-terms", type=int, default=128)
    ap.add_argument("--experiment", choices=["tfim_sweep", "syk_sweep", "ensemble", "xxz26", "jw32",
                                             "observables"],
                    default=None,
                    help="instead of the benchmark line: the paper's fully connected TFIM "
                         "or SYK Majorana sweep, grouped vs term by term (one JSON line per n), "
                         "the 256-instance XXZ ensemble, the XXZ chain at n = 26, the "
                         "Jordan-Wigner workload at n = 32 or the per-term expectation "
                         "values of the benchmark Hamiltonian (one JSON line each)")
    ap.add_argument("--nstep", type=int, default=2)
    ap.add_argument("--no-autotune", action="store_true",
                    help="plan with the default tile sizes (2^13) instead of autotuning them; "
                         "the profiled runs use this so that their traces hold the timed plan only")
    ap.add_argument("--accuracy-steps", type=int, default=0,
                    help="steps of the complex64 vs complex128 accuracy run (default: 10)")
    ap.add_argument("--modes", default="paper_layers,termwise",
                    help="sweeps: reference modes timed beside the tiles")
    ap.add_argument("--termwise-sample", type=int, default=0,
                    help="sweeps: time the term-by-term step on its first K terms and scale "
                         "by m/K (every term is one rotation pass of the same cost)")
    ap.add_argument("--tile-shrink", type=int, default=1,
                    help="ensemble: plans' tile_shrink_c64 (1: smallest tile per complex64 "
                         "pass, 0: one tile size per plan)")
    ap.add_argument("--nmin", type=int, default=12)
    ap.add_argument("--nmax", type=int, default=30)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain elementwise copy (negation) of a 2^n complex64 "
                         "vector, the calibration kernel of the HBM counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the state-vector path is not sharded across GPUs in this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2206_11664_amd import sd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.experiment == "ensemble":
        ensemble_experiment(args, torch, workloads, sd)
        return
    if args.experiment in ("xxz26", "jw32"):
        config_experiment(args, torch, workloads, sd)
        return
    if args.experiment == "observables":
        observables_experiment(args, torch, workloads, sd)
        return
    if args.experiment:
        paper_sweep(args, torch, workloads, sd)
        return
    n = args.n
    m = workloads.random_klocal(n=n)
    log("initial state")
    psi_host = workloads.random_state(n, m.init_seed)  # complex128, normalised in FP64
    d128_0 = torch.from_numpy(psi_host).cuda()
    dim = 1 << n
    # tile sizes: the library's autotuner on this GPU (one timed step per
    # candidate on a scratch copy of the state)
    tune = {}
    opts = sd.sd_plan_options_default()
    h = sd.sd_hamiltonian_create(n, m.paulis, m.coeffs)
    def passes_at(dt_, size):
        o = sd.sd_plan_options_default()
        o.small_state_tiles = 0
        if dt_ == sd.SD_C64:
            o.tile_log2_c64 = size
        else:
            o.tile_log2_c128 = size
        p = sd.sd_plan(h, o)
        i = sd.sd_plan_info_get(p)
        sd.sd_plan_destroy(p)
        return int(i.passes_c64 if dt_ == sd.SD_C64 else i.passes_c128)

    for name, dt_, tdt, cands in (() if args.no_autotune else
                                  (("c64", sd.SD_C64, torch.complex64, [11, 12, 13]),
                                   ("c128", sd.SD_C128, torch.complex128, [12, 13]))):
        # complex64: only tile sizes that need no more passes than 2^13 (each
        # pass rounds every amplitude once: more passes would loosen the
        # 1000-step accuracy the default plan is tested at)
        budget = passes_at(dt_, 13)
        all_cands = cands
        cands = [c for c in cands if dt_ != sd.SD_C64 or passes_at(dt_, c) <= budget]
        log(f"autotune {name} tile size {cands} (of {all_cands}; pass budget {budget})")
        scratch = d128_0.to(tdt)
        best, secs = sd.sd_autotune_tiles(h, dt_, scratch, m.dt, 1, 1, cands)
        del scratch
        # the largest tile within 1% of the fastest: as fast within the
        # timing noise, and the fewest passes (each pass rounds every
        # complex64 amplitude once)
        size = max(c for c, t in zip(cands, secs) if t <= 1.01 * min(secs))
        if dt_ == sd.SD_C64:
            opts.tile_log2_c64 = size
        else:
            opts.tile_log2_c128 = size
        tune[name] = {"step_ms": {str(c): round(s * 1e3, 2) for c, s in zip(cands, secs)}, "chosen": size,
                      "passes_by_tile": {str(c): passes_at(dt_, c) for c in all_cands}}
    sd.sd_hamiltonian_destroy(h)
    t0 = time.time()
    plan = sd.Plan(n, m.paulis, m.coeffs, opts)
    info = plan.info
    log(f"plan: {info.n_terms} terms, {info.n_groups} groups, passes/step c64 {info.passes_c64} "
        f"c128 {info.passes_c128}, paper-model passes {info.paper_model_passes}, "
        f"{time.time() - t0:.2f} s")
    plan.bind("cuda")
    stream = torch.cuda.current_stream()

    def timed(state, steps, warmup):
        for _ in range(warmup):
            plan.evolve(state, m.dt, 1, 1)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        plan.evolve(state, m.dt, steps, 1)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3

    # complex64 (the headline path)
    log("c64 timing")
    a64 = d128_0.to(torch.complex64)
    t64 = timed(a64, args.steps, args.warmup)
    sps64 = args.steps / t64
    # complex128 reference path
    log("c128 timing")
    a128 = d128_0.clone()
    k128 = max(2, args.steps // 2)
    t128 = timed(a128, k128, args.warmup)
    sps128 = k128 / t128

    # accuracy: same number of steps from the same state, c64 vs c128
    steps_acc = args.accuracy_steps if args.accuracy_steps else min(10, args.steps)
    log(f"accuracy run ({steps_acc} steps)")
    b64 = d128_0.to(torch.complex64)
    b128 = d128_0.clone()
    done = 0
    while done < steps_acc:
        k = min(100, steps_acc - done)
        plan.evolve(b64, m.dt, k, 1)
        plan.evolve(b128, m.dt, k, 1)
        torch.cuda.synchronize()
        done += k
        if steps_acc > 100:
            log(f"accuracy run: {done} of {steps_acc} steps")
    ov = sd.sd_inner(b128, b64.to(torch.complex128), n)
    n64 = sd.sd_norm2(b64, n)
    n128 = sd.sd_norm2(b128, n)
    fid = abs(ov) ** 2 / (n64 * n128)
    diff = b64.to(torch.complex128) - b128
    l2 = float(torch.linalg.vector_norm(diff))
    maxerr = float(diff.abs().max())
    e64 = plan.expectation(b64)
    e128 = plan.expectation(b128)
    e0 = plan.expectation(d128_0)
    del diff, b64, b128, a64, a128

    if args.calib_copy:
        log("calibration copy")
        src = torch.ones(dim, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"calibration copy: {dim * 8} bytes read, {dim * 8} bytes written")
        del src, dst

    # Roofline by group applications (the method's unit): every application
    # of a group reads and writes the state once, 2 * 2^n * B bytes.  A
    # launch is one tile pass; a group split into sub-groups takes several,
    # so one launch does applications / passes of a unit.
    K = int(info.n_groups)
    apps = applications_per_step(K, 1)
    unit64 = 2 * dim * 8
    alg_step64 = apps * unit64
    launches = args.steps * info.passes_c64
    avg_launch_s = t64 / launches
    achieved = alg_step64 * args.steps / t64 / 1e9        # = (apps / passes) * unit / avg launch
    pass_gbps = unit64 / avg_launch_s / 1e9               # what one pass moves per launch time
    traffic = counter_traffic()                           # counter bytes per launch (or None)
    alg_step128 = apps * 2 * dim * 16
    result = {
        "metric": "Trotter steps/s (grouped, c64 amplitudes + FP64 phase), n=28 random k-local",
        "value": round(sps64, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t64 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random_klocal_n28", "n_qubits": n, "terms": int(info.n_terms),
                   "groups": K, "order": 1, "dt": m.dt,
                   "storage": "complex64", "seed": 3, "init_seed": m.init_seed,
                   "tile_log2_c64": int(opts.tile_log2_c64), "tile_log2_c128": int(opts.tile_log2_c128),
                   "coalesce_log2_c64": int(opts.coalesce_log2_c64),
                   "coalesce_min_log2_c64": int(opts.coalesce_min_log2_c64)},
        "autotune": tune,
        "c128_steps_per_s": round(sps128, 4),
        "c64_over_c128": round(sps64 / sps128, 3),
        "group_applications_per_step": apps,
        "passes_per_step_c64": int(info.passes_c64),
        "passes_per_step_c128": int(info.passes_c128),
        "paper_model_passes_per_step": int(info.paper_model_passes),
        "algorithmic_bytes_per_step_c64": alg_step64,
        "hbm_gbps_algorithmic_c64": round(achieved, 1),
        "hbm_gbps_algorithmic_c128": round(alg_step128 * k128 / t128 / 1e9, 1),
        "frac_of_hbm_peak_c128": round(alg_step128 * k128 / t128 / 1e9 / HBM_PEAK_GBPS, 4),
        "accuracy_c64_vs_c128": {"steps": steps_acc, "fidelity": fid, "l2": l2, "max_abs": maxerr,
                                 "norm_drift_c64": n64 - 1.0, "norm_drift_c128": n128 - 1.0,
                                 "energy_drift_c64": e64 - e0, "energy_drift_c128": e128 - e0},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": ROOFLINE_KERNEL,
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "units_per_launch": round(apps / info.passes_c64, 4),
                     "bytes_per_unit": unit64,
                     "pass_bytes_per_launch": unit64,
                     "pass_gbps_per_launch": round(pass_gbps, 1),
                     "traffic_per_step": None if traffic is None else traffic * int(info.passes_c64),
                     "traffic_over_algorithmic": None if traffic is None
                     else round(traffic * int(info.passes_c64) / alg_step64, 3)},
    }

    if not args.no_reference_modes:
        # the paper's own comparison on this GPU: term-by-term rotations (its
        # baseline) and its circuit applied layer by layer, one step each, c64
        ref = {}
        for name, mode in (("termwise", sd.SD_MODE_TERMWISE), ("paper_layers", sd.SD_MODE_PAPER_LAYERS)):
            log(f"reference mode {name}")
            o = sd.sd_plan_options_default()
            o.mode = mode
            rp = sd.Plan(n, m.paulis, m.coeffs, o).bind("cuda")
            a = d128_0.to(torch.complex64)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            rp.evolve(a, m.dt, 1, 1)
            ev1.record(stream)
            torch.cuda.synchronize()
            sec = ev0.elapsed_time(ev1) / 1e3
            ref[name + "_steps_per_s"] = round(1.0 / sec, 5)
            ref["tiles_speedup_vs_" + name] = round(sps64 * sec, 2)
            del a, rp
        ref["termwise_passes_per_step"] = int(info.n_terms)
        result["paper_comparison_c64"] = ref

    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle sample, 3 runs)")
        t = oracle.build_terms(n, m.paulis, m.coeffs)
        k = min(args.cpu_sample_terms, len(t.c))
        import ctypes
        xs = np.ascontiguousarray(t.x[:k], dtype=np.uint64)
        zs = np.ascontiguousarray(t.z[:k], dtype=np.uint64)
        th = np.ascontiguousarray(t.c[:k] * m.dt, dtype=np.float64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        runs = []
        for _ in range(3):
            psi = psi_host.copy()
            ts = time.time()
            oracle.lib().or_apply_rotations(n, psi.view(np.float64).ctypes.data_as(dp), k,
                                            xs.ctypes.data_as(u64p), zs.ctypes.data_as(u64p),
                                            th.ctypes.data_as(dp))
            runs.append(time.time() - ts)
            del psi
        med = sorted(runs)[1]
        per_rot = med / k
        result["cpu_baseline"] = {
            "value": round(1.0 / (per_rot * len(t.c)), 6), "unit": "steps/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{k} of {len(t.c)} term rotations of one Trotter step at n={n} (FP64), "
                      f"median of 3 runs ({', '.join(f'{r:.1f}' for r in runs)} s); "
                      f"steps/s = 1/(time per rotation x {len(t.c)})"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
