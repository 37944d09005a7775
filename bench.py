"""Benchmark: grid-point RK-stage updates per second of the coupled BSSN +
Valencia GRMHD spectral stage on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A step is one classic RK4 step (four RHS evaluations + RK updates) followed by
the spectral filter, over the whole grid of the workload, with the state
resident in HBM.  value = points x 4 x K / (wall time of K steps).  Prints one
JSON line.  Also reported: per-launch durations measured with HIP events on
the library's stream (the dominant kernel's roofline), the bandwidth a plain
device copy reaches on this GPU, and the plain FP64 oracle timed on this
host: two full RK4 steps of the same workload and the ten steps of the 16^3
workload with the BLAS pool on every core this process may use, and one RK
stage of the same workload on one thread."""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "point-updates/s per RK stage (BSSN+GRMHD), FP64 vs mixed; p50/p99 job latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 (matrix and vector)
RIDGE = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)


def progress(msg):
    """One progress line on stderr (the JSON result goes to stdout)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def launch_costs(nr, nth, nph):
    """Per grid point, for one launch of each kind: algorithmic HBM bytes
    (compulsory reads + writes of that launch) and the FP64 MFMA flops the
    kernel executes.  A dense line operator costs 2N flops per output; the
    folded (even/odd) form used for even N costs N."""
    d = 8.0
    def fl(n):
        return n if n % 2 == 0 else 2 * n
    c = {}
    c["c2p_flux"] = (54 * d, 0.0)                       # 24 in, 30 out
    c["deriv_r2"] = (33 * d, 2 * fl(nr) * 11)           # 11 in, 22 out
    c["deriv_r1"] = (20 * d, fl(nr) * 10)               # 10 in, 10 out
    c["deriv_t2"] = (33 * d, 2 * fl(nth) * 11)
    c["deriv_t1"] = (42 * d, fl(nth) * 21)              # 10 + 11 mixed in, 21 out
    c["deriv_p2"] = (33 * d, 2 * fl(nph) * 11)
    c["deriv_p1"] = (64 * d, fl(nph) * 32)              # 10 + 22 mixed in, 32 out
    for k, n in (("dflux_r", nr), ("dflux_t", nth), ("dflux_p", nph)):
        c[k] = (16 * d, fl(n) * 8)                      # 8 fluxes in, 8 out
    # one launch per axis holding both kinds of task (folded FP64 / FP32 forms)
    for k, a, b in (("deriv_r", "deriv_r2", "deriv_r1"), ("deriv_t", "deriv_t2", "deriv_t1"),
                    ("deriv_p", "deriv_p2", "deriv_p1")):
        c[k] = (c[a][0] + c[b][0], c[a][1] + c[b][1])
    c["ricci"] = (84 * d, 0.0)                          # a separate Ricci launch (none in the stage)
    # RHS with the Ricci tensor: mean over the 4 stage modes (255, 319, 319, 255)
    c["rhs_rk"] = (287 * d, 0.0)
    for k, n in (("filter_r", nr), ("filter_t", nth), ("filter_p", nph)):
        c[k] = (64 * d, fl(n) * 32)
    return c


def fixed_launch_costs(nr, nth, nph):
    """launch_costs for the fixed-background (Cowling) stage: the same
    recovery and flux-derivative launches, the GRMHD-only RHS kernel
    (background 15 fields and 33 first derivatives, stage fluid 8, primitives
    5, flux derivatives 24, and the RK traffic of the 8 GRMHD fields: mean over
    the 4 stage modes of 109 doubles) and a filter over the 8 GRMHD fields."""
    d = 8.0
    c = launch_costs(nr, nth, nph)
    c["rhs_rk"] = (109 * d, 0.0)
    for k, n in (("filter_r", nr), ("filter_t", nth), ("filter_p", nph)):
        c[k] = (16 * d, (n if n % 2 == 0 else 2 * n) * 8)
    return c


def bound_of(kind, costs):
    b, f = costs[kind]
    return "mfma" if f > 0 and f / b > RIDGE else "hbm"


def ideal_ms(kind, P, costs):
    b, f = costs[kind]
    return max(b * P / (HBM_PEAK_GBS * 1e9), f * P / (FP64_PEAK_TFLOPS * 1e12)) * 1e3


def roofline(kind, ms, P, costs):
    b, f = costs[kind]
    sec = ms * 1e-3
    if bound_of(kind, costs) == "mfma":
        ach = f * P / sec / 1e12
        return {"kernel": kind, "bound": "mfma", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS, "traffic": None}
    ach = b * P / sec / 1e9
    return {"kernel": kind, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None}


def cpu_baseline(w):
    """The oracle as it stands, timed on this host.  Cores: the CPUs this
    process may run on (os.sched_getaffinity), and the BLAS pool is set to
    that many threads (the oracle's einsum, FFT and elementwise work runs on
    one thread whatever the pool).  value: two full RK4 steps of the workload
    (8 RHS evaluations, 8 stage updates, 2 filter passes) from the oracle's
    initial data, points x 4 x 2 / wall time.  Also: all ten steps of the
    16^3 workload, and one RK stage of the workload with the pool set to one
    thread."""
    from oracle import spectral, evolve
    from threadpoolctl import threadpool_limits
    cores = len(os.sched_getaffinity(0))

    def setup(wl):
        ga, pk, ik = workloads.oracle_kwargs(wl)
        g = spectral.Grid(*ga)
        pb = evolve.Problem(g, **pk)
        U, K0, _ = evolve.initial_state(g, pb, **ik)
        return g, pb, U, K0

    def timed_steps(wl, nsteps, threads):
        g, pb, U, K0 = setup(wl)
        dt = pb.dt()
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            pb.evolve(U, K0, dt, nsteps)
            t = time.perf_counter() - t0
        return g.npts * 4 * nsteps / t, t

    name = "x".join(str(w["grid"][k]) for k in ("nr", "nth", "nph"))
    rate, t = timed_steps(w, 2, cores)
    progress(f"oracle: 2 RK4 steps of {name} on {cores} cores, {t:.1f} s")
    w16 = workloads.WORKLOADS["ks_michel_16x16x16"]
    rate16, t16 = timed_steps(w16, w16["steps"], cores)
    rate16_1, t16_1 = timed_steps(w16, w16["steps"], 1)
    g, pb, U, K0 = setup(w)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        k1 = pb.rhs(U, K0)
        U1 = U + 0.5 * pb.dt() * k1
        t1 = time.perf_counter() - t0
    progress(f"oracle: 16^3 10 steps {t16:.1f} s ({cores} cores), {t16_1:.1f} s (1 thread); "
             f"one stage of {name} on 1 thread {t1:.1f} s")
    del U1
    return {"value": rate, "unit": "point-stage updates/s", "cores": cores, "kind": "oracle",
            "sample": f"two full RK4 steps of {name} (8 RHS evaluations and stage updates, 2 filter passes) "
                      f"from the oracle's initial data (untimed), {t:.1f} s; NumPy FP64, BLAS pool "
                      f"{cores} threads (the CPUs this process may use), einsum/FFT/elementwise on one thread",
            "seconds": round(t, 2),
            "ks_michel_16x16x16_10_steps": {"value": rate16, "seconds": round(t16, 3), "threads": cores},
            "single_thread": {"ks_michel_16x16x16_10_steps": {"value": rate16_1, "seconds": round(t16_1, 3)},
                              f"one_rk_stage_{name}": {"value": g.npts / t1, "seconds": round(t1, 2)}}}


def stream_ceiling(torch):
    """Bandwidth of plain device streams on this GPU (torch's own kernels):
    a copy of 1 GiB (read + write) and a three-array add c = a + b of 1 GiB
    arrays, beyond the last-level cache; and copies of 32, 128 and 512 MiB
    (32 MiB each way is what one flux-derivative launch of 64x64x128 moves),
    to show how the rate of a single short launch falls with its size.
    Median of 10 timed launches with HIP events on the current stream, after
    3 untimed ones."""
    n = 128 * 1024 * 1024  # doubles: 1 GiB per array
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)

    def rate(fn, nbytes):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(10):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return round(nbytes / sorted(ts)[len(ts) // 2] / 1e9, 1)

    out = {"copy_GB_per_s": rate(lambda: c.copy_(a), 2 * 8 * n),
           "add_GB_per_s": rate(lambda: torch.add(a, b, out=c), 3 * 8 * n),
           "bytes_per_array": 8 * n, "copy_GB_per_s_by_size": {}}
    for mib in (32, 128, 512):
        m = mib * 1024 * 1024 // 8
        out["copy_GB_per_s_by_size"][f"{mib}MiB"] = rate(lambda: c[:m].copy_(a[:m]), 2 * 8 * m)
    del a, b, c
    torch.cuda.empty_cache()
    return out


# tensor groups of the 32 evolved fields (phi | gt | At | K | Gt and the driver
# | alpha | beta | D | S_j | tau | B): per-field errors are scaled by the
# largest magnitude in the field's group
GROUPS = [[0], list(range(1, 7)), list(range(7, 13)), [13], [14, 15, 16, 21, 22, 23], [17],
          [18, 19, 20], [24], [25, 26, 27], [28], [29, 30, 31]]


def group_errors(got, ref):
    import numpy as np
    e = [0.0] * 32
    for grp in GROUPS:
        sg = max(float(np.abs(ref[f]).max()) for f in grp)
        for f in grp:
            den = max(float(np.abs(ref[f]).max()), sg)
            d = float(np.abs(got[f] - ref[f]).max())
            e[f] = 0.0 if d == 0 else (d / den if den > 0 else float("inf"))
    return e


def mixed_forms(w, K, fp64_rate, Solver, make_grid, make_phys, torch):
    """Reduced-precision forms (FP32 and split-BF16x3 contractions, FP64
    contractions with FP32 derivative arrays): the same K steps from the same
    initial data; throughput, speedup over FP64, and the
    errors against the FP64 path (itself equal to the oracle to 1e-11 per
    field): density L2 relative (unweighted over the nodes), the ratio of
    Hamiltonian-constraint L2 norms, and the per-field relative error of all
    32 fields (tensor-group scaled)."""
    ref = Solver(make_grid(**w["grid"]), make_phys(**w["phys"]), prec=0)
    ref.init_state()
    ref.step(K)
    d_ref = ref.diagnostics()
    U_ref = ref.get_state()
    shape = ref.shape
    prim_ref = torch.empty((5,) + shape, dtype=torch.float64, device="cuda")
    ref.con2prim(ref.U, prim_ref)
    rho_ref = prim_ref[0].clone()
    ref.close()
    out = {"reference": "the FP64 GPU path after the same steps (equal to the oracle to 1e-11 per field)",
           "store32": "FP64 MFMA contractions, FP32 derivative arrays (GRMHD_STORE_FP32)"}
    out["fp64_from_fp32_rounded_state"] = sensitivity(
        w, K, {"fp64": U_ref, "fp64_rho": rho_ref.cpu().numpy(), "fp64_ham_l2": d_ref["ham_l2"]}, torch, Solver,
        make_grid, make_phys)
    g = w["grid"]
    P = g["nr"] * g["nth"] * g["nph"]
    for name, prec in (("fp32", 1), ("bf16x3", 2), ("store32", 3)):
        s = Solver(make_grid(**w["grid"]), make_phys(**w["phys"]), prec=prec)
        s.init_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        d = s.diagnostics()
        prim = torch.empty_like(prim_ref)
        s.con2prim(s.U, prim)
        rho = prim[0]
        l2 = float(torch.sqrt(torch.sum((rho - rho_ref) ** 2) / torch.sum(rho_ref ** 2)))
        rate = P * 4 * K / wall
        ef = group_errors(s.get_state(), U_ref)
        out[name] = {"value": rate, "speedup_vs_fp64": rate / fp64_rate, "ms_per_step": wall * 1e3 / K,
                     "rho_l2_rel_vs_fp64": l2, "ham_l2": d["ham_l2"], "ham_l2_fp64": d_ref["ham_l2"],
                     "ham_ratio": d["ham_l2"] / d_ref["ham_l2"], "c2p_fail": d["c2p_fail"],
                     "nonfinite": d["nonfinite"], "field_rel_err_max": max(ef),
                     "field_rel_err": [float(f"{x:.3g}") for x in ef],
                     "within_bounds": bool(l2 <= 1e-6 and d["ham_l2"] <= 2 * d_ref["ham_l2"])}
        s.close()
    return out


def glm_study(w_main, K_main, value_fp64, torch, Solver, make_grid, make_phys):
    """GLM constraint damping (psi field; c_h = 1, tau = 0.5): the main
    workload's throughput with it on, and its cleaning effect on 16^3 on the
    fixed Kerr-Schild background (only the GRMHD fields evolve) from the
    library's initial data with a divergence-carrying field perturbation:
    max |d_i(sqrt(gamma) B^i)| (library diagnostics) every 25 RK4 steps up to
    200 (t = 1.77 M), with and without it."""
    glm = dict(glm=True, glm_ch=1.0, glm_tau=0.5)
    g = w_main["grid"]
    P = g["nr"] * g["nth"] * g["nph"]
    s = Solver(make_grid(**g), make_phys(**dict(w_main["phys"], **glm)))
    s.init_state()
    s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(K_main)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = s.diagnostics()
    s.close()
    out = {"c_h": 1.0, "tau": 0.5, "value": P * 4 * K_main / wall, "ms_per_step": wall * 1e3 / K_main,
           "cost_vs_plain": value_fp64 / (P * 4 * K_main / wall), "nonfinite": d["nonfinite"]}
    w16 = workloads.WORKLOADS["ks_michel_16x16x16"]
    study = {"grid": [16, 16, 16], "background": "fixed (Cowling)", "steps_between": 25, "max_abs_divB": {},
             "nonfinite_end": {}}
    for name, on in (("with_glm", True), ("without_glm", False)):
        phys = dict(w16["phys"], cowling=True, **(glm if on else {}))
        s = Solver(make_grid(**w16["grid"]), make_phys(**phys))
        s.init_state()
        U = workloads.divergence_seed(w16["grid"], s.get_state())
        s.set_state(U, s.get_state(with_k0=True)[1])
        series = [s.diagnostics()["max_abs_divB"]]
        for _ in range(8):
            s.step(25)
            series.append(s.diagnostics()["max_abs_divB"])
        study["t_end"] = s.time
        study["max_abs_divB"][name] = series
        study["nonfinite_end"][name] = s.diagnostics()["nonfinite"]
        s.close()
    out["divergence_study"] = study
    return out


def fixed_background(w, K, value_fp64, torch, Solver, make_grid, make_phys):
    """Fixed-background (Cowling) form of the main workload: only the 8
    GRMHD fields evolve on the Kerr-Schild background (its first derivatives
    computed once).  FP64 and FP32-form throughput, per-launch times and the
    RHS kernel's roofline."""
    g = w["grid"]
    P = g["nr"] * g["nth"] * g["nph"]
    costs = fixed_launch_costs(g["nr"], g["nth"], g["nph"])
    out = {"workload": "fixed Kerr-Schild background, " + "x".join(str(g[k]) for k in ("nr", "nth", "nph"))}
    for name, prec in (("fp64", 0), ("fp32", 1)):
        s = Solver(make_grid(**g), make_phys(**dict(w["phys"], cowling=True)), prec=prec)
        s.init_state()
        s.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = s.profile_step(2)
        d = s.diagnostics()
        s.close()
        r = {"value": P * 4 * K / wall, "unit": "point-stage updates/s", "ms_per_step": wall * 1e3 / K,
             "vs_coupled_fp64": (P * 4 * K / wall) / value_fp64, "nonfinite": d["nonfinite"],
             "c2p_fail": d["c2p_fail"],
             "kernels_ms": {k: round(v[0], 5) for k, v in prof.items() if v[1]}}
        if prec == 0:
            r["roofline"] = roofline("rhs_rk", prof["rhs_rk"][0], P, costs)
            r["roofline"]["kernel"] = "rhs_fixed"
            r["roofline"]["traffic"] = traffic_record("rhs_fixed")
            r["stage_ideal_ms_per_step"] = round(sum(ideal_ms(k, P, costs) * v[1] / 2 for k, v in prof.items()
                                                     if v[1]), 5)
        out[name] = r
    return out


def paper_variants(w, K, torch, Solver, make_grid, make_phys):
    """How far the paper's literal scheme is from the unsplit hot path on the
    main workload: the operator-split coupled step, 2/3 dealiasing and the
    damped primitive recovery, each alone, over the same K steps from the
    library's initial data; step time and the largest per-group relative
    difference from the unsplit FP64 path (groups as in the parity tests)."""
    import numpy as np
    g = w["grid"]
    variants = (("unsplit", {}, {}), ("operator_split", {}, {"split": True}), ("dealias_2_3", {"dealias": True}, {}),
                ("damped_c2p", {}, {"c2p": "damped"}))
    states, out = {}, {"workload": "x".join(str(g[k]) for k in ("nr", "nth", "nph")), "steps": K}
    for name, gk, pk in variants:
        s = Solver(make_grid(**dict(g, **gk)), make_phys(**dict(w["phys"], **pk)))
        s.init_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        states[name] = s.get_state()
        d = s.diagnostics()
        s.close()
        out[name] = {"ms_per_step": wall * 1e3 / K, "nonfinite": d["nonfinite"], "c2p_fail": d["c2p_fail"],
                     "ham_l2": d["ham_l2"]}
    ref = states["unsplit"]
    for name, _, _ in variants[1:]:
        diff = [float(np.abs(states[name][q] - ref[q]).max() / np.abs(ref[q]).max()) for q in GROUPS]
        out[name]["max_group_rel_diff_vs_unsplit"] = max(diff)
        out[name]["group_rel_diff_vs_unsplit"] = [float(f"{x:.3g}") for x in diff]
    return out


def second_config(name, torch, Solver, make_grid, make_phys, profile_steps=2):
    """A second measured configuration (the magnetised torus at 128x96x192):
    FP64 and FP32-form throughput over the workload's step count from the
    library's initial data, the dominant launch's roofline, the stage
    fraction, and the FP32 form's errors against the FP64 path after the same
    1 + K steps; and the FP64 path from the FP32-rounded initial state (how
    far FP32-level rounding alone moves this evolution)."""
    w = workloads.WORKLOADS[name]
    g = w["grid"]
    P = g["nr"] * g["nth"] * g["nph"]
    K = w["steps"]
    costs = launch_costs(g["nr"], g["nth"], g["nph"])
    out = {"workload": name, "grid": [g["nr"], g["nth"], g["nph"]], "points": P, "steps": K}
    states = {}
    for name_p, prec in (("fp64", 0), ("fp32", 1), ("store32", 3)):
        s = Solver(make_grid(**g), make_phys(**w["phys"]), prec=prec)
        s.init_state()
        s.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        d = s.diagnostics()
        rec = {"value": P * 4 * K / wall, "ms_per_step": wall * 1e3 / K, "c2p_fail": d["c2p_fail"],
               "nonfinite": d["nonfinite"], "ham_l2": d["ham_l2"]}
        # the state after the warm-up and the timed steps (1 + K), before the
        # profiled steps below advance it further
        states[name_p] = s.get_state()
        states[name_p + "_ham_l2"] = d["ham_l2"]
        prim = torch.empty((5,) + s.shape, dtype=torch.float64, device="cuda")
        s.con2prim(s.U, prim)
        states[name_p + "_rho"] = prim[0].cpu().numpy()
        if prec == 0:
            prof = s.profile_step(profile_steps)
            per_step = {k: ms * cnt / profile_steps for k, (ms, cnt) in prof.items()}
            dom = max(per_step, key=per_step.get)
            rec["roofline"] = roofline(dom, prof[dom][0], P, costs)
            ideal = sum(ideal_ms(k, P, costs) * cnt / profile_steps for k, (ms, cnt) in prof.items())
            rec["stage_roofline_fraction"] = round(ideal / rec["ms_per_step"], 3)
            rec["serial_launch_sum_ms_per_step"] = round(sum(per_step.values()), 5)
            rec["kernels_avg_ms"] = {k: round(ms, 5) for k, (ms, cnt) in prof.items()}
        out[name_p] = rec
        s.close()
    import numpy as np
    out["fp64_from_fp32_rounded_state"] = sensitivity(w, K + 1, states, torch, Solver, make_grid, make_phys)
    r64 = states["fp64_rho"]
    for name_p in ("fp32", "store32"):
        r32 = states[name_p + "_rho"]
        o = out[name_p]
        o["speedup_vs_fp64"] = o["value"] / out["fp64"]["value"]
        o["rho_l2_rel_vs_fp64"] = float(np.sqrt(np.sum((r32 - r64) ** 2) / np.sum(r64 ** 2)))
        o["ham_ratio"] = o["ham_l2"] / out["fp64"]["ham_l2"]
        ef = group_errors(states[name_p], states["fp64"])
        o["field_rel_err_max"] = max(ef)
        o["field_rel_err"] = [float(f"{x:.3g}") for x in ef]
        o["within_bounds"] = bool(o["rho_l2_rel_vs_fp64"] <= 1e-6 and o["ham_ratio"] <= 2.0)
    return out


def sensitivity(w, K, states, torch, Solver, make_grid, make_phys):
    """How far FP32 rounding of the state alone moves the FP64 evolution: the
    FP64 path from the initial state rounded once to FP32 (K0 exact), the
    same K steps, against the FP64 path from the exact state
    (states["fp64"], states["fp64_rho"]): density L2, Hamiltonian-constraint
    ratio and the largest per-field error.  The FP32 and split-BF16x3 forms
    round their contraction inputs (the state) at least this much at every
    stage, so where this exceeds the bounds they cannot meet them; the
    FP32-storage form rounds only the computed derivatives."""
    import numpy as np
    s = Solver(make_grid(**w["grid"]), make_phys(**w["phys"]))
    s.init_state()
    U0, K0 = s.get_state(with_k0=True)
    s.set_state(U0.astype(np.float32).astype(np.float64), K0)
    s.step(K)
    d = s.diagnostics()
    got = s.get_state()
    prim = torch.empty((5,) + s.shape, dtype=torch.float64, device="cuda")
    s.con2prim(s.U, prim)
    rho = prim[0].cpu().numpy()
    s.close()
    r64 = states["fp64_rho"]
    d64 = states.get("fp64_ham_l2")
    return {"rho_l2_rel_vs_fp64": float(np.sqrt(np.sum((rho - r64) ** 2) / np.sum(r64 ** 2))),
            "ham_ratio": d["ham_l2"] / d64 if d64 else None, "c2p_fail": d["c2p_fail"],
            "field_rel_err_max": max(group_errors(got, states["fp64"])), "steps": K}


def traffic_probe(w, torch, Solver, make_grid, make_phys):
    """Workload for the HBM traffic counters (run under rocprofv3 --pmc): one
    plain device copy of 512 MiB (the counters' scale reference: 512 MiB read,
    512 MiB written) followed by one FP64 RK4 step of the workload, its
    launches in order on one stream (the profiled form of the step), then one
    step of its fixed-background form (after the one-off background
    derivatives)."""
    n = 64 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    s = Solver(make_grid(**w["grid"]), make_phys(**w["phys"]))
    s.init_state()
    s.profile_step(1)  # every launch in order on one stream
    torch.cuda.synchronize()
    s.close()
    s = Solver(make_grid(**w["grid"]), make_phys(**dict(w["phys"], cowling=True)))
    s.init_state()
    s.profile_step(1)
    torch.cuda.synchronize()
    s.close()
    print(json.dumps({"traffic_probe": True, "copy_bytes_each_way": n * 8, "steps": 1, "fixed_steps": 1}),
          flush=True)


def traffic_record(kernel):
    """HBM bytes per launch of `kernel` measured with the FETCH_SIZE and
    WRITE_SIZE counters (profiles/), reported only while the kernel source is
    the one that was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_ks_michel_64x64x128.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2508_18221_amd", "csrc", rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ks_michel_64x64x128")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-second", action="store_true", help="skip the 128x96x192 torus configuration")
    ap.add_argument("--no-glm", action="store_true", help="skip the GLM constraint-damping measurements")
    ap.add_argument("--no-fixed", action="store_true", help="skip the fixed-background (Cowling) form")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the paper-literal variants (split step, 2/3 dealiasing, damped recovery)")
    ap.add_argument("--serve-t-scale", type=float, default=1e-3)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one 512 MiB copy + one RK4 step, for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is described in the design notes, not built",
              file=sys.stderr)
        sys.exit(2)
    w = workloads.WORKLOADS[args.workload]
    K = args.steps if args.steps is not None else w["steps"]
    W = args.warmup

    import torch
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    torch.cuda.set_device(0)
    if args.traffic_probe:
        traffic_probe(w, torch, Solver, make_grid, make_phys)
        return
    s = Solver(make_grid(**w["grid"]), make_phys(**w["phys"]))
    g = w["grid"]
    P = g["nr"] * g["nth"] * g["nph"]
    s.init_state()
    if W > 0:
        s.step(W)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(3):  # three timed runs of K steps; the median is reported
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        s.step(K)
        e1.record()
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0, e0.elapsed_time(e1)))
    runs_sorted = sorted(runs)
    wall, ev_ms = runs_sorted[1]
    diag = s.diagnostics()
    # per-launch durations (HIP events on the library stream), a few more steps
    prof = s.profile_step(args.profile_steps)
    costs = launch_costs(g["nr"], g["nth"], g["nph"])
    per_step = {k: ms * cnt / args.profile_steps for k, (ms, cnt) in prof.items()}
    dom = max(per_step, key=per_step.get)
    rl = roofline(dom, prof[dom][0], P, costs)
    rl["traffic"] = traffic_record(dom)
    kernels = {}
    ideal_step = measured_step = 0.0
    for k, (ms, cnt) in prof.items():
        n = cnt // args.profile_steps
        ideal = ideal_ms(k, P, costs)
        kernels[k] = {"avg_ms": round(ms, 5), "launches_per_step": n,
                      "GB_per_s": round(costs[k][0] * P / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                      "TFLOP_per_s": round(costs[k][1] * P / (ms * 1e-3) / 1e12, 2) if ms > 0 else None,
                      "bound": bound_of(k, costs), "ideal_ms": round(ideal, 5),
                      "frac": round(ideal / ms, 3) if ms > 0 else None}
        ideal_step += ideal * n
        measured_step += ms * n
    s.close()
    out = {
        "metric": METRIC,
        "value": P * 4 * K / wall,
        "unit": "point-stage updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall * 1e3 / K,
        "ms_per_step_hip_events": ev_ms / K,
        "ms_per_step_runs": [round(w * 1e3 / K, 5) for w, _ in runs],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [g["nr"], g["nth"], g["nph"]], "points": P,
                   "rk_stages_per_step": 4, "precision": "fp64",
                   "physics": "Kerr-Schild a=0.5 + magnetised Michel accretion, BSSN+1+log+Gamma-driver"},
        "state_after": {"t": diag["t"], "c2p_fail": diag["c2p_fail"], "nonfinite": diag["nonfinite"],
                        "rest_mass": diag["rest_mass"], "ham_l2": diag["ham_l2"]},
        "roofline": rl,
        "stage_roofline_fraction": round(ideal_step / (wall * 1e3 / K), 3),
        "serial_launch_sum_ms_per_step": round(measured_step, 5),
        "kernels": kernels,
    }
    progress(f"main workload done: {out['value']:.4g} point-stage updates/s")
    out["stream_ceiling"] = stream_ceiling(torch)
    progress("stream ceiling done")
    if not args.no_mixed:
        out["mixed_precision"] = mixed_forms(w, K, out["value"], Solver, make_grid, make_phys, torch)
        progress("mixed-precision forms done")
    if not args.no_second:
        out["second_config"] = second_config("ks_torus_128x96x192", torch, Solver, make_grid, make_phys)
        progress("torus 128x96x192 done")
    if not args.no_glm:
        out["glm"] = glm_study(w, K, out["value"], torch, Solver, make_grid, make_phys)
        progress("GLM form done")
    if not args.no_fixed:
        out["fixed_background"] = fixed_background(w, K, out["value"], torch, Solver, make_grid, make_phys)
        progress("fixed-background form done")
    if not args.no_variants:
        out["paper_variants"] = paper_variants(w, K, torch, Solver, make_grid, make_phys)
        progress("paper-literal variants done")
    if not args.no_serving:
        from paper_2508_18221_amd.serve import run_stream
        jobs = workloads.served_stream(256, 4.0, t_scale=args.serve_t_scale)
        out["serving"] = {"stream": "256 jobs, Poisson arrivals 4/s, a~U[0,0.95], beta~logU[10,1000], "
                                    "grids {16^3, 32x32x64, 48x48x96, 64x64x128}, Michel+field, "
                                    f"T~U[10,100] M scaled by {args.serve_t_scale:g}, HBM budget 200 GB",
                          "t_scale": args.serve_t_scale}
        out["serving"]["fp64"] = run_stream(jobs, prec=0, budget=200e9, log=progress)
        progress("served stream (fp64) done")
        # capacity and per-grid latency under overload: the same 256 jobs all
        # arriving at t = 0 (continuous batching at full load), FP64, FP32 and
        # FP32 storage
        burst = [dict(j, arrival=0.0) for j in jobs]
        for name, prec in (("fp64_burst", 0), ("fp32_burst", 1), ("store32_burst", 3)):
            out["serving"][name] = run_stream(burst, prec=prec, budget=200e9, log=progress)
            progress(f"served burst ({name}) done")
        # mixed workload: half the jobs on the fixed background (a second job class per grid)
        mix = workloads.served_stream(256, 4.0, t_scale=args.serve_t_scale, cowling_frac=0.5)
        out["serving"]["fp64_half_fixed_background"] = run_stream(mix, prec=0, budget=200e9, log=progress)
        progress("served mixed workload done")
        out["serving"]["fp64_half_fixed_background"]["fixed_background_jobs"] = sum(j["cowling"] for j in mix)
    if not args.no_cpu_baseline:
        progress("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
