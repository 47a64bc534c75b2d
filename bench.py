"""Benchmark: damaged TLSPH steps on one MI355X.

Default workload (the headline): the GTN holed plate in plane-strain-like
tension (100 x 40 x 2 mm, central hole of 5 mm diameter, 0.125 mm lattice,
4 075 776 particles, seeded 3 % jitter), Johnson-Cook matrix flow and
Gurson-Tvergaard-Needleman damage (Algorithm 2 in double in both forms),
grips driven at +-10 m/s (1 - exp(-t / 1 ms)), v_z = 0 everywhere.  The plate
is first driven along the ramp, untimed, until at least 2 % of its particles
yield in a step; the timed steps follow from there, so the GTN return
mapping's Newton loops run in them.  A step is one pass of the whole path:
nodal forces with hourglass control, leapfrog update, damaged dF/dt, EOS,
return mapping, damage, PK1.  The headline value is the FP64 form; the mixed
FP32/FP64 form takes over the same state and is timed over the same steps.

Other workloads (--workload): the notched round bar (200 216 particles, JC
damage, from rest to past failure, with its failure displacement), the
Taylor bar (996 314 particles, CL, rigid wall, 5000 steps), and a batch of
256 notched bars of 2k-60k particles (8.55 M in all), among others.

Inputs and state are resident in HBM before the timed region starts.
Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s + achieved HBM GB/s; mixed FP32 vs FP64 at stated error"
HBM_PEAK_GBS = 8000.0
DIAG_EVERY = 20
TIMING_STRIDE = 10

# Algorithmic HBM bytes per particle of each step kernel: every per-particle
# field the kernel needs is read (or written) once; neighbour data is served
# by caches and not counted; plus 4 bytes of neighbour index per pair.
#   force pass  reads X,V0 (32) u (24) Q,F-I,1-D (152 | 76) D (8) v (24)
#               group, specimen, count (12); writes v,V0(1-D) (32) u (24)
#   deformation reads X,V0 (32) v (24) L^-1 (72 | 36) F-I (72 | 36)
#   pass        sigma (48 | 24) eps_p, rate, e, D (32) specimen, count (8)
#               + damage accumulators; writes Q,F-I,1-D (152 | 76),
#               sigma (48 | 24), eps_p, rate, e, D (32) + accumulators
ACC_BYTES = {0: 0, 1: 32, 2: 16, 3: 16}   # CL: D_init, W_p r/w; JC: D_init; GTN: f


def algorithmic_bytes(kernel: str, mixed: bool, damage: int, n: int, nnz: int,
                      av: bool = False, var_h: bool = False) -> int:
    """Bytes one launch must move: each per-particle field once, 4 bytes of
    neighbour index per pair.  The damping's force is written by the
    deformation pass and read by the force pass (24 bytes each); graded
    spacing reads each particle's support in both passes (8 bytes)."""
    if kernel == "force_pass":
        per = 32 + 24 + (76 if mixed else 152) + 8 + 24 + 12 + 32 + 24
    else:
        per = (32 + 24 + (36 if mixed else 72) * 2 + (24 if mixed else 48) + 32 + 8
               + (76 if mixed else 152) + (24 if mixed else 48) + 32)
        per += ACC_BYTES[damage]
    per += (24 if av else 0) + (8 if var_h else 0)
    return per * n + 4 * nnz


def kernel_symbol(kernel: str, info: dict, mixed: bool, model: int, flow_general=False,
                  var_h=False) -> str:
    """Kernel name as rocprofv3 reports it (template arguments included);
    model is the damage model the deformation pass is compiled for (-1: any),
    flow_general whether it is the variant with every flow law, var_h whether
    the kernels take per-pair supports (graded spacing: the general variant)."""
    r = "float" if mixed else "double"
    vh = "true" if var_h else "false"
    if kernel == "force_pass":
        name = "k_pass_b_staged" if info["staged"] else "k_pass_b"
        return f"{name}<{r}, {info['lanes_per_particle']}, {vh}>"
    name = "k_pass_a_staged" if info["block_deformation"] <= 0 else "k_pass_a"
    if var_h:
        model, flow_general = -1, True
    return f"{name}<{r}, {model}, {'true' if flow_general else 'false'}, {vh}>"


def counter_traffic(symbol: str, workload: str):
    """HBM bytes per launch of one kernel from the committed rocprofv3
    counter summary, if it was taken on the kernels as they are now (else
    None)."""
    from paper_1901_07374_amd.build import source_hash
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != source_hash():
        return None
    key = f"{symbol}_hbm_bytes_per_launch"
    return float(vals[key]) if key in vals else None


def failure_displacement(sep, reaction, level=0.1):
    """Grip separation where the reaction first drops below `level` times its
    running maximum after the peak, interpolated linearly between samples
    (None if it never does)."""
    run_max = 0.0
    peak_seen = False
    prev = None
    for s, r in zip(sep, reaction):
        if r > run_max:
            run_max = r
        elif run_max > 0 and r < 0.98 * run_max:
            peak_seen = True
        if peak_seen and r < level * run_max:
            if prev is None or prev[1] <= r:
                return float(s)
            s0, r0 = prev
            lvl = level * run_max
            return float(s0 + (s - s0) * (r0 - lvl) / (r0 - r))
        prev = (s, r)
    return None


FD_LEVELS = (0.1, 0.5)


def fd_mm(sep, reaction):
    out = {}
    for lvl in FD_LEVELS:
        v = failure_displacement(sep, reaction, lvl)
        out[f"{int(lvl * 100)}%"] = None if v is None else round(v * 1e3, 4)
    return out


def perturbed(I, p, seed, amp=1e-12):
    """The same problem with initial velocities perturbed by +-amp m/s: a
    rounding-level change that shows how far the failure point moves on its
    own."""
    rng = np.random.default_rng(seed)
    return I.Problem(p.name, p.X, p.V0, p.spec_offsets, p.materials, p.bc_group, p.bc_groups,
                     p.v_init + rng.uniform(-amp, amp, p.v_init.shape), p.steps, p.dx)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_form(prob, precision, steps, warmup, torch, T, flags=0, autotune=True, stream=None,
             diag=True, shape=None, k_cap=32, setup=None, sim=None):
    """Warm up, autotune (or apply a given launch shape), then time `steps`
    steps; diagnostics every DIAG_EVERY steps (inside the timed region).  A
    given context continues from its state."""
    log(f"{prob.name}: {prob.n} particles, precision {precision}, flags {flags}")
    if sim is None:
        sim = T.Sim(prob, precision=precision, flags=flags, stream=stream, k_cap=k_cap)
    if setup is not None:
        setup(sim)
    if shape is not None:
        sim.set_launch_shape(*shape)
    n_rec = (warmup + steps) // DIAG_EVERY + 1 if diag else 0
    n_bc = max(len(prob.bc_groups), 1)
    sd = torch.zeros((max(n_rec, 1), prob.n_spec, 8), dtype=torch.float64, device="cuda")
    bd = torch.zeros((max(n_rec, 1), n_bc, 8), dtype=torch.float64, device="cuda")
    L = T.lib()
    rec = 0

    def advance(k):
        nonlocal rec
        if not diag:
            sim.step(k)
            return
        done = 0
        while done < k:
            chunk = min(DIAG_EVERY, k - done)
            sim.step(chunk)
            done += chunk
            if chunk == DIAG_EVERY and rec < n_rec:
                st = L.tlsph_get_diagnostics(
                    sim.ctx, sd[rec].data_ptr(),
                    bd[rec].data_ptr() if prob.bc_groups else None, sim._sp())
                if st:
                    raise RuntimeError("diagnostics failed")
                rec += 1

    advance(warmup)
    if autotune and shape is None:
        sim.autotune()     # picks launch shapes on the current state; results unchanged
    use_timing = not (flags & T.USE_GRAPHS)
    torch.cuda.synchronize()
    if use_timing:
        # every step's kernels timed on short runs, a sample of them on long ones
        sim.enable_kernel_timing(max(1, min(TIMING_STRIDE, steps // 100)))
    t0 = time.perf_counter()
    advance(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = sim.kernel_times() if use_timing else None
    sim.enable_kernel_timing(0)
    log(f"  {steps} steps in {t1 - t0:.3f} s")
    return dict(seconds=t1 - t0, kernel_times=kt, info=sim.info(), sim=sim,
                sd=sd[:rec].cpu().numpy(), bd=bd[:rec].cpu().numpy())


def kernel_table(kt, mixed, damage, n, nnz, av=False, var_h=False):
    kts = {k: v[0] / max(v[1], 1) for k, v in kt.items()}
    return kts, {k: {"avg_launch_us": round(v * 1e3, 2),
                     "algorithmic_GBs": round(algorithmic_bytes(k, mixed, damage, n, nnz, av, var_h)
                                              / (v * 1e-3) / 1e9, 1)} for k, v in kts.items()}


def roofline_of(run, damage, n, workload, mixed=False, flow_general=False, var_h=False,
                av=False):
    nnz = run["info"]["nnz"]
    kts, _ = kernel_table(run["kernel_times"], mixed, damage, n, nnz, av, var_h)
    dom = max(kts, key=kts.get)
    bytes_launch = algorithmic_bytes(dom, mixed, damage, n, nnz, av, var_h)
    achieved = bytes_launch / (kts[dom] * 1e-3) / 1e9
    symbol = kernel_symbol(dom, run["info"], mixed, damage, flow_general, var_h)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(symbol, workload), "kernel": dom, "symbol": symbol,
            "avg_launch_us": round(kts[dom] * 1e3, 2),
            "algorithmic_bytes_per_launch": bytes_launch}


def cpu_baseline(prob, label, target_seconds=15.0, max_steps=400):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload (the same particles, a few steps from the start)."""
    import oracle
    log(f"cpu baseline: {label}")
    o = oracle.Sim(prob)
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    k = int(max(2, min(max_steps, target_seconds / max(one, 1e-6))))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    return {"value": prob.n * k / dt, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{label}, {prob.n} particles, FP64 oracle, {k} steps after 1 untimed "
                      f"step, {threads} OpenMP threads"}


def base_line(args, workload, value, ms_step, dtype, config):
    return {"metric": METRIC, "value": round(value, 1), "unit": "particle-steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": dict({"workload": workload}, **config)}


def launch_shape(info):
    """(staged, lanes, force block, deformation block, tile) of a run."""
    return (int(info["staged"]), info["lanes_per_particle"],
            info["block_force"] if not info["staged"] else 256, info["block_deformation"],
            info["tile"] if info["staged"] else 0)


def shape_of(info):
    return {"force_pass_variant": "LDS-staged tiles" if info["staged"] else "global gathers",
            "tile": info["tile"],
            "force_pass_block": info["block_force"],
            "force_lanes_per_particle": info["lanes_per_particle"],
            "deformation_pass_block": max(info["block_deformation"], 0),
            "deformation_pass_tile": (-info["block_deformation"] if info["block_deformation"] < 0
                                      else info["tile"] if info["block_deformation"] == 0 else 0)}


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
FLOW_NAMES = {0: "johnson-cook", 1: "linear", 2: "swift", 3: "voce"}


def bench_notched_bar(args, torch, I, T, workload="notched_bar_200k", **mat_over):
    prob = I.notched_bar(**mat_over)
    damage = prob.materials[0]["damage"]
    flags = T.NO_STAGING if args.unstaged else 0
    tune = not args.no_autotune

    def curve(r):
        # reaction on the top grip (group 1) and grip separation
        bd = r["bd"]
        return -bd[:, 1, 2], bd[:, 1, 5] - bd[:, 0, 5]

    fp = run_form(prob, T.FP64, args.steps, args.warmup, torch, T, flags, tune)
    nnz = fp["info"]["nnz"]
    _, ktab = kernel_table(fp["kernel_times"], False, damage, prob.n, nnz)
    out = base_line(args, workload, prob.n * args.steps / fp["seconds"],
                    fp["seconds"] / args.steps * 1e3, "f64",
                    dict({"particles": prob.n, "neighbour_pairs": nnz, "damage": "johnson-cook",
                          "flow": FLOW_NAMES[prob.materials[0]["flow"]],
                          "return": "implicit" if prob.materials[0]["implicit_return"] else
                                    "explicit (Algorithm 1)",
                          "precision": "fp64", "steps_from_rest": args.warmup + args.steps,
                          "dt_s": prob.materials[0]["dt"]}, **shape_of(fp["info"])))
    step_bytes = sum(algorithmic_bytes(k, False, damage, prob.n, nnz) for k in ktab)
    out["step_algorithmic_GBs"] = round(step_bytes * args.steps / fp["seconds"] / 1e9, 1)
    out["kernels"] = ktab
    m0 = prob.materials[0]
    out["roofline"] = roofline_of(fp, damage, prob.n, workload,
                                  flow_general=m0["flow"] != I.FLOW_JC or m0["implicit_return"])
    r64, s64 = curve(fp)
    fd64 = fd_mm(s64, r64)
    out["fp64_failure_displacement_mm"] = fd64
    out["fp64_peak_reaction_kN"] = round(float(r64.max()) / 1e3, 3) if len(r64) else None
    shape64 = fp["info"]
    del fp["sim"]

    # FP64 runs from rounding-level perturbed starts (untimed): the spread
    # of the failure point that FP64 itself shows
    ens = []
    for seed in range(1, args.ensemble + 1):
        e = run_form(perturbed(I, prob, seed), T.FP64, args.steps, args.warmup, torch, T, flags,
                     False, shape=launch_shape(shape64))
        re_, se_ = curve(e)
        ens.append(fd_mm(se_, re_))
        del e["sim"]
    if ens:
        allfd = [fd64] + ens
        ok = [k for k in fd64 if all(d[k] for d in allfd)]
        out["fp64_ensemble"] = {
            "perturbation": "initial velocities +-1e-12 m/s, seeds 1..%d" % args.ensemble,
            "failure_displacement_mm": ens,
            "mean_mm": {k: round(float(np.mean([d[k] for d in allfd])), 4) for k in ok},
            "std_mm": {k: round(float(np.std([d[k] for d in allfd], ddof=1)), 4) for k in ok},
            "spread_rel": {k: round((max(d[k] for d in allfd) - min(d[k] for d in allfd))
                                    / np.mean([d[k] for d in allfd]), 5) for k in ok}}

    if not args.no_mixed:
        mx = run_form(prob, T.MIXED, args.steps, args.warmup, torch, T, flags, tune)
        rmx, smx = curve(mx)
        fdm = fd_mm(smx, rmx)
        ipk = int(np.argmax(r64))
        dev = float(np.max(np.abs(rmx[: ipk + 1] - r64[: ipk + 1])) / max(r64.max(), 1e-30))
        _, mtab = kernel_table(mx["kernel_times"], True, damage, prob.n, nnz)
        mixed = {
            "value": round(prob.n * args.steps / mx["seconds"], 1), "unit": "particle-steps/s",
            "ms_per_step": round(mx["seconds"] / args.steps * 1e3, 5), "dtype": "f32/f64",
            "launch": shape_of(mx["info"]), "kernels": mtab,
            "reaction_curve_max_rel_dev_to_peak_vs_fp64": round(dev, 6),
            "failure_displacement_mm": fdm,
            "failure_displacement_rel_diff_vs_fp64": {
                k: (round(abs(fdm[k] - fd64[k]) / fd64[k], 5) if fdm[k] and fd64[k] else None)
                for k in fd64}}
        if ens:
            allfd = [fd64] + ens
            ok = [k for k in fd64 if all(d[k] for d in allfd)]
            mean = {k: float(np.mean([d[k] for d in allfd])) for k in ok}
            mixed["failure_displacement_rel_diff_vs_fp64_ensemble_mean"] = {
                k: (round(abs(fdm[k] - mean[k]) / mean[k], 5) if fdm[k] else None) for k in mean}
            # the failure point is chaotic: the mixed form's is one more sample,
            # judged against the FP64 runs' median +- their range
            inside = {}
            for k in ok:
                v = [d[k] for d in allfd]
                med, rng = float(np.median(v)), max(v) - min(v)
                inside[k] = bool(fdm[k] is not None and med - rng <= fdm[k] <= med + rng)
            mixed["failure_displacement_within_fp64_median_pm_range"] = inside
        out["mixed"] = mixed
        del mx["sim"]
    assert shape64 is not None
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, "notched bar from rest, JC damage")
    return out


def final_shape(sim, prob):
    """Taylor bar after impact, over particles that have not failed: length,
    radius of the impact face (99th percentile of the bottom two layers),
    median and 99th-percentile plastic strain, and the failed count."""
    X = prob.X
    x = X + sim.get("u")
    eps = sim.get("eps_p")
    alive = sim.get("D") < 1.0
    foot = alive & (X[:, 2] < 2.0 * float(prob.dx[0]))
    rad = np.sqrt(x[foot, 0] ** 2 + x[foot, 1] ** 2)
    return {"length_mm": float(x[alive, 2].max() - x[alive, 2].min()) * 1e3,
            "foot_radius_p99_mm": float(np.percentile(rad, 99)) * 1e3,
            "eps_p_median": float(np.median(eps[alive])),
            "eps_p_p99": float(np.percentile(eps[alive], 99)),
            "failed": int(np.sum(~alive))}


def bench_single(args, torch, I, T, workload, prob, label, damage_name, result, k_cap=32,
                 setup=None):
    """One large specimen: FP64, then mixed, each with its end-state summary."""
    damage = prob.materials[0]["damage"]
    tune = not args.no_autotune
    fp = run_form(prob, T.FP64, args.steps, args.warmup, torch, T, 0, tune, k_cap=k_cap,
                  setup=setup)
    nnz = fp["info"]["nnz"]
    m0 = prob.materials[0]
    av, var_h = bool(m0["av_q1"] or m0["av_q2"]), bool(m0["h_per_spacing"])
    _, ktab = kernel_table(fp["kernel_times"], False, damage, prob.n, nnz, av, var_h)
    out = base_line(args, workload, prob.n * args.steps / fp["seconds"],
                    fp["seconds"] / args.steps * 1e3, "f64",
                    dict({"particles": prob.n, "neighbour_pairs": nnz, "damage": damage_name,
                          "precision": "fp64", "steps_total": args.warmup + args.steps,
                          "dt_s": prob.materials[0]["dt"]}, **shape_of(fp["info"])))
    if av:
        out["config"]["artificial_viscosity"] = {"q1": m0["av_q1"], "q2": m0["av_q2"]}
    out["kernels"] = ktab
    out["roofline"] = roofline_of(fp, damage, prob.n, workload,
                                  flow_general=bool(m0["flow"] != I.FLOW_JC or m0["implicit_return"]
                                                    or av),
                                  var_h=var_h, av=av)
    res64 = result(fp)
    out["fp64_result"] = res64
    del fp["sim"]
    if not args.no_mixed:
        mx = run_form(prob, T.MIXED, args.steps, args.warmup, torch, T, 0, tune, k_cap=k_cap,
                      setup=setup)
        _, mtab = kernel_table(mx["kernel_times"], True, damage, prob.n, nnz, av, var_h)
        resm = result(mx)
        out["mixed"] = {
            "value": round(prob.n * args.steps / mx["seconds"], 1), "unit": "particle-steps/s",
            "ms_per_step": round(mx["seconds"] / args.steps * 1e3, 5), "dtype": "f32/f64",
            "launch": shape_of(mx["info"]), "kernels": mtab, "result": resm,
            "rel_diff_vs_fp64": {k: (round(abs(resm[k] - res64[k]) / abs(res64[k]), 6)
                                     if res64[k] else None) for k in res64}}
        del mx["sim"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, label, max_steps=50)
    return out


def bench_taylor(args, torch, I, T):
    prob = I.taylor_bar()
    return bench_single(args, torch, I, T, "taylor_bar_1m", prob,
                        "Taylor bar on a rigid wall, CL damage", "cockcroft-latham",
                        lambda r: final_shape(r["sim"], prob))


def bench_taylor_av(args, torch, I, T):
    """The Taylor bar with the artificial particle-velocity damping on
    (Q1 = 1, Q2 = 2): the general deformation-pass variant."""
    prob = I.with_materials(I.taylor_bar(), **I.DAMPING)
    return bench_single(args, torch, I, T, "taylor_bar_1m_av", prob,
                        "Taylor bar on a rigid wall, CL damage, artificial viscosity",
                        "cockcroft-latham", lambda r: final_shape(r["sim"], prob))


def bench_graded(args, torch, I, T):
    """The graded notched bar (0.1 / 0.2 / 0.4 / 0.8 mm zones, 92 774
    particles, per-particle supports): the kernels with per-pair supports,
    staged or not as the autotuner finds faster."""
    prob = I.graded_notched_bar()

    def result(r):
        bd, sd = r["bd"], r["sd"]
        eps = r["sim"].get("eps_p")
        return {"reaction_kN": float(-bd[-1, 1, 2]) / 1e3,
                "grip_separation_mm": float(bd[-1, 1, 5] - bd[-1, 0, 5]) * 1e3,
                "eps_p_max": float(eps.max()), "max_D": float(sd[-1, 0, 3])}
    return bench_single(args, torch, I, T, "graded_bar_93k", prob,
                        "graded notched bar, JC damage", "johnson-cook", result, k_cap=64)


def bench_collision(args, torch, I, T):
    """Two bars (R 2.5 mm, 10 mm long, dx 0.1 mm, 395 200 particles) meeting
    head on at 100 m/s each, CL damage, penalty contact with candidate lists
    rebuilt every 10 steps (skin 0.2 dx)."""
    prob = I.bar_collision_395k()
    dx = float(prob.dx[0])
    n0 = int(prob.spec_offsets[1])
    m = prob.materials[0]["rho0"] * prob.V0

    def result(r):
        v = r["sim"].get("v")
        ke = 0.5 * float(np.sum(m[:, None] * v * v))
        ke0 = 0.5 * float(np.sum(m[:, None] * prob.v_init ** 2))
        return {"v_lower_bar": float(v[:n0, 2].mean()), "v_upper_bar": float(v[n0:, 2].mean()),
                "kinetic_energy_ratio": ke / ke0,
                "eps_p_max": float(r["sim"].get("eps_p").max()),
                "failed": int((r["sim"].get("D") >= 1.0).sum())}
    out = bench_single(args, torch, I, T, "bar_collision_395k", prob,
                       "two bars meeting head on, CL damage, penalty contact", "cockcroft-latham",
                       result, setup=lambda sim: sim.set_contact(10, 0.2 * dx))
    out["config"]["contact"] = {"rebuild_every": 10, "skin_m": 0.2 * dx}
    # the same FP64 run replayed from graphs (twenty steps a replay, the
    # lists rebuilt at the first and the eleventh)
    side = torch.cuda.Stream()
    gr = run_form(prob, T.FP64, args.steps, args.warmup, torch, T, T.USE_GRAPHS,
                  not args.no_autotune, stream=side, diag=False,
                  setup=lambda sim: sim.set_contact(10, 0.2 * dx))
    out["fp64_graphs"] = {"value": round(prob.n * args.steps / gr["seconds"], 1),
                          "ms_per_step": round(gr["seconds"] / args.steps * 1e3, 5)}
    del gr["sim"]
    return out


PLASTIC_TARGET = 0.02     # share of particles yielding in a step before the plate is timed
PRELOAD_CAP = 60000       # most steps spent reaching it
PRELOAD_CHUNK = 1000


def plastic_share(sim, torch):
    """Share of particles whose plastic strain grew in the last step."""
    r = sim.get_tensor("eps_p_rate")
    torch.cuda.synchronize()
    return float((r > 0).sum().item()) / sim.n


def plate_state(sim, torch):
    f = sim.get_tensor("f_void")
    torch.cuda.synchronize()
    return {"plastic_share": plastic_share(sim, torch), "max_void_fraction": float(f.max().item())}


def bench_plate(args, torch, I, T):
    """The GTN holed plate (4.08 M particles) in its yielding regime: the
    FP64 context is driven along the grip ramp (untimed) until at least 2 %
    of the particles yield in a step, so that Algorithm 2's Newton loops run
    in the timed steps; the mixed context takes over that same state and is
    timed over the same steps."""
    prob = I.holed_plate()
    workload = "gtn_plate_4m"
    damage = I.DMG_GTN
    tune = not args.no_autotune
    fp_sim = T.Sim(prob, precision=T.FP64)
    pre = 0
    target = args.preload if args.preload is not None else -1
    t0 = time.perf_counter()
    while (target < 0 and pre < PRELOAD_CAP) or (target >= 0 and pre < target):
        k = PRELOAD_CHUNK if target < 0 else min(PRELOAD_CHUNK, target - pre)
        fp_sim.step(k)
        pre += k
        share = plastic_share(fp_sim, torch)
        if pre % (4 * PRELOAD_CHUNK) == 0:
            log(f"preload: {pre} steps, {time.perf_counter() - t0:.1f} s, plastic share {share:.4f}")
        if target < 0 and share >= PLASTIC_TARGET:
            break
    torch.cuda.synchronize()
    start = plate_state(fp_sim, torch)
    log(f"preload: {pre} steps in {time.perf_counter() - t0:.1f} s, {start}")
    mx_sim = None
    if not args.no_mixed:
        mx_sim = T.Sim(prob, precision=T.MIXED)
        mx_sim.copy_state_from(fp_sim)

    def result(r):
        bd, sd = r["bd"], r["sd"]
        st = plate_state(r["sim"], torch)
        return {"reaction_kN": float(-bd[-1, 1, 0]) / 1e3,
                "grip_separation_mm": float(bd[-1, 1, 3] - bd[-1, 0, 3]) * 1e3,
                "max_void_fraction": st["max_void_fraction"], "max_D": float(sd[-1, 0, 3]),
                "plastic_share_last_step": st["plastic_share"]}

    fp = run_form(prob, T.FP64, args.steps, args.warmup, torch, T, 0, tune, sim=fp_sim)
    nnz = fp["info"]["nnz"]
    _, ktab = kernel_table(fp["kernel_times"], False, damage, prob.n, nnz)
    out = base_line(args, workload, prob.n * args.steps / fp["seconds"],
                    fp["seconds"] / args.steps * 1e3, "f64",
                    dict({"particles": prob.n, "neighbour_pairs": nnz, "damage": "gtn",
                          "precision": "fp64", "preload_steps": pre,
                          "steps_total": pre + args.warmup + args.steps,
                          "dt_s": prob.materials[0]["dt"],
                          "timed_from": {"plastic_share": round(start["plastic_share"], 5),
                                         "max_void_fraction": round(start["max_void_fraction"],
                                                                    6)}},
                         **shape_of(fp["info"])))
    step_bytes = sum(algorithmic_bytes(k, False, damage, prob.n, nnz) for k in ktab)
    out["step_algorithmic_GBs"] = round(step_bytes * args.steps / fp["seconds"] / 1e9, 1)
    out["kernels"] = ktab
    out["roofline"] = roofline_of(fp, damage, prob.n, workload)
    res64 = result(fp)
    out["fp64_result"] = res64
    out["fp64_device_flags"] = fp_sim.info()["flags"]
    del fp["sim"], fp_sim
    if mx_sim is not None:
        mx = run_form(prob, T.MIXED, args.steps, args.warmup, torch, T, 0, tune, sim=mx_sim)
        _, mtab = kernel_table(mx["kernel_times"], True, damage, prob.n, nnz)
        resm = result(mx)
        out["mixed"] = {
            "value": round(prob.n * args.steps / mx["seconds"], 1), "unit": "particle-steps/s",
            "ms_per_step": round(mx["seconds"] / args.steps * 1e3, 5), "dtype": "f32/f64",
            "from": "the FP64 state after the preload (float fields rounded)",
            "device_flags": mx_sim.info()["flags"],
            "launch": shape_of(mx["info"]), "kernels": mtab, "result": resm,
            "rel_diff_vs_fp64": {k: (round(abs(resm[k] - res64[k]) / abs(res64[k]), 6)
                                     if res64[k] else None) for k in res64}}
        del mx["sim"], mx_sim
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, "GTN holed plate from rest (elastic steps)",
                                           max_steps=60)
    return out


def bench_batch(args, torch, I, T):
    """256 specimens: mixed form, one context, graph replays (two launches
    per step for the whole batch), against 256 separate FP64 contexts stepped
    one after the other (two launches per specimen per step); the batched
    FP64 form is reported too."""
    prob = I.bar_batch()
    workload = "batch_256_bars"
    damage = I.DMG_JC
    side = torch.cuda.Stream()
    mx = run_form(prob, T.MIXED, args.steps, args.warmup, torch, T, T.USE_GRAPHS,
                  not args.no_autotune, stream=side, diag=False)
    nnz = mx["info"]["nnz"]
    out = base_line(args, workload, prob.n * args.steps / mx["seconds"],
                    mx["seconds"] / args.steps * 1e3, "f32/f64",
                    dict({"particles": prob.n, "specimens": prob.n_spec, "neighbour_pairs": nnz,
                          "damage": "johnson-cook", "precision": "mixed", "graphs": True},
                         **shape_of(mx["info"])))
    del mx["sim"]
    fb = run_form(prob, T.FP64, args.steps, args.warmup, torch, T, 0, not args.no_autotune,
                  diag=False)
    _, ktab = kernel_table(fb["kernel_times"], False, damage, prob.n, nnz)
    out["fp64_batched"] = {"value": round(prob.n * args.steps / fb["seconds"], 1),
                           "ms_per_step": round(fb["seconds"] / args.steps * 1e3, 5),
                           "kernels": ktab, "launch": shape_of(fb["info"])}
    out["roofline"] = roofline_of(fb, damage, prob.n, workload)
    out["roofline"]["form"] = "fp64 batched"
    del fb["sim"]
    # 256 separate FP64 contexts, default launch shapes, eager launches
    log("256 separate FP64 contexts")
    sims = [T.Sim(I.subset(prob, [s]), precision=T.FP64) for s in range(prob.n_spec)]
    for s in sims:
        s.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(args.steps)
    torch.cuda.synchronize()
    sep = time.perf_counter() - t0
    out["fp64_separate_256"] = {"value": round(prob.n * args.steps / sep, 1),
                                "ms_per_step": round(sep / args.steps * 1e3, 5)}
    out["speedup_batched_mixed_vs_separate_fp64"] = round(sep / mx["seconds"], 3)
    del sims
    out["to_failure"] = batch_to_failure(prob, torch, T, not args.no_autotune,
                                         mx["seconds"] / args.steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, "256 notched bars, JC damage", max_steps=20)
    return out


# run control of the batch: each bar stops once its load (the reaction of its
# pulled grip) has dropped below half its peak, or at the cap.  The peak must
# first reach 20 kN (the bars peak at 50-90 kN): the coarsest bars' grip
# reactions ring at a few kN while the ramp starts, dips that are no failure.
BATCH_STOP = {"axis": 2, "sign": -1.0, "drop": 0.5, "min_peak": 20000.0}
BATCH_CAP = 60000


def batch_to_failure(prob, torch, T, autotune, lockstep_s_per_step):
    """Mixed form, graphs, from rest: every specimen runs until it fails or
    reaches the cap while the others go on; a stopped specimen drops out of
    the staged passes' tile list.  Throughput counts the particle-steps
    actually taken.  The lockstep figure is what stepping the whole batch
    until the last specimen stops would have cost at the batch's measured
    time per step."""
    side = torch.cuda.Stream()
    sim = T.Sim(prob, precision=T.MIXED, flags=T.USE_GRAPHS, stream=side)
    if autotune:
        sim.autotune()
    sim.set_run_control([dict(BATCH_STOP, group=2 * q + 1, step_cap=BATCH_CAP)
                         for q in range(prob.n_spec)])
    counts = np.diff(prob.spec_offsets)
    log(f"batch to failure: {prob.n_spec} specimens, cap {BATCH_CAP} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ran = sim.run(BATCH_CAP, check_every=500)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = sim.run_status()
    ps = int(np.sum(counts * st["steps"]))
    log(f"  {ran} steps in {secs:.3f} s, failed {int(np.sum(st['why'] == T.FAILED))}")
    lock = lockstep_s_per_step * int(st["steps"].max())
    del sim
    return {"value": round(ps / secs, 1), "unit": "particle-steps/s", "seconds": round(secs, 3),
            "particle_steps": ps, "steps_launched": ran,
            "failed": int(np.sum(st["why"] == T.FAILED)),
            "stopped_at_cap": int(np.sum(st["why"] == T.STOPPED_AT_CAP)),
            "steps_min_median_max": [int(st["steps"].min()), int(np.median(st["steps"])),
                                     int(st["steps"].max())],
            "rule": dict(BATCH_STOP, cap=BATCH_CAP),
            "lockstep_estimate_s": round(lock, 3),
            "speedup_vs_lockstep": round(lock / secs, 3)}


def bench_notched_bar_voce(args, torch, I, T):
    """The headline bar with Voce hardening (fitted near the Johnson-Cook
    curve: A = 792 MPa, B = 510 MPa, beta = 5) and the implicit return: the
    general deformation-pass variant."""
    return bench_notched_bar(args, torch, I, T, "notched_bar_200k_voce_implicit",
                             **I.VOCE_IMPLICIT)


WORKLOADS = {"notched_bar_200k": (bench_notched_bar, 42000, 1000),
             "notched_bar_200k_voce_implicit": (bench_notched_bar_voce, 42000, 1000),
             "taylor_bar_1m": (bench_taylor, 4900, 100),
             "taylor_bar_1m_av": (bench_taylor_av, 4900, 100),
             "graded_bar_93k": (bench_graded, 4900, 100),
             "bar_collision_395k": (bench_collision, 1900, 100),
             "gtn_plate_4m": (bench_plate, 200, 20),
             "batch_256_bars": (bench_batch, 400, 50)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="gtn_plate_4m", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision form")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--ensemble", type=int, default=5,
                    help="extra untimed FP64 runs from perturbed starts (notched bar)")
    ap.add_argument("--unstaged", action="store_true",
                    help="force pass gathers from global memory instead of LDS tiles")
    ap.add_argument("--preload", type=int, default=None,
                    help="GTN plate: untimed steps before the timed region (default: until "
                         "2%% of the particles yield)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    fn, steps, warmup = WORKLOADS[args.workload]
    args.steps = steps if args.steps is None else args.steps
    args.warmup = warmup if args.warmup is None else args.warmup

    import torch
    from paper_1901_07374_amd import inputs as I
    from paper_1901_07374_amd import tlsph as T

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    out = fn(args, torch, I, T)

    if args.copy_probe_mib > 0:
        # counter calibration: a plain device copy of known size, and a gather
        # of 64-byte rows in random order (each row read once)
        nb = args.copy_probe_mib * 1024 * 1024
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nb
        del a, b
        rows = nb // 64
        tab = torch.ones((rows, 8), dtype=torch.float64, device="cuda")
        idx = torch.randperm(rows, device="cuda")
        torch.cuda.synchronize()
        g = tab.index_select(0, idx)
        torch.cuda.synchronize()
        out["gather_probe"] = {"rows": rows, "row_bytes": 64, "index_bytes": 8,
                               "read_bytes": rows * 72, "write_bytes": rows * 64}
        del tab, idx, g
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
