"""Benchmark: damaged TLSPH steps of the notched round bar on one MI355X.

Workload: the notched round bar in tension (radius 5 mm, length 40 mm,
90-degree V-notch 1 mm deep, 0.25 mm lattice, 200 216 particles, seeded 3 %
jitter), Johnson-Cook plasticity and Johnson-Cook damage, grips driven at
+-10 m/s (1 - exp(-t / 1 ms)).  A step is one pass of the whole path: nodal
forces with hourglass control, leapfrog update, damaged dF/dt, EOS, radial
return, damage, PK1.  The default run goes from rest to past failure.

The headline value is the FP64 form; the mixed FP32/FP64 form runs the same
steps and is reported beside it with its deviation from FP64 (reaction-
force curve and failure displacement).  Inputs and state are resident in HBM
before the timed region starts.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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


def algorithmic_bytes(kernel: str, mixed: bool, damage: int, n: int, nnz: int) -> int:
    if kernel == "force_pass":
        per = 32 + 24 + (76 if mixed else 152) + 8 + 24 + 12 + 32 + 24
    else:
        per = (32 + 24 + (36 if mixed else 72) * 2 + (24 if mixed else 48) + 32 + 8
               + (76 if mixed else 152) + (24 if mixed else 48) + 32)
        per += ACC_BYTES[damage]
    return per * n + 4 * nnz


def kernel_symbol(kernel: str, info: dict, mixed: bool) -> str:
    r = "float" if mixed else "double"
    if kernel == "force_pass":
        name = "k_pass_b_staged" if info["staged"] else "k_pass_b"
        return f"{name}<{r}, {info['lanes_per_particle']}>"
    return f"k_pass_a<{r}>"


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


def failure_displacement(sep, reaction):
    """Grip separation where the reaction first drops below 10 % of its running
    maximum after the peak, interpolated linearly between samples (None if it
    never does)."""
    run_max = 0.0
    peak_seen = False
    prev = None
    for s, r in zip(sep, reaction):
        if r > run_max:
            run_max = r
        elif run_max > 0 and r < 0.98 * run_max:
            peak_seen = True
        if peak_seen and r < 0.1 * run_max:
            if prev is None or prev[1] <= r:
                return float(s)
            s0, r0 = prev
            lvl = 0.1 * run_max
            return float(s0 + (s - s0) * (r0 - lvl) / (r0 - r))
        prev = (s, r)
    return None


def run_form(prob, precision, steps, warmup, torch, T, flags=0, autotune=True):
    sim = T.Sim(prob, precision=precision, flags=flags)
    n_rec = (warmup + steps) // DIAG_EVERY + 1
    sd = torch.zeros((n_rec, prob.n_spec, 8), dtype=torch.float64, device="cuda")
    bd = torch.zeros((n_rec, len(prob.bc_groups), 8), dtype=torch.float64, device="cuda")
    L = T.lib()
    rec = 0

    def advance(k):
        nonlocal rec
        done = 0
        while done < k:
            chunk = min(DIAG_EVERY, k - done)
            sim.step(chunk)
            done += chunk
            if chunk == DIAG_EVERY and rec < n_rec:
                st = L.tlsph_get_diagnostics(sim.ctx, sd[rec].data_ptr(), bd[rec].data_ptr(),
                                             sim._sp())
                if st:
                    raise RuntimeError("diagnostics failed")
                rec += 1

    advance(warmup)
    if autotune:
        sim.autotune()     # picks launch shapes on the current state; results unchanged
    torch.cuda.synchronize()
    sim.enable_kernel_timing(TIMING_STRIDE)
    t0 = time.perf_counter()
    advance(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = sim.kernel_times()
    sim.enable_kernel_timing(0)
    bdh = bd[:rec].cpu().numpy()
    sdh = sd[:rec].cpu().numpy()
    # reaction on the top grip (group 1) and grip separation
    reaction = -bdh[:, 1, 2]
    sep = bdh[:, 1, 5] - bdh[:, 0, 5]
    return dict(seconds=t1 - t0, kernel_times=kt, info=sim.info(), reaction=reaction, sep=sep,
                failed=sdh[:, 0, 2], sim=sim)


def cpu_baseline(prob, target_seconds=15.0):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload (the full notched bar, a few steps from rest)."""
    import oracle
    o = oracle.Sim(prob)
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    k = int(max(2, min(400, target_seconds / max(one, 1e-6))))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    return {"value": prob.n * k / dt, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"notched bar {prob.n} particles, JC damage, FP64 oracle, {k} steps from "
                      f"rest after 1 untimed step, {threads} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=42000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision form")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--unstaged", action="store_true",
                    help="force pass gathers from global memory instead of LDS tiles")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1901_07374_amd import inputs as I
    from paper_1901_07374_amd import tlsph as T

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    prob = I.notched_bar()
    damage = prob.materials[0]["damage"]
    workload = "notched_bar_200k"

    flags = T.NO_STAGING if args.unstaged else 0
    fp = run_form(prob, T.FP64, args.steps, args.warmup, torch, T, flags, not args.no_autotune)
    nnz = fp["info"]["nnz"]
    value = prob.n * args.steps / fp["seconds"]
    ms_step = fp["seconds"] / args.steps * 1e3

    # roofline of the dominant kernel
    kts = {k: v[0] / max(v[1], 1) for k, v in fp["kernel_times"].items()}
    dom = max(kts, key=kts.get)
    bytes_launch = algorithmic_bytes(dom, False, damage, prob.n, nnz)
    achieved = bytes_launch / (kts[dom] * 1e-3) / 1e9
    symbol = kernel_symbol(dom, fp["info"], False)
    traffic = counter_traffic(symbol, workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": dom, "symbol": symbol,
                "avg_launch_us": round(kts[dom] * 1e3, 2),
                "algorithmic_bytes_per_launch": bytes_launch}
    step_bytes = sum(algorithmic_bytes(k, False, damage, prob.n, nnz) for k in kts)
    kernels = {k: {"avg_launch_us": round(v * 1e3, 2),
                   "algorithmic_GBs": round(algorithmic_bytes(k, False, damage, prob.n, nnz)
                                            / (v * 1e-3) / 1e9, 1)} for k, v in kts.items()}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "particles": prob.n, "neighbour_pairs": nnz,
                   "damage": "johnson-cook", "precision": "fp64",
                   "force_pass_variant": ("LDS-staged tiles" if fp["info"]["staged"] else
                                          "global gathers"),
                   "launch_shape": {"force_pass": fp["info"]["block_force"],
                                    "force_lanes_per_particle": fp["info"]["lanes_per_particle"],
                                    "deformation_pass": fp["info"]["block_deformation"]},
                   "steps_from_rest": args.warmup + args.steps,
                   "dt_s": prob.materials[0]["dt"]},
        "step_algorithmic_GBs": round(step_bytes * args.steps / fp["seconds"] / 1e9, 1),
        "kernels": kernels,
        "roofline": roofline,
    }
    fd64 = failure_displacement(fp["sep"], fp["reaction"])
    out["fp64_failure_displacement_mm"] = None if fd64 is None else round(fd64 * 1e3, 4)
    out["fp64_peak_reaction_kN"] = round(float(fp["reaction"].max()) / 1e3, 3)
    del fp["sim"]

    if not args.no_mixed:
        mx = run_form(prob, T.MIXED, args.steps, args.warmup, torch, T, flags, not args.no_autotune)
        fdm = failure_displacement(mx["sep"], mx["reaction"])
        r64, rmx = fp["reaction"], mx["reaction"]
        ipk = int(np.argmax(r64))
        dev = float(np.max(np.abs(rmx[: ipk + 1] - r64[: ipk + 1])) / max(r64.max(), 1e-30))
        mkts = {k: v[0] / max(v[1], 1) for k, v in mx["kernel_times"].items()}
        out["mixed"] = {
            "value": round(prob.n * args.steps / mx["seconds"], 1), "unit": "particle-steps/s",
            "ms_per_step": round(mx["seconds"] / args.steps * 1e3, 5), "dtype": "f32/f64",
            "kernels": {k: {"avg_launch_us": round(v * 1e3, 2),
                            "algorithmic_GBs": round(algorithmic_bytes(k, True, damage, prob.n, nnz)
                                                     / (v * 1e-3) / 1e9, 1)}
                        for k, v in mkts.items()},
            "reaction_curve_max_rel_dev_to_peak_vs_fp64": round(dev, 6),
            "failure_displacement_mm": None if fdm is None else round(fdm * 1e3, 4),
            "failure_displacement_rel_diff_vs_fp64": (None if (fdm is None or fd64 is None)
                                                      else round(abs(fdm - fd64) / fd64, 5)),
        }
        del mx["sim"]

    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib * 1024 * 1024
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nb

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
