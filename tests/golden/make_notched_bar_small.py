"""Write notched_bar_small_oracle.json: the FP64 oracle's run of the small
notched bar (0.5 mm lattice, Johnson-Cook plasticity and damage, grips at
+-10 m/s with a 1 ms ramp) from rest to past failure; with --full, write
notched_bar_oracle.json, the same run of the full-size bar (0.25 mm lattice,
200 216 particles).

Every 20 steps it records the reaction on the top grip (minus the sum of the
axial nodal forces of its particles) and the grip separation (difference of
the two grips' mean axial displacements).  Only the oracle and the seeded
input generator are used.

Usage: python tests/golden/make_notched_bar_small.py [--full]
(about a minute on 8 cores; with --full about an hour on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1901_07374_amd import inputs as I  # noqa: E402

EVERY = 20
MAX_STEPS = 60000


def main():
    full = "--full" in sys.argv
    dx = 0.25e-3 if full else 0.5e-3
    name = "notched_bar_oracle.json" if full else "notched_bar_small_oracle.json"
    p = I.notched_bar(dx=dx)
    o = oracle.Sim(p)
    top, bot = p.bc_group == 1, p.bc_group == 0
    steps, reac, sep = [], [], []
    peak, done_at = 0.0, None
    t0 = time.time()
    k = 0
    while k < MAX_STEPS:
        o.step(EVERY)
        k += EVERY
        f = o.get("force")
        u = o.get("u")
        r = -float(f[top, 2].sum())
        s = float(u[top, 2].mean() - u[bot, 2].mean())
        steps.append(k)
        reac.append(r)
        sep.append(s)
        peak = max(peak, r)
        if done_at is None and peak > 0 and r < 0.05 * peak and s > 1e-3:
            done_at = k
        if done_at is not None and k >= done_at + 1000:
            break
        if k % 2000 == 0:
            print(f"step {k} sep {s * 1e3:.4f} mm reaction {r / 1e3:.3f} kN "
                  f"({time.time() - t0:.0f} s)", flush=True)
    out = {
        "what": f"FP64 oracle run of the {'full-size' if full else 'small'} notched bar to "
                "past failure",
        "workload": f"notched_bar(dx={dx:g}): R 5 mm, L 40 mm, 90-degree V-notch 1 mm deep, "
                    "jitter 3 %, JC plasticity + JC damage, grips +-10 m/s (1 - exp(-t/1 ms))",
        "written_by": "tests/golden/make_notched_bar_small.py" + (" --full" if full else "") +
                      " (oracle only)",
        "particles": p.n, "dt_s": p.materials[0]["dt"], "diag_every": EVERY,
        "step": steps, "reaction_N": reac, "separation_m": sep,
    }
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(out, fh)
    print("wrote", len(steps), "samples, peak", peak, "N", flush=True)


if __name__ == "__main__":
    main()
