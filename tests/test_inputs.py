"""Input recipe checks (host only)."""
import json
import math
import os

import numpy as np
import pytest

from paper_1901_07374_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "weldox_tables.json")


def test_sound_speed_reading_matches_table1():
    # Table 1 prints c0 = 5166 m/s for rho0 = 7750, E = 211 GPa, nu = 0.33.
    # The caption's formula sqrt(E / (2 (1 - 2 nu) rho0)) would give 6328 m/s;
    # the printed value is reproduced by sqrt(E / (3 (1 - 2 nu)) / rho0) = sqrt(K / rho0).
    t = json.load(open(GOLDEN))["table1_material"]
    c0 = I.bulk_sound_speed(t["E_GPa"] * 1e9, t["nu"], t["rho0_kg_m3"])
    assert abs(c0 - t["c0_m_s"]) < 1.0
    caption = math.sqrt(t["E_GPa"] * 1e9 / (2 * (1 - 2 * t["nu"]) * t["rho0_kg_m3"]))
    assert abs(caption - t["c0_m_s"]) > 1000.0


def test_workload_sizes():
    assert I.cube().n == 1000
    assert I.notched_bar().n == 200216
    counts = I.batch_counts()
    assert counts.sum() == 8514409 and counts.min() == 2397 and counts.max() == 59926


def test_seeded_and_deterministic():
    a, b = I.notched_bar(dx=1e-3), I.notched_bar(dx=1e-3)
    assert np.array_equal(a.X, b.X)
    assert a.materials[0]["dt"] == pytest.approx(0.3 * 1e-3 / a.materials[0]["c0"])


def test_batch_subset_roundtrip():
    p = I.bar_batch(n_spec=3, lo=2000, hi=3000)
    q = I.subset(p, [1])
    a, b = p.spec_offsets[1], p.spec_offsets[2]
    assert np.array_equal(q.X, p.X[a:b])
    assert set(np.unique(q.bc_group)) == {-1, 0, 1}
