"""bench.py's host-side helpers: the kernel names it looks up in the
committed rocprofv3 summaries are the names the profiler reports, and a
request for more than one GPU is refused.  Host only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

STAGED = {"staged": True, "lanes_per_particle": 2, "block_deformation": 0}


def test_headline_symbols_are_in_the_profiles():
    force = bench.kernel_symbol("force_pass", STAGED, False, 2)
    deform = bench.kernel_symbol("deformation_pass", STAGED, False, 2)
    assert force == "k_pass_b_staged<double, 2, false>"
    assert deform == "k_pass_a_staged<double, 2, false, false>"
    for name in ("pmc_notched_bar_200k.txt", "trace_notched_bar_200k.txt"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert force in text and deform in text, name


def test_plate_symbols_are_in_the_profiles():
    # the FP64 GTN plate's autotuned kernels (staged force pass, two lanes;
    # staged deformation pass with the GTN model)
    force = bench.kernel_symbol("force_pass", STAGED, False, 3)
    deform = bench.kernel_symbol("deformation_pass", STAGED, False, 3)
    for name in ("pmc_gtn_plate_4m.txt", "trace_gtn_plate_4m.txt", "sq_gtn_plate_4m.txt"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert force in text and deform in text, name


def test_deformation_pass_over_its_own_tiles():
    own = dict(STAGED, block_deformation=-128, tile=96, block_force=192)
    assert bench.kernel_symbol("deformation_pass", own, False, 3) == \
        "k_pass_a_staged<double, 3, false, false>"
    sh = bench.shape_of(own)
    assert sh["deformation_pass_block"] == 0 and sh["deformation_pass_tile"] == 128
    assert bench.launch_shape(own) == (1, 2, 256, -128, 96)


def test_graded_and_general_symbols():
    unstaged = {"staged": False, "lanes_per_particle": 4, "block_deformation": 128}
    assert bench.kernel_symbol("force_pass", unstaged, True, 2, var_h=True) == \
        "k_pass_b<float, 4, true>"
    assert bench.kernel_symbol("deformation_pass", unstaged, True, 2, var_h=True) == \
        "k_pass_a<float, -1, true, true>"
    assert bench.kernel_symbol("deformation_pass", STAGED, False, 1, flow_general=True) == \
        "k_pass_a_staged<double, 1, true, false>"


def test_algorithmic_bytes_of_the_headline_force_pass():
    # 308 bytes per particle and 4 per neighbour pair (200 216 particles,
    # 3 476 976 pairs)
    assert bench.algorithmic_bytes("force_pass", False, 2, 200216, 3476976) == \
        308 * 200216 + 4 * 3476976
    assert bench.algorithmic_bytes("force_pass", False, 2, 10, 0, av=True, var_h=True) == \
        (308 + 24 + 8) * 10


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in (r.stdout + r.stderr)
