"""Parity at the benchmark workloads' full sizes, in the launch configuration
the benchmark times (autotuned shapes): the Taylor bar on the rigid wall
(996 314 particles, Cockcroft-Latham), with and without the artificial
damping, the GTN holed plate (4.08 M particles), the batch of 256 notched
bars (8.55 M particles, uneven counts, scattered parameters), the notched bar
with Voce hardening and the implicit return (200 216), the graded notched bar
(92 774, per-particle supports) and the two colliding bars with penalty
contact (395 200).  Neighbour lists are compared bit for bit; one step from an
injected state is compared field by field with the FP64 oracle over every
particle (the oracle finishes these sizes in seconds)."""
import numpy as np
import pytest

from paper_1901_07374_amd import inputs as I
from parity_util import compare
from test_gpu_parity import consistent_gtn, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_07374_amd import tlsph
    return tlsph


def injected(orc, p, seed, f_hi=0.24):
    st = I.random_state(p, seed=seed)
    st["t"] = np.full(p.n_spec, 2.1e-6)
    if any(m["av_q1"] or m["av_q2"] for m in p.materials):
        st["fvisc"] = np.random.default_rng(seed + 1).uniform(-1e-3, 1e-3, (p.n, 3))
    if p.materials[0]["damage"] == I.DMG_GTN:
        consistent_gtn(orc, p, st, f_hi=f_hi, seed=seed)
    return st


def run_case(tl, orc, p, precisions, seed, k_cap=32, setup=None):
    o = orc.Sim(p)
    st = injected(orc, p, seed)
    o.set_state(st)
    o.step(1)
    first = True
    for prec, tol in precisions:
        g = tl.Sim(p, precision=prec, flags=tl.STORE_FORCE, k_cap=k_cap)
        if setup:
            setup(g)
        if first:
            rp, col = g.neighbors()
            assert np.array_equal(rp, o.row_ptr)
            assert np.array_equal(col, o.col[: o.row_ptr[-1]])
            first = False
        g.set_state(st)
        g.autotune()
        g.step(1)
        errs = compare(g, o)
        say(p.name, p.n, prec, g.info(), {k: f"{v:.1e}" for k, v in errs.items()})
        bad = {k: v for k, v in errs.items() if not v <= tol}
        assert not bad, bad
        # every Newton loop of the step ended by its convergence test
        assert g.info()["flags"] & 2 == 0
        del g


def test_taylor_bar_full_size(tl, orc):
    p = I.taylor_bar()
    assert 990_000 < p.n < 1_000_000
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 41)


def test_gtn_plate_full_size(tl, orc):
    p = I.holed_plate()
    assert p.n > 4_000_000
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 42)


def test_batch_of_256_full_size(tl, orc):
    p = I.bar_batch()
    assert p.n_spec == 256
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 43)


def test_taylor_bar_damping_full_size(tl, orc):
    p = I.with_materials(I.taylor_bar(), **I.DAMPING)
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 44)


def test_voce_implicit_bar_full_size(tl, orc):
    p = I.notched_bar(**I.VOCE_IMPLICIT)
    assert p.n == 200216
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 45)


def test_graded_bar_full_size(tl, orc):
    p = I.graded_notched_bar()
    assert 90_000 < p.n < 95_000
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 46, k_cap=64)


def test_bar_collision_full_size(tl, orc):
    p = I.bar_collision_395k()
    assert p.n == 395200
    dx = float(p.dx[0])
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 47,
             setup=lambda g: g.set_contact(10, 0.2 * dx))
