"""Parity at the benchmark workloads' full sizes, in the launch configuration
the benchmark times (autotuned shapes): the Taylor bar on the rigid wall
(996 314 particles, Cockcroft-Latham), the GTN holed plate (4.08 M
particles) and the batch of 256 notched bars (8.55 M particles, uneven counts,
scattered parameters).  Neighbour lists are compared bit for bit; one step
from an injected state is compared field by field with the FP64 oracle over
every particle (the oracle finishes these sizes in seconds)."""
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
    if p.materials[0]["damage"] == I.DMG_GTN:
        consistent_gtn(orc, p, st, f_hi=f_hi, seed=seed)
    return st


def run_case(tl, orc, p, precisions, seed):
    o = orc.Sim(p)
    st = injected(orc, p, seed)
    o.set_state(st)
    o.step(1)
    first = True
    for prec, tol in precisions:
        g = tl.Sim(p, precision=prec, flags=tl.STORE_FORCE)
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
        del g


def test_taylor_bar_full_size(tl, orc):
    p = I.taylor_bar()
    assert 990_000 < p.n < 1_000_000
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 41)


def test_gtn_plate_full_size(tl, orc):
    p = I.holed_plate()
    assert p.n > 4_000_000
    run_case(tl, orc, p, [(tl.FP64, 1e-12)], 42)


def test_batch_of_256_full_size(tl, orc):
    p = I.bar_batch()
    assert p.n_spec == 256
    run_case(tl, orc, p, [(tl.FP64, 1e-12), (tl.MIXED, 1e-5)], 43)
