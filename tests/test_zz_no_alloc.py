"""The allocation-free diagnostics entry point, tlsph_get_diagnostics_static,
against tlsph_get_diagnostics through the C ABI: same kernels and order, so
the outputs must be identical bit for bit, on two calls in a row with the
second on a smaller problem (the static scratch keeps the first call's
contents), and a problem whose partials exceed the static array is refused
while the workspace-backed call still serves it."""
import ctypes as C

import numpy as np
import pytest

from paper_1901_07374_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_07374_amd import tlsph
    return tlsph


def both(tl, g):
    import torch
    L = tl.lib()
    nb = max(g.n_bc, 1)
    out = []
    for fn in (L.tlsph_get_diagnostics, L.tlsph_get_diagnostics_static):
        sd = torch.full((g.n_spec, 8), -1.0, dtype=torch.float64, device=g.device)
        bd = torch.full((nb, 8), -1.0, dtype=torch.float64, device=g.device)
        st = fn(g.ctx, sd.data_ptr(), bd.data_ptr() if g.n_bc else None, g._sp())
        assert st == 0, L.tlsph_last_error(g.ctx)
        g.stream.synchronize()
        out.append((sd.cpu().numpy(), bd.cpu().numpy()))
    return out


def many_cubes(n_spec):
    """n_spec specimens of 27 particles: one chunk partial each."""
    base = I.cube(nside=3)
    n0 = base.n
    X = np.concatenate([base.X + np.array([0.01 * (s % 100), 0.01 * (s // 100), 0.0])
                        for s in range(n_spec)])
    offs = np.arange(n_spec + 1, dtype=np.int64) * n0
    return I.Problem("cubes", X, np.tile(base.V0, n_spec), offs, [base.materials[0]] * n_spec,
                     np.full(n_spec * n0, -1, np.int32), [], np.zeros((n_spec * n0, 3)))


def test_static_diagnostics_equal_workspace_diagnostics(tl):
    big = I.notched_bar(dx=0.5e-3)                 # about 25 000 particles, 13 + 2 partials
    small = I.cube(nside=6)                        # 216 particles
    for p, steps in ((big, 2), (small, 3)):
        g = tl.Sim(p, flags=tl.STORE_FORCE)
        g.set_state(I.random_state(p, seed=5))
        g.step(steps)
        (sd0, bd0), (sd1, bd1) = both(tl, g)
        print(p.name, p.n, sd0[:, :4].ravel()[:4], flush=True)
        assert np.array_equal(sd0, sd1) and np.array_equal(bd0, bd1)
        assert sd0[:, 2].sum() > 0                 # some failed particles counted
        del g


def test_static_diagnostics_refuse_too_many_partials(tl):
    p = many_cubes(16385)
    g = tl.Sim(p)
    import torch
    L = tl.lib()
    sd = torch.zeros((p.n_spec, 8), dtype=torch.float64, device=g.device)
    assert L.tlsph_get_diagnostics_static(g.ctx, sd.data_ptr(), None, g._sp()) == 6
    assert b"static" in L.tlsph_last_error(g.ctx)
    assert L.tlsph_get_diagnostics(g.ctx, sd.data_ptr(), None, g._sp()) == 0
    g.stream.synchronize()
    assert np.all(sd.cpu().numpy()[:, 4] == 0.0)
