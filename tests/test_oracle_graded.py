"""Oracle pins for graded particle spacing (the paper's finest specimens
refine the spacing towards the notch; reading: per-particle support
h_i = k V_i^(1/3) and the pair support h_ij = (h_i + h_j) / 2 for membership
and kernel).  Neighbour lists against brute force, the patch test through
unconforming zone boundaries, momentum balance of the pair forces, and the
reduction to the uniform method on a uniform lattice.  Host only."""
import math

import numpy as np
import pytest

from paper_1901_07374_amd import inputs as I


def small_graded(**over):
    return I.graded_notched_bar(R=0.6e-3, L=2.0e-3, rho=0.15e-3,
                                spacings=(0.05e-3, 0.1e-3, 0.2e-3),
                                bounds=(0.25e-3, 0.6e-3), **over)


def no_bc(p, **over):
    mats = [dict(m, **over) for m in p.materials]
    return I.Problem(p.name, p.X, p.V0, p.spec_offsets, mats, np.full(p.n, -1, np.int32), [],
                     p.v_init, p.steps, p.dx)


def test_support_radii(orc):
    p = small_graded()
    hs = orc.support_radii(p.V0, p.spec_id(), p.materials)
    dx = np.cbrt(p.V0)
    assert np.allclose(hs, 1.75 * dx, rtol=1e-15)
    assert set(np.round(hs / 1.75e-3, 6)) == {0.05, 0.1, 0.2}


def test_graded_neighbours_equal_brute_force(orc):
    p = small_graded()
    assert p.n <= 6000
    spec = p.spec_id()
    hs = orc.support_radii(p.V0, spec, p.materials)
    rp, col = orc.neighbors(p.X, spec, p.materials, hs)
    X = p.X
    for i in range(p.n):
        d = X - X[i]
        r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        hij = 0.5 * (hs + hs[i])
        m = r2 < hij * hij
        m[i] = False
        assert np.array_equal(col[rp[i]:rp[i + 1]], np.nonzero(m)[0]), i
    # pairs straddle the zone boundaries
    z = np.abs(X[:, 2])
    cross = sum(1 for i in range(p.n) for j in col[rp[i]:rp[i + 1]] if hs[i] != hs[j])
    assert cross > 1000


def test_graded_patch_test(orc):
    # first-order completeness of the corrected gradient does not depend on
    # the spacing: a linear velocity field gives dF/dt = G at every particle
    rng = np.random.default_rng(11)
    G = rng.uniform(-1e3, 1e3, (3, 3))
    p = small_graded()
    q = I.Problem(p.name, p.X, p.V0, p.spec_offsets, p.materials,
                  np.zeros(p.n, np.int32), [I.bc_group(7, grad=np.ravel(G))], p.v_init,
                  p.steps, p.dx)
    s = orc.Sim(q)
    s.step(1)
    dt = p.materials[0]["dt"]
    F = s.get("F").reshape(-1, 3, 3)
    assert np.abs(F - (np.eye(3) + dt * G)).max() < 1e-14


def test_graded_pair_forces_balance(orc):
    p = no_bc(small_graded())
    s = orc.Sim(p)
    st = I.random_state(p, seed=21)
    s.set_state(st)
    s.step(1)
    f = s.get("force")
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * np.abs(f).sum()


def test_uniform_lattice_reduces_to_uniform_support(orc):
    # h_per_spacing = 1.5 with V = dx^3 is the uniform method with h = 1.5 dx
    base = no_bc(I.cube(nside=8))
    dx = float(np.cbrt(base.V0[0]))
    grad = no_bc(I.cube(nside=8), h_per_spacing=1.5)
    a, b = orc.Sim(base), orc.Sim(grad)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert b.hs == pytest.approx(1.5 * dx, rel=1e-15)
    st = I.random_state(base, seed=22)
    a.set_state(st)
    b.set_state(st)
    a.step(3)
    b.step(3)
    for k in ("F", "sig", "force", "v", "e"):
        ra, rb = a.get(k), b.get(k)
        assert np.abs(ra - rb).max() <= 1e-12 * max(np.abs(ra).max(), 1e-300), k
