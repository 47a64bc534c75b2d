"""Oracle pins: kernel (Sec. 2.2), neighbour sets (Sec. 2) and the corrected
gradient (eqs. 1st_order_complete_SPH_gradient_approx, correction_matrix)."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1901_07374_amd import inputs as I


@pytest.mark.parametrize("h", [1e-3, 0.37])
def test_kernel_unit_integral_and_compact_support(orc, h):
    # normalisation condition: integral of W over its support is 1
    val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * orc.kernel(r, h)[0], 0, h,
                            points=[0.5 * h], epsabs=0, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-12
    assert orc.kernel(h, h) == (0.0, 0.0)
    assert orc.kernel(1.2 * h, h) == (0.0, 0.0)
    # W and W' continuous where the spline pieces meet, W' -> 0 at the support edge
    a, b = orc.kernel(0.5 * h * (1 - 1e-12), h), orc.kernel(0.5 * h * (1 + 1e-12), h)
    assert abs(a[0] - b[0]) < 1e-9 * abs(a[0]) and abs(a[1] - b[1]) < 1e-9 * abs(a[1])
    assert abs(orc.kernel(h * (1 - 1e-9), h)[1]) < 1e-12 * abs(orc.kernel(0.5 * h, h)[1])


def test_kernel_derivative_is_derivative(orc):
    h = 1.5e-3
    for q in [0.05, 0.3, 0.49, 0.51, 0.7, 0.95]:
        r = q * h
        d = 1e-7 * h
        fd = (orc.kernel(r + d, h)[0] - orc.kernel(r - d, h)[0]) / (2 * d)
        assert abs(fd - orc.kernel(r, h)[1]) < 1e-6 * abs(orc.kernel(r, h)[1])


def brute_force(X, spec, hs):
    n = X.shape[0]
    out = []
    for i in range(n):
        d = X - X[i]
        r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        m = (r2 < hs[spec[i]] ** 2) & (spec == spec[i])
        m[i] = False
        out.append(np.nonzero(m)[0])
    return out


@pytest.mark.parametrize("make", [
    lambda: I.cube(nside=9),
    lambda: I.notched_bar(dx=1.6e-3),
    lambda: I.subset(I.bar_batch(n_spec=4, lo=300, hi=900), [0, 1, 2, 3]),
])
def test_neighbours_equal_brute_force(orc, make):
    p = make()
    assert p.n <= 4000
    spec = p.spec_id()
    rp, col = orc.neighbors(p.X, spec, p.materials)
    ref = brute_force(p.X, spec, np.array([m["h"] for m in p.materials]))
    for i in range(p.n):
        assert np.array_equal(col[rp[i]:rp[i + 1]], ref[i]), i
    # symmetric relation, no cross-specimen pairs
    pairs = {(i, int(j)) for i in range(p.n) for j in col[rp[i]:rp[i + 1]]}
    assert all((j, i) in pairs for (i, j) in pairs)
    assert all(spec[i] == spec[j] for (i, j) in pairs)


def test_bulk_neighbour_count_on_perfect_lattice(orc):
    # h = 1.5 dx on a simple cubic lattice: 6 face + 12 edge neighbours
    p = I.cube(nside=7, jitter=0.0)
    rp, _ = orc.neighbors(p.X, p.spec_id(), p.materials)
    k = np.diff(rp).reshape(7, 7, 7)
    assert k[3, 3, 3] == 18 and k.min() == 6


def _affine_velocity_problem(p, G):
    q = I.Problem(p.name, p.X, p.V0, p.spec_offsets, p.materials,
                  np.zeros(p.n, np.int32), [I.bc_group(7, grad=np.ravel(G))], p.v_init,
                  p.steps, p.dx)
    return q


@pytest.mark.parametrize("make", [lambda: I.cube(nside=8),
                                  lambda: I.notched_bar(dx=1.6e-3)])
def test_patch_test_linear_velocity_gives_exact_Fdot(orc, make):
    # first-order completeness (corrected gradient): a linear velocity field
    # v = G X gives dF/dt = G at every particle, surface and jitter included
    rng = np.random.default_rng(3)
    G = rng.uniform(-1e3, 1e3, (3, 3))
    p = _affine_velocity_problem(make(), G)
    s = orc.Sim(p)
    s.step(1)
    dt = p.materials[0]["dt"]
    F = s.get("F").reshape(-1, 3, 3)
    err = np.abs(F - (np.eye(3) + dt * G)).max()
    assert err < 1e-14, err


def test_correction_matrix_is_symmetric_and_near_minus_identity_in_bulk(orc):
    p = I.cube(nside=7, jitter=0.0)
    s = orc.Sim(p)
    L = s.L.reshape(-1, 3, 3)
    assert np.abs(L - L.transpose(0, 2, 1)).max() < 1e-15
    Lc = L[3 * 49 + 3 * 7 + 3]
    # the neighbour-side gradient convention makes L negative definite
    assert np.allclose(Lc, Lc[0, 0] * np.eye(3), atol=1e-14)
    assert -1.0 < Lc[0, 0] < -0.5
    Li = s.Linv.reshape(-1, 3, 3)
    assert np.abs(np.einsum("nab,nbc->nac", L, Li) - np.eye(3)).max() < 1e-13


def test_isolated_particle_is_singular(orc):
    p = I.cube(nside=4, jitter=0.0)
    X = p.X.copy()
    X[0] = [-0.1, -0.1, -0.1]
    q = I.Problem(p.name, X, p.V0, p.spec_offsets, p.materials, p.bc_group, p.bc_groups,
                  p.v_init, p.steps, p.dx)
    with pytest.raises(orc.OracleError):
        orc.Sim(q)
