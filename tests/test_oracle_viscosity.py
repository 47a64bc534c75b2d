"""Oracle pins for the artificial particle-velocity damping (Sec. 2 says TLSPH
needs it against rank deficiency; the Monaghan form on the reference pair
geometry is a reading): pairwise antisymmetric, dissipative, zero for rigid
motion and separating pairs, linear / quadratic in the relative velocity for
its two coefficients, inactive for failed particles, and applied in the next
step's kick.  Host only."""
import numpy as np
import pytest

from paper_1901_07374_amd import inputs as I


def cube_problem(q1=1.0, q2=2.0, **over):
    p = I.cube(nside=7)
    mats = [dict(m, av_q1=q1, av_q2=q2, **over) for m in p.materials]
    return I.Problem(p.name, p.X, p.V0, p.spec_offsets, mats, np.full(p.n, -1, np.int32), [],
                     np.zeros_like(p.v_init), p.steps, p.dx)


def visc_after_one_step(orc, p, v, D=None):
    """fvisc computed in one step from half-step velocity v (no stress, no
    force otherwise: F = I, sigma = 0, Q = 0)."""
    o = orc.Sim(p)
    st = {"v": v}
    if D is not None:
        st["D"] = D
    o.set_state(st)
    o.step(1)
    return o.get("v"), o.get("fvisc")


def rand_v(p, seed, scale=3.0):
    return np.random.default_rng(seed).uniform(-scale, scale, (p.n, 3))


def test_momentum_and_dissipation(orc):
    p = cube_problem()
    v0 = rand_v(p, 1)
    v, f = visc_after_one_step(orc, p, v0)
    assert np.abs(f).max() > 0.0
    # antisymmetric pair forces: no net force
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * np.abs(f).sum()
    # the damping does negative work on the velocities it was computed from
    power = float(np.sum(v * f))
    assert power < 0.0


@pytest.mark.parametrize("kind", ["translation", "rotation", "expansion"])
def test_rigid_motion_and_separation_are_free(orc, kind):
    p = cube_problem()
    X = p.X - p.X.mean(axis=0)
    if kind == "translation":
        v0 = np.tile([1.5, -0.7, 2.0], (p.n, 1))
    elif kind == "rotation":
        w = np.array([300.0, -200.0, 500.0])
        v0 = np.cross(w, X)
    else:
        v0 = 500.0 * X
    _, f = visc_after_one_step(orc, p, v0)
    ref = np.abs(visc_after_one_step(orc, p, rand_v(p, 2))[1]).max()
    assert np.abs(f).max() <= 1e-12 * ref


def test_linear_and_quadratic_terms(orc):
    v0 = rand_v(cube_problem(), 3)
    # Q2 = 0: linear in the coefficient and in the velocity
    p1 = cube_problem(q1=1.0, q2=0.0)
    p2 = cube_problem(q1=2.0, q2=0.0)
    _, fa = visc_after_one_step(orc, p1, v0)
    _, fb = visc_after_one_step(orc, p2, v0)
    _, fc = visc_after_one_step(orc, p1, 2.0 * v0)
    assert np.allclose(fb, 2.0 * fa, rtol=1e-13, atol=1e-13 * np.abs(fa).max())
    assert np.allclose(fc, 2.0 * fa, rtol=1e-13, atol=1e-13 * np.abs(fa).max())
    # Q1 = 0: quadratic in the velocity
    pq = cube_problem(q1=0.0, q2=1.0)
    _, fq = visc_after_one_step(orc, pq, v0)
    _, fq2 = visc_after_one_step(orc, pq, 2.0 * v0)
    assert np.abs(fq).max() > 0.0
    assert np.allclose(fq2, 4.0 * fq, rtol=1e-13, atol=1e-13 * np.abs(fq).max())
    # off by default
    _, f0 = visc_after_one_step(orc, cube_problem(q1=0.0, q2=0.0), v0)
    assert not f0.any()


def test_failed_particles_take_no_part(orc):
    p = cube_problem()
    v0 = rand_v(p, 4)
    D = np.zeros(p.n)
    k = p.n // 2
    D[k] = 1.0
    _, f = visc_after_one_step(orc, p, v0, D)
    assert not f[k].any()
    # the pairs that remain still balance
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * np.abs(f).sum()


def test_applied_in_the_next_kick(orc):
    p = cube_problem()
    p_off = cube_problem(q1=0.0, q2=0.0)
    rng = np.random.default_rng(5)
    st = I.random_state(p, seed=5, frac_failed=0.0)
    fvis = rng.uniform(-1e-3, 1e-3, (p.n, 3))
    on, off = orc.Sim(p), orc.Sim(p_off)
    on.set_state(dict(st, fvisc=fvis))
    off.set_state(st)
    on.step(1)
    off.step(1)
    m = p.materials[0]
    # differences of nearly equal velocities and forces: rounding of the
    # larger quantities sets the absolute floor
    dv = on.get("v") - off.get("v")
    expect = m["dt"] * fvis / (m["rho0"] * p.V0[:, None])
    assert np.allclose(dv, expect, rtol=1e-9, atol=1e-15 * np.abs(off.get("v")).max())
    assert np.allclose(on.get("force") - off.get("force"), fvis, rtol=1e-9,
                       atol=1e-15 * np.abs(off.get("force")).max())
