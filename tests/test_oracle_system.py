"""Oracle pins on the assembled particle system: invariants of the damaged
TLSPH approximation (Secs. 3, 3.1), rigid motion, boundary conditions and
determinism.  Host only."""
import math

import numpy as np
import pytest

from paper_1901_07374_amd import inputs as I


def no_bc(p, **mat_over):
    mats = [dict(m, **mat_over) for m in p.materials]
    return I.Problem(p.name, p.X, p.V0, p.spec_offsets, mats, np.full(p.n, -1, np.int32), [],
                     p.v_init, p.steps, p.dx)


def all_bc(p, G, **mat_over):
    mats = [dict(m, **mat_over) for m in p.materials]
    return I.Problem(p.name, p.X, p.V0, p.spec_offsets, mats, np.zeros(p.n, np.int32),
                     [I.bc_group(7, grad=np.ravel(G))], p.v_init, p.steps, p.dx)


def rot(axis, th):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def voigt(a):
    return np.array([a[0, 0], a[1, 1], a[2, 2], a[1, 2], a[0, 2], a[0, 1]])


def full(s):
    return np.array([[s[0], s[5], s[4]], [s[5], s[1], s[3]], [s[4], s[3], s[2]]])


@pytest.mark.parametrize("prestress", [False, True])
def test_rigid_rotation(orc, prestress):
    """Secant rigid rotation v^{n+1/2} = (R^{n+1} - R^n) X / dt on every particle:
    F^n = R^n, no strain, and a deviatoric prestress is carried as R s0 R^T."""
    p = I.cube(nside=6)
    G0 = np.zeros((3, 3))
    q = all_bc(p, G0)
    s = orc.Sim(q)
    dt = q.materials[0]["dt"]
    s0 = np.zeros((3, 3))
    if prestress:
        s0 = np.array([[100e6, 40e6, -20e6], [40e6, -60e6, 10e6], [-20e6, 10e6, -40e6]])
        s.set("sig", np.tile(voigt(s0), (p.n, 1)))
    axis, nsteps, total = (1.0, 2.0, 0.5), 40, math.pi / 3
    for k in range(nsteps):
        Rk, Rk1 = rot(axis, total * k / nsteps), rot(axis, total * (k + 1) / nsteps)
        s.set_bc_groups([I.bc_group(7, grad=((Rk1 - Rk) / dt).ravel())])
        s.step(1)
    R = rot(axis, total)
    F = s.get("F").reshape(-1, 3, 3)
    assert np.abs(F - R).max() < 1e-13
    x = p.X + s.get("u")
    assert np.abs(x - p.X @ R.T).max() < 1e-15
    sig = s.get("sig")
    expect = voigt(R @ s0 @ R.T)
    assert np.abs(sig - expect).max() < 1e-12 * max(np.abs(s0).max(), 1.0) + 1e-3
    assert s.get("eps_p").max() == 0.0
    if not prestress:
        assert np.abs(s.get("force")).max() < 1e-9


def random_state(orc, p, seed, **kw):
    st = I.random_state(p, seed, **kw)
    return st


def test_total_internal_force_vanishes(orc):
    # pairwise anti-symmetry of the damaged nodal forces (Sec. 3.1): the sum
    # over all particles is zero for any state, hourglass forces included
    p = no_bc(I.notched_bar(dx=1.2e-3))
    s = orc.Sim(p)
    s.set_state(I.random_state(p, 11))
    s.step(1)
    f = s.get("force")
    assert np.abs(f.sum(0)).max() < 1e-13 * np.abs(f).sum()


def test_power_identity_links_forces_and_Fdot(orc):
    """Sec. 3.1: the damaged force is the one whose power balances the stress
    power of the damaged dF/dt: sum_i f_i . v_i = - sum_i V_i P_i : dF_i/dt for
    any velocity field (hourglass off, no prescribed velocities)."""
    p = no_bc(I.cube(nside=7), hg_alpha=0.0)
    s = orc.Sim(p)
    st = I.random_state(p, 12, frac_failed=0.0)
    s.set_state(st)
    F0 = st["F"].copy()
    s.step(1)
    dt = p.materials[0]["dt"]
    Fdot = (s.get("F") - F0).reshape(-1, 3, 3) / dt
    L = s.L.reshape(-1, 3, 3)
    P = st["Q"].reshape(-1, 3, 3) @ L.transpose(0, 2, 1)
    stress_power = np.sum(p.V0[:, None, None] * P * Fdot)
    power = np.sum(s.get("force") * s.get("v"))
    assert abs(power + stress_power) < 1e-9 * np.sum(np.abs(p.V0[:, None, None] * P * Fdot))


def test_uniform_deformation_interior_and_hourglass(orc):
    """Uniform F with consistent displacement on a perfect lattice: interior
    nodal forces vanish by symmetry; with zero stress all forces (hourglass
    included) vanish everywhere."""
    n = 8
    p = no_bc(I.cube(nside=n, jitter=0.0))
    s = orc.Sim(p)
    rng = np.random.default_rng(2)
    F0 = np.eye(3) + rng.uniform(-0.01, 0.01, (3, 3))
    s.set("F", np.tile(F0.ravel(), (p.n, 1)))
    s.set("u", p.X @ (F0 - np.eye(3)).T)
    s.step(1)
    assert np.abs(s.get("force")).max() < 1e-9      # sigma = 0: hourglass alone
    s = orc.Sim(p)
    sig0 = np.array([[300e6, 50e6, 0], [50e6, -100e6, 20e6], [0, 20e6, 80e6]])
    J = np.linalg.det(F0)
    P0 = J * sig0 @ np.linalg.inv(F0).T
    Linv = s.Linv.reshape(-1, 3, 3)
    s.set("F", np.tile(F0.ravel(), (p.n, 1)))
    s.set("u", p.X @ (F0 - np.eye(3)).T)
    s.set("Q", (P0[None] @ Linv.transpose(0, 2, 1)).reshape(-1, 9))
    s.step(1)
    f = s.get("force").reshape(n, n, n, 3)
    scale = np.abs(f).max()
    assert scale > 1.0
    assert np.abs(f[2:-2, 2:-2, 2:-2]).max() < 1e-12 * scale


def test_hourglass_is_restoring(orc):
    p = no_bc(I.cube(nside=7, jitter=0.0))
    s = orc.Sim(p)
    u = np.zeros((p.n, 3))
    k = 3 * 49 + 3 * 7 + 3
    u[k, 0] = 1e-6
    s.set("u", u)
    s.step(1)
    f = s.get("force")
    assert f[k, 0] < 0 and abs(f[k, 1]) < 1e-12 * abs(f[k, 0])
    assert np.abs(f.sum(0)).max() < 1e-13 * np.abs(f).sum()


def test_failed_particle_is_a_crack(orc):
    """D_k = 1 (Sec. 3.1): k carries no stress, is held at rest, and drops out of
    its neighbours' dF/dt, which is the corrected gradient over the remaining
    support; with Q_k = 0 its neighbours' forces no longer depend on it."""
    p = I.cube(nside=7)
    rng = np.random.default_rng(4)
    G = rng.uniform(-500, 500, (3, 3))
    q = all_bc(p, G)
    s = orc.Sim(q)
    k = 3 * 49 + 3 * 7 + 2
    D = np.zeros(p.n)
    D[k] = 1.0
    s.set("D", D)
    s.step(1)
    dt = q.materials[0]["dt"]
    F = s.get("F").reshape(-1, 3, 3)
    assert np.all(s.get("v")[k] == 0.0)
    nb = set(s.col[s.row_ptr[k]:s.row_ptr[k + 1]].tolist())
    Linv = s.Linv.reshape(-1, 3, 3)
    h = q.materials[0]["h"]
    for i in range(p.n):
        if i == k:
            continue
        expect = np.eye(3) + dt * G
        if i in nb:
            Xik = p.X[k] - p.X[i]
            r = np.linalg.norm(Xik)
            gW = orc.kernel(r, h)[1] * Xik / r
            gh = Linv[i].T @ gW
            expect = expect - dt * p.V0[k] * np.outer(G @ Xik, gh)
        assert np.abs(F[i] - expect).max() < 1e-14, i
    # forces of the neighbours do not see u_k, F_k once Q_k = 0
    p2 = no_bc(I.cube(nside=7))
    outs = []
    for pert in (0.0, 1e-5):
        s2 = orc.Sim(p2)
        st = I.random_state(p2, 9, frac_failed=0.0)
        st["D"][k] = 1.0
        st["Q"][k] = 0.0
        st["u"][k] += pert
        st["F"][k] += pert * 100
        s2.set_state(st)
        s2.step(1)
        outs.append(s2.get("force"))
    assert np.array_equal(outs[0][list(nb)], outs[1][list(nb)])


@pytest.mark.parametrize("smooth", [True, False])
def test_momentum_and_energy_in_free_vibration(orc, smooth):
    """eq. conservation3 integrated alongside the leapfrog: kinetic plus
    internal energy stays bounded (no secular drift), momentum is exact."""
    p = no_bc(I.cube(nside=8), hg_alpha=0.0)
    s = orc.Sim(p)
    rng = np.random.default_rng(8)
    if smooth:
        v0 = np.zeros((p.n, 3))
        v0[:, 0] = 0.5 * np.sin(p.X[:, 2] / 8e-3 * np.pi)
    else:
        v0 = rng.uniform(-0.5, 0.5, (p.n, 3))
    s.set("v", v0)
    m = p.materials[0]["rho0"] * p.V0
    P0 = (m[:, None] * v0).sum(0)
    E0 = 0.5 * np.sum(m[:, None] * v0 ** 2)
    Es = []
    for _ in range(10):
        s.step(20)
        v = s.get("v")
        assert np.abs((m[:, None] * v).sum(0) - P0).max() < 1e-12 * np.abs(m[:, None] * v0).sum()
        Es.append(0.5 * np.sum(m[:, None] * v ** 2) + np.sum(m * s.get("e")))
    assert s.get("eps_p").max() == 0.0
    tol = 1e-2 if smooth else 8e-2
    assert max(abs(E - E0) for E in Es) < tol * E0
    assert abs(Es[-1] - Es[0]) < 0.4 * tol * E0


def test_prescribed_velocity_ramp(orc):
    p = I.notched_bar(dx=1.5e-3)
    s = orc.Sim(p)
    s.step(7)
    dt = p.materials[0]["dt"]
    th = 6.5 * dt
    v = s.get("v")
    ramp = 10.0 * (1 - math.exp(-th / 1e-3))
    assert np.allclose(v[p.bc_group == 1, 2], ramp, rtol=0, atol=1e-15)
    assert np.allclose(v[p.bc_group == 0, 2], -ramp, rtol=0, atol=1e-15)
    assert s.get("t")[0] == pytest.approx(7 * dt, rel=1e-15)


def test_rigid_wall(orc):
    p = I.taylor_bar(dx=0.8e-3, R=3e-3, L=8e-3)
    s = orc.Sim(p)
    s.step(40)
    x = p.X + s.get("u")
    assert x[:, 2].min() >= 0.0
    on = x[:, 2] == 0.0
    assert on.sum() > 0 and np.all(s.get("v")[on, 2] >= 0.0)


def test_thread_count_does_not_change_results(orc):
    p = no_bc(I.notched_bar(dx=1.0e-3))
    out = []
    for nt in (1, 3, 8):
        orc.set_threads(nt)
        s = orc.Sim(p)
        s.set_state(I.random_state(p, 21))
        s.step(3)
        out.append({k: s.get(k) for k in ("u", "v", "F", "sig", "Q", "D", "f_void", "eps_p")})
    orc.set_threads(8)
    for o in out[1:]:
        for k in o:
            assert np.array_equal(o[k], out[0][k]), k


def test_diagnostics_are_the_plain_sums(orc):
    """The oracle's diagnostics (the grip force and displacement the runs of
    Sec. 6 are read by, the energies of eq. conservation3, failed count and
    max D) equal the same sums taken by numpy over its exported state, for
    two specimens with both grips, some particles failed."""
    p = I.bar_batch(n_spec=2, counts=(1500, 2500))
    s = orc.Sim(p)
    st = I.random_state(p, 31)
    s.set_state(st)
    s.step(2)
    sd, bd = s.diagnostics()
    sid = p.spec_id()
    v, e, D, u, f = (s.get(k) for k in ("v", "e", "D", "u", "force"))
    for q in range(p.n_spec):
        sel = sid == q
        m = p.materials[q]["rho0"] * p.V0[sel]
        assert sd[q, 0] == pytest.approx(0.5 * np.sum(m[:, None] * v[sel] ** 2), rel=1e-13)
        assert sd[q, 1] == pytest.approx(np.sum(m * e[sel]), rel=1e-13)
        assert sd[q, 2] == np.sum(D[sel] >= 1.0) and sd[q, 2] > 0
        assert sd[q, 3] == D[sel].max()
        assert sd[q, 4] == s.get("t")[q]
    for g in range(len(p.bc_groups)):
        sel = p.bc_group == g
        assert bd[g, 6] == sel.sum() > 0
        assert np.allclose(bd[g, :3], f[sel].sum(0), rtol=1e-13, atol=1e-13 * np.abs(f[sel]).sum())
        assert np.allclose(bd[g, 3:6], u[sel].mean(0), rtol=1e-13, atol=1e-20)


def test_diagnostics_energy_in_free_vibration(orc):
    """Read through the diagnostics, the free elastic vibration keeps kinetic
    plus internal energy at the initial kinetic energy (eq. conservation3,
    bounded leapfrog error)."""
    p = no_bc(I.cube(nside=8), hg_alpha=0.0)
    s = orc.Sim(p)
    v0 = np.zeros((p.n, 3))
    v0[:, 0] = 0.5 * np.sin(p.X[:, 2] / 8e-3 * np.pi)
    s.set("v", v0)
    E0 = 0.5 * np.sum(p.materials[0]["rho0"] * p.V0[:, None] * v0 ** 2)
    for _ in range(5):
        s.step(40)
        sd, _ = s.diagnostics()
        assert sd[0, 1] > 0.0
        assert abs(sd[0, 0] + sd[0, 1] - E0) < 1e-2 * E0
