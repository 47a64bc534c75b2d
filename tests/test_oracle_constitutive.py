"""Oracle pins for the constitutive pieces (Secs. 4-5): closed forms, textbook
special cases and the paper's defining equations checked on the converged
state.  Host only."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_1901_07374_amd import inputs as I


def steel(**over):
    m = I.material(1e-3, I.DMG_NONE)
    m.update(over)
    return m


def K_of(m):
    return m["rho0"] * m["c0"] ** 2


def G_of(m):
    return m["E"] / (2 * (1 + m["nu"]))


def vm(s6):
    s = np.asarray(s6, float)
    p = s[:3].mean()
    d = s[:3] - p
    return math.sqrt(1.5 * (d @ d + 2 * (s[3:] @ s[3:])))


def full(s6):
    s = s6
    return np.array([[s[0], s[5], s[4]], [s[5], s[1], s[3]], [s[4], s[3], s[2]]])


def voigt(a):
    return np.array([a[0, 0], a[1, 1], a[2, 2], a[1, 2], a[0, 2], a[0, 1]])


def drive(pt, F_of_t, nsteps, dt):
    """Secant drive: dF/dt = (F(t_{n+1}) - F_n)/dt each step."""
    hist = []
    for k in range(nsteps):
        Fn = pt.F.reshape(3, 3)
        Fd = (F_of_t((k + 1) * dt) - Fn) / dt
        pt.update(Fd, dt)
        hist.append((pt.sig.copy(), pt.eps_p, pt.d_init, pt.D, pt.f_void, pt.w_p))
    return hist


# --------------------------------------------------------------------------
# Mie-Grueneisen EOS (Sec. 4, eq. pH)
# --------------------------------------------------------------------------
def test_eos_linear_limit(orc):
    m = steel(S_alpha=0.0, Gamma0=0.0)
    for J in [0.97, 0.999, 1.0, 1.001, 1.03]:
        sm = orc.mean_stress_eos(m, J)
        assert abs(sm - K_of(m) * (J - 1.0)) <= 1e-14 * K_of(m)


def test_eos_on_the_hugoniot(orc):
    # Gamma0 = 0: the EOS is the shock Hugoniot of Us = c0 + S up (Rankine-Hugoniot:
    # p = rho0 Us up, rho/rho0 = Us / (Us - up))
    m = steel()
    for up in [10.0, 100.0, 500.0]:
        Us = m["c0"] + m["S_alpha"] * up
        eta = Us / (Us - up)
        p = m["rho0"] * Us * up
        assert abs(orc.mean_stress_eos(m, 1.0 / eta) + p) <= 1e-12 * p


def test_eos_textbook_mu_form_with_gruneisen_energy(orc):
    # p = rho0 c0^2 mu [1 + (1 - G0/2) mu] / [1 - (S - 1) mu]^2 + G0 rho0 e, mu = eta - 1
    m = steel(Gamma0=1.8)
    e = 3.0e4
    for J in [0.9, 0.98, 0.999]:
        mu = 1.0 / J - 1.0
        p = K_of(m) * mu * (1 + (1 - 0.9) * mu) / (1 - (m["S_alpha"] - 1) * mu) ** 2 \
            + 1.8 * m["rho0"] * e
        assert abs(orc.mean_stress_eos(m, J, 0.0, e) + p) <= 1e-13 * abs(p)


def test_eos_bulk_modulus(orc):
    m = steel(Gamma0=1.2)
    d = 1e-7
    dp = (orc.mean_stress_eos(m, 1 / (1 + d)) - orc.mean_stress_eos(m, 1 / (1 - d))) / (2 * d)
    assert abs(-dp - K_of(m)) < 1e-6 * K_of(m)


def test_eos_damaged_branch_reading(orc):
    # tension with damage: prefactor rho0 (1 - D) and eta = (1 - D)/J
    m = steel(S_alpha=0.0, Gamma0=0.0)
    D, J = 0.3, 1.002
    expect = m["rho0"] * (1 - D) * m["c0"] ** 2 * (J / (1 - D) - 1.0)
    assert abs(orc.mean_stress_eos(m, J, D) - expect) <= 1e-13 * abs(expect)
    # compression, or no damage, or the damage branch switched off (GTN): undamaged
    assert orc.mean_stress_eos(m, 0.998, D) == orc.mean_stress_eos(m, 0.998, 0.0)
    assert abs(orc.mean_stress_eos(m, J, 0.0) - K_of(m) * (J - 1)) <= 1e-14 * K_of(m)
    assert orc.mean_stress_eos(m, J, D, 0.0, False) == orc.mean_stress_eos(m, J, 0.0)


# --------------------------------------------------------------------------
# Johnson-Cook flow stress (Sec. 4, eq. JC_viscoplastic_model)
# --------------------------------------------------------------------------
def test_flow_stress_values(orc):
    m = steel()
    assert orc.flow_stress(m, 0.0, 0.0) == m["A"]
    assert orc.flow_stress(m, 1.0, 0.5) == pytest.approx(m["A"] + m["B"], rel=1e-15)
    assert orc.flow_stress(m, 0.2, math.e) == pytest.approx(
        (m["A"] + m["B"] * 0.2 ** m["n"]) * (1 + m["C"]), rel=1e-15)


# --------------------------------------------------------------------------
# objective rotation
# --------------------------------------------------------------------------
def test_hughes_winget_is_cayley_rotation(orc):
    rng = np.random.default_rng(1)
    s = rng.normal(size=(3, 3))
    s = s + s.T
    om, dt = 3.0e5, 2e-6
    w = om * np.array([[0, -1, 0], [1, 0, 0], [0, 0, 0.0]])
    th = 2 * math.atan(om * dt / 2)
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    out = orc.hughes_winget(dt, w, s)
    assert np.abs(out - R @ s @ R.T).max() < 1e-14 * np.abs(s).max()


# --------------------------------------------------------------------------
# Algorithm 1 under homogeneous uniaxial strain
# --------------------------------------------------------------------------
def test_uniaxial_elastic_closed_form(orc):
    m = steel(S_alpha=0.0, Gamma0=0.0, A=1e12)
    pt = orc.Point(m)
    rate, dt, n = 10.0, 1e-6, 300
    drive(pt, lambda t: np.diag([1 + rate * t, 1, 1]), n, dt)
    eps = rate * n * dt
    K, G = K_of(m), G_of(m)
    s = pt.sig
    assert abs(s[0] - (K * eps + 4 / 3 * G * math.log1p(eps))) < 1e-8 * K * eps
    assert abs(s[1] - (K * eps - 2 / 3 * G * math.log1p(eps))) < 1e-8 * K * eps
    assert abs(s[1] - s[2]) < 1e-6 and np.abs(s[3:]).max() < 1e-6


@pytest.mark.parametrize("D", [0.0, 0.3])
def test_uniaxial_perfect_plasticity(orc, D):
    # B = C = 0: sigma_eq = A (1 - D) once yielded; eps_p grows by 2/3 of the
    # axial log-strain increment (3G(1 - D) divisor matches the 2G(1 - D) trial)
    m = steel(S_alpha=0.0, Gamma0=0.0, B=0.0, C=0.0)
    pt = orc.Point(m, D=D)
    G = G_of(m)
    rate, dt, n = 20.0, 1e-6, 400
    hist = drive(pt, lambda t: np.diag([1 + rate * t, 1, 1]), n, dt)
    lny = m["A"] / (2 * G)             # first yield at 2 G ln(1+eps) = A (D cancels)
    for k, (s, ep, *_) in enumerate(hist):
        le = math.log1p(rate * (k + 1) * dt)
        if le < lny - 2 * rate * dt:
            assert ep == 0.0 and abs(vm(s) - 2 * G * (1 - D) * le) < 1e-6 * m["A"]
        elif le > lny + 2 * rate * dt:
            assert abs(vm(s) - m["A"] * (1 - D)) < 1e-9 * m["A"]
            assert abs(ep - 2 / 3 * (le - lny)) < 1e-8
    assert pt.eps_p > 0.0


def test_explicit_hardening_within_one_increment(orc):
    m = steel(S_alpha=0.0, Gamma0=0.0, C=0.0)
    pt = orc.Point(m)
    rate, dt = 20.0, 1e-6
    hist = drive(pt, lambda t: np.diag([1 + rate * t, 1, 1]), 600, dt)
    prev, plastic_steps = 0.0, 0
    for s, ep, *_ in hist:
        if ep > prev:  # a yielding step ends on the surface of the step's start
            plastic_steps += 1
            assert abs(vm(s) - (m["A"] + m["B"] * prev ** m["n"])) < 1e-9 * m["A"]
        else:
            assert vm(s) < m["A"] + m["B"] * prev ** m["n"]
        prev = ep
    assert plastic_steps > 100


def isochoric(lam_rate, J0=1.0):
    c = J0 ** (1.0 / 3.0)
    return lambda t: c * np.diag([math.exp(lam_rate * t), math.exp(-0.5 * lam_rate * t),
                                  math.exp(-0.5 * lam_rate * t)])


def test_rate_hardening_steady_state(orc):
    m = steel(B=0.0, C=0.014)
    pt = orc.Point(m, F=isochoric(0.0)(0))
    rate, dt = 1e4, 1e-7
    drive(pt, isochoric(rate), 3000, dt)
    assert pt.eps_p_rate == pytest.approx(rate, rel=1e-3)
    assert vm(pt.sig) == pytest.approx(m["A"] * (1 + m["C"] * math.log(rate)), rel=1e-6)


# --------------------------------------------------------------------------
# damage initiation and evolution (Secs. 5.1-5.3)
# --------------------------------------------------------------------------
def test_johnson_cook_damage_closed_form(orc):
    m = I.material(1e-3, I.DMG_JC, B=0.0, C=0.0, D1=0.02, D2=0.08, D4=0.0, S_alpha=0.0,
                   Gamma0=0.0)
    J0 = 1.001
    pt = orc.Point(m, F=isochoric(0.0, J0)(0))
    rate, dt = 50.0, 1e-6
    hist = drive(pt, isochoric(rate, J0), 3000, dt)
    sm = K_of(m) * (J0 - 1.0)
    ef = m["D1"] + m["D2"] * math.exp(m["D3"] * sm / m["A"])
    seen_fail = False
    for s, ep, dini, D, *_ in hist:
        if dini < 1.0:
            assert D == 0.0
            assert abs(dini - ep / ef) < 2e-9, (dini, ep / ef)
        assert D == pytest.approx(min(1.0, max(0.0, 10 * (dini - 1))), abs=1e-15)
        if D >= 1.0:
            seen_fail = True
            assert np.all(s == 0.0)
    assert seen_fail


def test_johnson_cook_damage_rate_term(orc):
    m = I.material(1e-3, I.DMG_JC, B=0.0, C=0.0, D4=0.05, D3=0.0, S_alpha=0.0, Gamma0=0.0)
    pt = orc.Point(m)
    rate, dt = 500.0, 1e-6
    hist = drive(pt, isochoric(rate), 800, dt)
    (s1, e1, d1, *_), (s2, e2, d2, *_) = hist[-201], hist[-1]
    ef = (m["D1"] + m["D2"]) * (1 + rate) ** 0.05
    assert (d2 - d1) / (e2 - e1) == pytest.approx(1 / ef, rel=1e-6)


def test_cockcroft_latham_closed_form(orc):
    m = I.material(1e-3, I.DMG_CL, Wcr=50e6, B=0.0, C=0.0, S_alpha=0.0, Gamma0=0.0)
    J0 = 1.0005
    pt = orc.Point(m, F=isochoric(0.0, J0)(0))
    hist = drive(pt, isochoric(50.0, J0), 3000, 1e-6)
    s1 = K_of(m) * (J0 - 1.0) + 2.0 / 3.0 * m["A"]
    reached = False
    for s, ep, dini, D, f, wp in hist:
        if dini < 1.0:
            assert abs(wp - s1 * ep) < 1e-9 * m["Wcr"]
            assert abs(dini - wp / m["Wcr"]) < 1e-15
            reached = reached or dini > 0.5
    assert reached and pt.D > 0


def test_failed_point_carries_no_stress(orc):
    m = I.material(1e-3, I.DMG_JC)
    pt = orc.Point(m, D=1.0, sig=[1e8] * 6)
    pt.update(np.full(9, 10.0))
    assert np.all(pt.sig == 0.0) and np.all(pt.P == 0.0)


# --------------------------------------------------------------------------
# GTN (Sec. 5.4, Algorithm 2)
# --------------------------------------------------------------------------
def gtn_mat(**over):
    base = dict(C=0.0, S_alpha=0.0, Gamma0=0.0)
    base.update(over)
    return I.material(1e-3, I.DMG_GTN, **base)


def test_gtn_without_voids_is_von_mises_with_implicit_linear_hardening(orc):
    m = gtn_mat(f0=0.0, fN=0.0, k_omega=0.0, n=1.0)
    G, H = G_of(m), m["B"]
    eps_n = 0.05
    s0 = m["A"] + H * eps_n
    sd = np.diag([2.0, -1.0, -1.0]) * s0 / 3.0
    pt = orc.Point(m, sig=voigt(sd), eps_p=eps_n, f_void=0.0, D=0.0)
    dt, a = 1e-6, 300.0
    pt.update(np.diag([a, -0.5 * a, -0.5 * a]), dt)
    d = np.array([a, -0.5 * a, -0.5 * a]) / (1 + 0.5 * dt * np.array([a, -0.5 * a, -0.5 * a]))
    de = d * dt - (d * dt).mean()
    s_tr = s0 + 3 * G * math.sqrt(2.0 / 3.0 * (de @ de))
    dlam = (s_tr - s0) / (3 * G + H)
    assert pt.eps_p - eps_n == pytest.approx(dlam, rel=1e-12)
    assert vm(pt.sig) == pytest.approx(s0 + H * dlam, rel=1e-12)
    assert pt.f_void == 0.0 and pt.D == 0.0


def _inject_trial(orc, m, J0, sd, eps, f, D):
    """A point whose trial state is the injected one: dF/dt = 0, F = J0^(1/3) I."""
    F0 = J0 ** (1.0 / 3.0) * np.eye(3)
    pt = orc.Point(m, F=F0, sig=voigt(sd), eps_p=eps, f_void=f, D=D)
    pt.update(np.zeros(9))
    return pt


def test_gtn_zero_triaxiality_gives_one_minus_q1_fstar(orc):
    m = gtn_mat()
    for f in [0.01, 0.1, 0.2]:
        fs = orc.fstar(m, f)
        D = m["q1"] * fs
        sd = np.diag([1.0, -1.0, 0.0]) * 1.5e9
        pt = _inject_trial(orc, m, 1.0, sd, 0.1, f, D)
        x = vm(pt.sig) / orc.flow_stress(m, pt.eps_p)
        assert x == pytest.approx(1 - m["q1"] * fs, rel=1e-12)


@pytest.mark.parametrize("J0,f", [(1.003, 0.02), (0.998, 0.05), (1.006, 0.2), (1.0015, 0.001)])
def test_gtn_converged_state_satisfies_algorithm_2(orc, J0, f):
    m = gtn_mat(n=0.26, k_omega=2.0)
    rng = np.random.default_rng(int(J0 * 1e4))
    sd = rng.normal(size=(3, 3))
    sd = sd + sd.T
    sd -= np.trace(sd) / 3 * np.eye(3)
    sd *= 1.3e9 / math.sqrt(1.5 * np.sum(sd * sd))
    eps_n = 0.08
    fs = orc.fstar(m, f)
    D = m["q1"] * fs
    pt = _inject_trial(orc, m, J0, sd, eps_n, f, D)
    G = G_of(m)
    q1, q2, q3 = m["q1"], m["q2"], m["q3"]
    seq_tr = math.sqrt(1.5 * np.sum(sd * sd))
    sm_tr = orc.mean_stress_eos(m, J0, D, 0.0, False)
    sstar = sm_tr / seq_tr
    dem = pt.eps_p - eps_n
    sM = orc.flow_stress(m, pt.eps_p)
    s_out = full(pt.sig)
    sm_out = np.trace(s_out) / 3
    sy = vm(pt.sig)
    x = sy / sM
    # yield surface (Algorithm 2 first loop)
    Phi = x * x + 2 * q1 * fs * math.cosh(1.5 * q2 * sstar * x) - (1 + q3 * fs * fs)
    assert abs(Phi) < 1e-12
    # strain-increment equation (second loop, g = 0)
    sh = math.sinh(1.5 * q2 * sstar * x)
    rhs = (seq_tr - sy) / (3 * G * (1 - D) * (1 - f)) * (x + 1.5 * q1 * q2 * f * sstar * sh)
    assert dem == pytest.approx(rhs, rel=1e-10)
    # equivalence of matrix and macroscopic plastic work
    dep_eq = (seq_tr - sy) / (3 * G * (1 - D))
    alpha = 1.5 * sM / sy * q1 * q2 * f * sh
    assert (1 - f) * sM * dem == pytest.approx(sy * dep_eq * (1 + sstar * alpha), rel=1e-10)
    # radial return of the deviator and constant triaxiality of the mean stress
    sd_out = s_out - sm_out * np.eye(3)
    assert np.abs(sd_out - sy / seq_tr * sd).max() < 1e-12 * seq_tr
    assert sm_out == pytest.approx(sm_tr * sy / seq_tr, rel=1e-12)


def test_gtn_nucleation_follows_normal_cdf(orc):
    m = gtn_mat(f0=0.0, k_omega=0.0, B=0.0)
    pt = orc.Point(m, f_void=0.0, D=0.0)
    drive(pt, isochoric(100.0), 3000, 2e-6)
    e = pt.eps_p
    Fcdf = lambda z: stats.norm.cdf(z)
    expect = m["fN"] * (Fcdf((e - m["eN"]) / m["sN"]) - Fcdf(-m["eN"] / m["sN"]))
    assert e > 0.45
    assert pt.f_void == pytest.approx(expect, rel=2e-3)


def test_gtn_shear_softening_ode(orc):
    # pure shear (omega = 1, sigma* = 0, alpha = 0): df/deps_M = (1 - f) f k_w / x,
    # x = 1 - q1 f*, integrated by scipy as the reference
    m = gtn_mat(f0=0.002, fN=0.0, k_omega=3.5, B=0.0, fc=0.5, fF=0.6)
    pt = orc.Point(m, f_void=0.002, D=m["q1"] * 0.002)
    rate = 100.0
    drive(pt, lambda t: np.diag([math.exp(rate * t), math.exp(-rate * t), 1.0]), 2500, 2e-6)
    e = pt.eps_p
    sol = integrate.solve_ivp(lambda _, f: (1 - f) * f * 3.5 / (1 - 1.5 * f), (0.0, e), [0.002],
                              rtol=1e-11, atol=1e-14)
    assert e > 0.3
    assert pt.f_void == pytest.approx(sol.y[0, -1], rel=2e-3)


def test_fstar_continuity_and_failure(orc):
    m = gtn_mat()
    fc, fF, q1 = m["fc"], m["fF"], m["q1"]
    assert orc.fstar(m, fc) == fc
    assert abs(orc.fstar(m, fc * (1 + 1e-12)) - fc) < 1e-11
    assert orc.fstar(m, fF * (1 - 1e-15)) == pytest.approx(1 / q1, rel=1e-12)
    assert orc.fstar(m, 0.9) == 1 / q1
    pt = _inject_trial(orc, m, 1.002, np.diag([2.0, -1, -1]) * 1e9, 0.3, fF * 0.999, 0.99)
    assert pt.f_void >= fF and pt.D == 1.0 and np.all(pt.sig == 0.0)


def test_omega(orc):
    rng = np.random.default_rng(5)
    assert orc.omega(voigt(np.diag([3.0, 1.0, 1.0]))) == pytest.approx(0.0, abs=1e-14)
    assert orc.omega(voigt(np.diag([-2.0, 1.0, 1.0]))) == pytest.approx(0.0, abs=1e-14)
    assert orc.omega(voigt(np.diag([1.0, -1.0, 0.0]))) == pytest.approx(1.0, abs=1e-14)
    for _ in range(20):
        a = rng.normal(size=(3, 3))
        a = a + a.T
        w = orc.omega(voigt(a))
        assert 0.0 <= w <= 1.0
        assert orc.omega(voigt(3.7 * a)) == pytest.approx(w, abs=1e-12)
        assert orc.omega(voigt(a + 5.0 * np.eye(3))) == pytest.approx(w, abs=1e-12)
        Rq, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        assert orc.omega(voigt(Rq @ a @ Rq.T)) == pytest.approx(w, abs=1e-10)


def test_principal_max_matches_eigvalsh(orc):
    rng = np.random.default_rng(7)
    for scale in [1.0, 1e9, 1e-3]:
        for _ in range(50):
            a = rng.normal(size=(3, 3)) * scale
            a = a + a.T
            ref = np.linalg.eigvalsh(a).max()
            assert abs(orc.principal_max(voigt(a)) - ref) < 1e-14 * np.abs(a).max() * 10
    assert orc.principal_max(voigt(np.diag([1.0, 5.0, -2.0]))) == 5.0


@pytest.mark.parametrize("model", [I.DMG_JC, I.DMG_GTN])
def test_elastic_shear_of_a_damaged_point(orc, model):
    """A damaged point (D > 0) under a small symmetric shear stays elastic;
    the deviatoric stress takes 2 G (1 - D) times the strain increment
    d dt, d = sym(dF/dt Fbar^-1) with the midpoint Fbar (Algorithm 1 trial
    line and Algorithm 2 trial state, Sec. 4-5).  For GTN, D = q1 f*(f)."""
    m = I.material(1e-3, model)
    G = G_of(m)
    f = 0.1
    D = m["q1"] * orc.fstar(m, f) if model == I.DMG_GTN else 0.3
    pt = orc.Point(m, D=D, f_void=f, eps_p=0.01)
    dt = m["dt"]
    Fd = np.zeros((3, 3))
    Fd[0, 1] = Fd[1, 0] = 0.5 * 1e3       # symmetric: no spin
    pt.update(Fd, dt)
    Fb = np.eye(3) + 0.5 * dt * Fd
    d = Fd @ np.linalg.inv(Fb)
    assert pt.eps_p == pytest.approx(0.01, abs=0)      # elastic
    assert pt.sig[5] == pytest.approx(2 * G * (1 - D) * d[0, 1] * dt, rel=1e-12)


@pytest.mark.parametrize("J0,f", [(1.004, 0.05), (1.002, 0.12)])
def test_gtn_yield_onset_at_high_triaxiality(orc, J0, f):
    """Algorithm 2 decides elastic or plastic by the sign of the trial yield
    function Phi = r^2 + 2 q1 f* cosh(3/2 q2 sigma_m / sigma_M) - (1 + q3 f*^2)
    (eq. yield_GTN with r = sigma_eq / sigma_M).  Trial states 0.1 % inside
    and outside the surface, at high mean stress, must fall on either side."""
    m = gtn_mat(n=0.26)
    fs = orc.fstar(m, f)
    D = m["q1"] * fs
    eps_n = 0.05
    sM = orc.flow_stress(m, eps_n)
    sm = orc.mean_stress_eos(m, J0, D, 0.0, False)
    c = (1 + m["q3"] * fs * fs) - 2 * m["q1"] * fs * math.cosh(1.5 * m["q2"] * sm / sM)
    assert c > 0.05
    seq0 = sM * math.sqrt(c)
    shape = np.diag([1.0, -0.5, -0.5])                    # von Mises norm 1.5
    for scale, plastic in ((0.999, False), (1.001, True)):
        sd = shape * (scale * seq0 / 1.5)
        pt = _inject_trial(orc, m, J0, sd, eps_n, f, D)
        assert (pt.eps_p > eps_n) == plastic, (scale, pt.eps_p - eps_n)


# --------------------------------------------------------------------------
# GTN void growth (Sec. 5.4, eq. GTN_damage_growth), derived here from the
# yield function by normality rather than from Algorithm 2's closed form
# --------------------------------------------------------------------------
def _gtn_phi(s33, sM, fs, q1, q2, q3):
    """eq. yield_GTN as a function of the full stress tensor."""
    sm = np.trace(s33) / 3.0
    sd = s33 - sm * np.eye(3)
    seq = math.sqrt(1.5 * np.sum(sd * sd))
    return (seq / sM) ** 2 + 2 * q1 * fs * math.cosh(1.5 * q2 * sm / sM) - (1 + q3 * fs * fs)


def _normal_fd(s33, phi, h):
    """d phi / d sigma (symmetric) by central differences, one independent
    component at a time (an off-diagonal pair moves together: half the
    difference is each entry's derivative)."""
    N = np.zeros((3, 3))
    for a in range(3):
        for b in range(a, 3):
            E = np.zeros((3, 3))
            E[a, b] = E[b, a] = h
            d = (phi(s33 + E) - phi(s33 - E)) / (2 * h)
            N[a, b] = N[b, a] = d if a == b else 0.5 * d
    return N


def _gtn_growth_case(orc, J0, f, k_omega, fN=0.0, seed=11):
    """Inject a plastic trial state at high tensile mean stress, return the
    oracle's step and what the flow rule predicts for the void growth.

    The prediction uses only: the flow rule (plastic strain along d Phi /
    d sigma at the returned stress, eq. flow_rule, evaluated here by finite
    differences of eq. yield_GTN), the equivalent plastic strain increment
    from the stress drop (eq. delta_epsilon_p_eq) and the growth law
    f_dot = (1 - f) tr(eps_p_dot) + k_w f omega sigma_d : eps_p_dot / sigma_eq
    (eq. GTN_damage_growth), plus Chu-Needleman nucleation A_N d eps_M when
    F_N > 0.  Algorithm 2's last line (alpha, the factor 1 / (alpha sigma* + 1),
    sigma_M / sigma_y) is not used."""
    m = gtn_mat(n=0.26, k_omega=k_omega, fN=fN)
    q1, q2, q3 = m["q1"], m["q2"], m["q3"]
    fs = orc.fstar(m, f)
    assert fs == f                          # below f_c: f* = f in the flow rule too
    D = q1 * fs
    eps_n = 0.08
    sM0 = orc.flow_stress(m, eps_n)
    sm_tr = orc.mean_stress_eos(m, J0, D, 0.0, False)
    c = (1 + q3 * fs * fs) - 2 * q1 * fs * math.cosh(1.5 * q2 * sm_tr / sM0)
    assert c > 0.1
    rng = np.random.default_rng(seed)
    sd = rng.normal(size=(3, 3))
    sd = sd + sd.T
    sd -= np.trace(sd) / 3 * np.eye(3)
    seq_tr = 1.08 * sM0 * math.sqrt(c)       # 8 % outside the surface
    sd *= seq_tr / math.sqrt(1.5 * np.sum(sd * sd))
    pt = _inject_trial(orc, m, J0, sd, eps_n, f, D)
    dem = pt.eps_p - eps_n
    assert dem > 0
    s_out = full(pt.sig)
    sm_out = np.trace(s_out) / 3
    sd_out = s_out - sm_out * np.eye(3)
    seq_out = math.sqrt(1.5 * np.sum(sd_out * sd_out))
    sstar = sm_out / seq_out
    assert 0.8 < sstar < 2.5                # high triaxiality
    sM = orc.flow_stress(m, pt.eps_p)
    N = _normal_fd(s_out, lambda s: _gtn_phi(s, sM, fs, q1, q2, q3), 1e-6 * seq_out)
    Nd = N - np.trace(N) / 3 * np.eye(3)
    neq = math.sqrt(2.0 / 3.0 * np.sum(Nd * Nd))
    tr_ratio = np.trace(N) / neq             # tr(d eps_p) / d eps_p_eq
    shear_ratio = np.sum(sd_out * N) / (seq_out * neq)   # sigma_d : d eps_p / (sigma_eq d eps_p_eq)
    G = G_of(m)
    dep_eq = (seq_tr - seq_out) / (3 * G * (1 - D))
    detd = np.linalg.det(sd_out)
    om = 1.0 - (27.0 * detd / (2.0 * seq_out ** 3)) ** 2
    growth = ((1 - f) * tr_ratio + k_omega * f * om * shear_ratio) * dep_eq
    nucl = 0.0
    if fN > 0:
        z = (pt.eps_p - m["eN"]) / m["sN"]
        nucl = fN / (m["sN"] * math.sqrt(2 * math.pi)) * math.exp(-0.5 * z * z) * dem
    return pt.f_void - f, growth + nucl, tr_ratio, sstar


@pytest.mark.parametrize("J0,f", [(1.006, 0.02), (1.009, 0.05), (1.005, 0.1)])
def test_gtn_dilatational_void_growth_from_normality(orc, J0, f):
    """F_N = 0, k_w = 0: the void fraction grows by (1 - f) tr(d eps_p), with
    the trace from the normal to the yield surface and d eps_p_eq from the
    stress drop.  At these triaxialities the trace is a sizeable fraction of
    the equivalent increment, so a wrong factor in the ratio or in the
    work-equivalence conversion shows at once."""
    df, expect, tr_ratio, sstar = _gtn_growth_case(orc, J0, f, 0.0)
    assert tr_ratio * sstar > 0.05
    assert df > 0
    assert df == pytest.approx(expect, rel=1e-7)


@pytest.mark.parametrize("J0,f,fN", [(1.007, 0.04, 0.0), (1.006, 0.08, 0.0), (1.008, 0.06, 0.04)])
def test_gtn_void_growth_with_shear_and_nucleation(orc, J0, f, fN):
    """k_w = 3.5 on a non-axisymmetric deviator (omega > 0): the shear term
    k_w f omega sigma_d : d eps_p / sigma_eq adds to the dilatational one
    (eq. GTN_damage_growth, omega of eq. omega), and with F_N > 0 the
    nucleation A_N d eps_M at the step's end strain."""
    df, expect, _, _ = _gtn_growth_case(orc, J0, f, 3.5, fN=fN, seed=23)
    assert df == pytest.approx(expect, rel=1e-7)


def test_gtn_newton_converges_on_small_increments(orc):
    """Algorithm 2's second loop on the plastic increments of steady loading
    at rates from 1e-3 to 300 per second (increments down to about 1e-12 per
    step): every step must end by the loop's convergence test within a few
    iterations, not at the iteration cap.  (A stopping rule relative to the
    increment itself is not attainable in double for small increments: the
    residual's rounding scales with the trial stress, not with the
    increment.)"""
    m = I.material(0.125e-3, I.DMG_GTN, C=0.0)
    dt = m["dt"]
    for rate in np.geomspace(1e-3, 300.0, 25):
        pt = orc.Point(m, f_void=0.001, D=m["q1"] * 0.001)
        for _ in range(2600):                     # into the plastic range
            pt.update(np.diag([300.0, -90.0, 0.0]), dt)
        Fd = np.diag([rate, -0.3 * rate, 0.0])
        for _ in range(4):
            pt.update(Fd, dt)
            info = pt.info
            assert info.yielded == 1 and info.dep > 0.0, rate
            assert info.newton_failed == 0 and info.newton_e_iters <= 8, (
                rate, info.newton_e_iters, info.dep)
