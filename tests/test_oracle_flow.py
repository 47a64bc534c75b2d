"""Oracle pins for the flow laws Sec. 4 names besides Johnson-Cook (linear
plastic, Swift, Voce) and for the implicit radial return (the consistency
condition solved with the flow stress at the end of the step).  The laws are
pinned against each other where one reduces to another, the return against
closed forms and against a bracketing root finder on its defining equation,
and against the GTN return of Algorithm 2, an independent Newton solver,
which without voids must give the same point.  Also the factors of a
constant homologous temperature (flow stress and JC failure strain) against
their closed forms.  Host only."""
import math

import numpy as np
import pytest
from scipy import optimize

from paper_1901_07374_amd import inputs as I


def mat(flow, implicit=1, **over):
    base = dict(flow=flow, implicit_return=implicit, S_alpha=0.0, Gamma0=0.0, C=0.0)
    if flow == I.FLOW_SWIFT:
        base.update(B=1100e6, n=0.2, flow_e0=0.002)
    if flow == I.FLOW_VOCE:
        base.update(A=700e6, B=450e6, flow_beta=12.0)
    if flow == I.FLOW_LINEAR:
        base.update(A=792e6, B=2.0e9)
    base.update(over)
    return I.material(1e-3, I.DMG_NONE, **base)


def G_of(m):
    return m["E"] / (2 * (1 + m["nu"]))


def vm(s6):
    s = np.asarray(s6, float)
    d = s[:3] - s[:3].mean()
    return math.sqrt(1.5 * (d @ d + 2 * (s[3:] @ s[3:])))


def voigt(a):
    return np.array([a[0, 0], a[1, 1], a[2, 2], a[1, 2], a[0, 2], a[0, 1]])


SHAPE = np.array([[1.0, 0.3, 0.0], [0.3, -0.4, 0.2], [0.0, 0.2, -0.6]])
SHAPE = SHAPE / math.sqrt(1.5 * np.sum(SHAPE * SHAPE))   # unit von Mises deviator


def trial(orc, m, seq, eps, D=0.0, f=None):
    """One update whose trial deviator is seq * SHAPE (dF/dt = 0, F = I)."""
    init = dict(sig=voigt(seq * SHAPE), eps_p=eps, D=D)
    if f is not None:
        init["f_void"] = f
    pt = orc.Point(m, **init)
    pt.update(np.zeros(9))
    return pt


# --------------------------------------------------------------------------
# the laws against each other
# --------------------------------------------------------------------------
@pytest.mark.parametrize("eps", [0.0, 1e-4, 0.01, 0.3, 2.0])
def test_laws_reduce_to_linear(orc, eps):
    lin = mat(I.FLOW_LINEAR, A=500e6, B=800e6)
    # Swift with n = 1: B (e0 + eps) is linear with A = B e0
    sw = mat(I.FLOW_SWIFT, B=800e6, n=1.0, flow_e0=0.625)
    assert orc.flow_stress(sw, eps) == pytest.approx(orc.flow_stress(lin, eps), rel=1e-15)
    # Johnson-Cook with n = 1
    jc = mat(I.FLOW_JC, A=500e6, B=800e6, n=1.0)
    assert orc.flow_stress(jc, eps) == pytest.approx(orc.flow_stress(lin, eps), rel=1e-15)
    # Voce for beta eps << 1 is linear with slope B beta, to O((beta eps)^2)
    beta = 1e-6
    vo = mat(I.FLOW_VOCE, A=500e6, B=800e6 / beta, flow_beta=beta)
    err = 0.5 * 800e6 * beta * eps * eps
    assert abs(orc.flow_stress(vo, eps) - orc.flow_stress(lin, eps)) <= 1.01 * err + 1e-6


def test_voce_saturates(orc):
    vo = mat(I.FLOW_VOCE)
    assert orc.flow_stress(vo, 0.0) == vo["A"]
    assert orc.flow_stress(vo, 60.0 / vo["flow_beta"]) == pytest.approx(vo["A"] + vo["B"],
                                                                        rel=1e-15)


@pytest.mark.parametrize("flow", [I.FLOW_JC, I.FLOW_LINEAR, I.FLOW_SWIFT, I.FLOW_VOCE])
def test_rate_factor_is_common(orc, flow):
    m = mat(flow, C=0.02)
    for eps in (0.0, 0.05, 0.4):
        base = orc.flow_stress(m, eps, 0.0)
        assert orc.flow_stress(m, eps, 0.5) == base           # below the reference rate
        assert orc.flow_stress(m, eps, 300.0) == pytest.approx(base * (1 + 0.02 * math.log(300)),
                                                               rel=1e-14)


# --------------------------------------------------------------------------
# the implicit return
# --------------------------------------------------------------------------
@pytest.mark.parametrize("D", [0.0, 0.25])
def test_implicit_linear_hardening_closed_form(orc, D):
    m = mat(I.FLOW_LINEAR)
    G, H, A = G_of(m), m["B"], m["A"]
    eps_n = 0.03
    sy0 = (1 - D) * (A + H * eps_n)
    for over in (1.0001, 1.2, 3.0):
        pt = trial(orc, m, over * sy0, eps_n, D)
        # textbook: d = (seq_tr - (1 - D) sigma_y(eps_n)) / ((1 - D)(3G + H))
        d = (over * sy0 - sy0) / ((1 - D) * (3 * G + H))
        assert pt.eps_p - eps_n == pytest.approx(d, rel=1e-11)
        assert vm(pt.sig) == pytest.approx((1 - D) * (A + H * pt.eps_p), rel=1e-13)
        # radial: the deviator keeps its direction
        s = pt.sig
        dev = np.array([s[0], s[1], s[2]]) - s[:3].mean()
        assert dev / vm(s) == pytest.approx(np.diag(SHAPE), abs=1e-12)


def _h(m, e):
    f = m["flow"]
    if f == I.FLOW_LINEAR:
        return m["A"] + m["B"] * e
    if f == I.FLOW_SWIFT:
        return m["B"] * (m["flow_e0"] + e) ** m["n"]
    if f == I.FLOW_VOCE:
        return m["A"] + m["B"] * (1 - math.exp(-m["flow_beta"] * e))
    return m["A"] + m["B"] * e ** m["n"]


@pytest.mark.parametrize("flow,C", [(I.FLOW_SWIFT, 0.0), (I.FLOW_VOCE, 0.0), (I.FLOW_JC, 0.0),
                                    (I.FLOW_JC, 0.014), (I.FLOW_VOCE, 0.03)])
def test_implicit_increment_solves_consistency(orc, flow, C):
    m = mat(flow, C=C)
    G, dt = G_of(m), m["dt"]
    for eps_n, D, over in ((0.0, 0.0, 1.5), (0.02, 0.0, 1.01), (0.2, 0.4, 2.0), (1.0, 0.1, 1.3)):
        sy0 = (1 - D) * _h(m, eps_n)

        def g(d):
            rs = max(d / dt / m["eps_dot0"], 1.0)
            return over * sy0 - 3 * G * (1 - D) * d - (1 - D) * _h(m, eps_n + d) * (
                1 + C * math.log(rs))

        dmax = (over - 1) * sy0 / (3 * G * (1 - D))
        d = optimize.brentq(g, 0.0, dmax, xtol=1e-300, rtol=1e-15, maxiter=500)
        pt = trial(orc, m, over * sy0, eps_n, D)
        assert pt.eps_p - eps_n == pytest.approx(d, rel=1e-10)
        assert pt.eps_p_rate == pytest.approx(d / dt, rel=1e-10)
        assert vm(pt.sig) == pytest.approx(over * sy0 - 3 * G * (1 - D) * d, rel=1e-12)


@pytest.mark.parametrize("flow", [I.FLOW_JC, I.FLOW_LINEAR, I.FLOW_SWIFT, I.FLOW_VOCE])
def test_implicit_elastic_below_surface(orc, flow):
    m = mat(flow, C=0.02)
    for eps_n in (0.0, 0.1):
        sy0 = _h(m, eps_n)
        pt = trial(orc, m, 0.999 * sy0, eps_n)
        assert pt.eps_p == eps_n and pt.eps_p_rate == 0.0
        assert vm(pt.sig) == pytest.approx(0.999 * sy0, rel=1e-13)


def test_perfect_plasticity_implicit_equals_explicit(orc):
    for over in (1.001, 1.5):
        a = trial(orc, mat(I.FLOW_LINEAR, B=0.0, implicit=1), over * 792e6, 0.05, 0.2)
        b = trial(orc, mat(I.FLOW_LINEAR, B=0.0, implicit=0), over * 792e6, 0.05, 0.2)
        assert a.eps_p == pytest.approx(b.eps_p, rel=1e-14)
        assert np.allclose(a.sig, b.sig, rtol=1e-14, atol=0)


@pytest.mark.parametrize("flow", [I.FLOW_LINEAR, I.FLOW_SWIFT, I.FLOW_VOCE, I.FLOW_JC])
def test_implicit_stays_on_surface_along_a_path(orc, flow):
    # isochoric stretching: every yielding step ends on the surface of the
    # step's end, sigma_eq = sigma_f(eps_p^{n+1}) (explicit: of its start)
    m = mat(flow)
    pt = orc.Point(m)
    rate, dt = 20.0, 1e-6
    plastic = 0
    for k in range(800):
        a = rate
        Fd = np.diag([a, -0.5 * a, -0.5 * a]) * pt.F.reshape(3, 3).diagonal()
        e0 = pt.eps_p
        pt.update(np.diag(Fd.diagonal()), dt)
        if pt.eps_p > e0:
            plastic += 1
            assert vm(pt.sig) == pytest.approx(_h(m, pt.eps_p), rel=1e-11)
    assert plastic > 100


@pytest.mark.parametrize("flow", [I.FLOW_LINEAR, I.FLOW_SWIFT, I.FLOW_VOCE, I.FLOW_JC])
def test_gtn_without_voids_is_the_implicit_return(orc, flow):
    # Algorithm 2 with f = f0 = F_N = 0 is von Mises plasticity with the flow
    # stress at the end of the step: the same point as the implicit Alg. 1
    # (rate independent: Algorithm 2 takes the rate factor of the step's start)
    gt = mat(flow)
    gt.update(damage=I.DMG_GTN, q1=1.5, q2=1.0, q3=2.25, f0=0.0, fN=0.0, eN=0.3, sN=0.1,
              fc=0.15, fF=0.25, k_omega=0.0)
    a1 = mat(flow)
    for eps_n, over in ((0.0, 1.2), (0.1, 1.05), (0.5, 2.5)):
        sy0 = _h(a1, eps_n)
        pg = trial(orc, gt, over * sy0, eps_n, 0.0, f=0.0)
        pa = trial(orc, a1, over * sy0, eps_n)
        assert pg.eps_p == pytest.approx(pa.eps_p, rel=1e-11)
        assert vm(pg.sig) == pytest.approx(vm(pa.sig), rel=1e-11)


# --------------------------------------------------------------------------
# a constant homologous temperature (eq. JC_viscoplastic_model, Sec. 5.2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("flow", [I.FLOW_JC, I.FLOW_LINEAR, I.FLOW_SWIFT, I.FLOW_VOCE])
def test_thermal_softening_factor(orc, flow):
    # sigma_f carries 1 - T*^m for every law, at every strain and rate
    for Ts, m_exp in ((0.25, 0.8), (0.6, 1.7)):
        hot = mat(flow, C=0.02, T_star=Ts, m=m_exp)
        cold = mat(flow, C=0.02)
        theta = 1.0 - math.pow(Ts, m_exp)
        for eps in (0.0, 0.05, 0.4):
            for rate in (0.0, 300.0):
                assert orc.flow_stress(hot, eps, rate) == pytest.approx(
                    theta * orc.flow_stress(cold, eps, rate), rel=1e-15)
    # T* = 0 is isothermal whatever the exponent (no 0^0)
    for m_exp in (0.0, 1.0, 2.5):
        z = mat(flow, T_star=0.0, m=m_exp)
        assert orc.flow_stress(z, 0.1, 10.0) == orc.flow_stress(mat(flow), 0.1, 10.0)


def test_thermal_factor_of_the_failure_strain(orc):
    # Johnson-Cook failure strain times 1 + D5 T*: with the flow stress held
    # equal (A scaled by 1 - T*^m at T* = 0), the same plastic increment
    # raises D_init by 1 / (1 + D5 T*) times as much
    Ts, m_exp = 0.3, 1.2
    theta = 1.0 - math.pow(Ts, m_exp)
    jc = dict(damage=I.DMG_JC, D1=0.05, D2=3.44, D3=-2.12, D4=0.002, D5=0.61)
    hot = dict(mat(I.FLOW_LINEAR, implicit=0, A=792e6, B=0.0, T_star=Ts, m=m_exp), **jc)
    cold = dict(mat(I.FLOW_LINEAR, implicit=0, A=792e6 * theta, B=0.0), **jc)
    seq = 1.4 * 792e6 * theta
    a = trial(orc, hot, seq, 0.1, 0.0)
    b = trial(orc, cold, seq, 0.1, 0.0)
    assert a.eps_p == b.eps_p and a.eps_p > 0.1
    assert np.array_equal(a.sig, b.sig)
    assert a.d_init * (1.0 + 0.61 * Ts) == pytest.approx(b.d_init, rel=1e-14)
