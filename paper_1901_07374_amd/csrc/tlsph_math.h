// Device-side small-tensor helpers and the constitutive update of one
// particle (Secs. 4-5 of de Vaucorbeil & Hutchinson, arXiv:1901.07374).
// Tensors are row-major 3x3 (A_ab at 3a+b); symmetric ones in Voigt order
// (xx, yy, zz, yz, xz, xy).  R is the working precision of the bulk
// arithmetic (double for the FP64 form, float for the mixed form); the GTN
// return mapping and every accumulator are always double.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tlsph_internal.h"

namespace tlsph {

// Reciprocal for the constitutive update: on the device the hardware
// estimate refined by Newton-Raphson steps r <- r + r (1 - x r) (two for
// double, one for float), a few ulp from 1/x instead of the correctly
// rounded division sequence; on the host the plain division.  Where the
// estimate is 0 or infinite (x infinite or 0) it is already exact and the
// refinement (which would give NaN) is skipped.
__host__ __device__ __forceinline__ double rcp_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double r0 = __builtin_amdgcn_rcp(x);
    double r = fma(r0, fma(-x, r0, 1.0), r0);
    r = fma(r, fma(-x, r, 1.0), r);
    return (r0 == 0.0 || __builtin_isinf(r0)) ? r0 : r;
#else
    return 1.0 / x;
#endif
}
__host__ __device__ __forceinline__ float rcp_nr(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const float r0 = __builtin_amdgcn_rcpf(x);
    const float r = fmaf(r0, fmaf(-x, r0, 1.0f), r0);
    return (r0 == 0.0f || __builtin_isinf(r0)) ? r0 : r;
#else
    return 1.0f / x;
#endif
}

// x^y for x >= 0, y > 0 as exp(y log x): within a few ulp of pow for the
// exponents of the flow and failure laws (|y log x| of order 1), at a
// fraction of its cost.
__host__ __device__ __forceinline__ double pow_el(double x, double y) {
    return exp(y * log(x));
}

// The small-tensor products below spell out their fused multiply-adds (the
// library is compiled without contraction, so every variant rounds alike):
// ab - cd as fma(a, b, -(c d)), dot products as fma chains.
template <typename R>
__host__ __device__ __forceinline__ R mdiff(R a, R b, R c, R d) {
    return fma(a, b, -(c * d));
}

template <typename R>
__host__ __device__ __forceinline__ R dot3(R a0, R b0, R a1, R b1, R a2, R b2) {
    return fma(a0, b0, fma(a1, b1, a2 * b2));
}

template <typename R>
__host__ __device__ __forceinline__ R det33(const R a[9]) {
    return dot3(a[0], mdiff(a[4], a[8], a[5], a[7]), a[1], mdiff(a[5], a[6], a[3], a[8]),
                a[2], mdiff(a[3], a[7], a[4], a[6]));
}

// cofactor matrix cof(a) = det(a) a^-T (no division)
template <typename R>
__host__ __device__ __forceinline__ void cof33(const R a[9], R o[9]) {
    o[0] = mdiff(a[4], a[8], a[5], a[7]);
    o[1] = mdiff(a[5], a[6], a[3], a[8]);
    o[2] = mdiff(a[3], a[7], a[4], a[6]);
    o[3] = mdiff(a[2], a[7], a[1], a[8]);
    o[4] = mdiff(a[0], a[8], a[2], a[6]);
    o[5] = mdiff(a[1], a[6], a[0], a[7]);
    o[6] = mdiff(a[1], a[5], a[2], a[4]);
    o[7] = mdiff(a[2], a[3], a[0], a[5]);
    o[8] = mdiff(a[0], a[4], a[1], a[3]);
}

// adjugate / determinant
template <typename R>
__host__ __device__ __forceinline__ void inv33(const R a[9], R o[9]) {
    R c[9];
    cof33(a, c);
    const R inv = rcp_nr(dot3(a[0], c[0], a[1], c[1], a[2], c[2]));
    o[0] = c[0] * inv; o[1] = c[3] * inv; o[2] = c[6] * inv;
    o[3] = c[1] * inv; o[4] = c[4] * inv; o[5] = c[7] * inv;
    o[6] = c[2] * inv; o[7] = c[5] * inv; o[8] = c[8] * inv;
}

template <typename R>
__host__ __device__ __forceinline__ void mm33(const R a[9], const R b[9], R o[9]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            o[3 * i + j] = dot3(a[3 * i], b[j], a[3 * i + 1], b[3 + j], a[3 * i + 2], b[6 + j]);
}

// o = a b^T
template <typename R>
__host__ __device__ __forceinline__ void mmT33(const R a[9], const R b[9], R o[9]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            o[3 * i + j] = dot3(a[3 * i], b[3 * j], a[3 * i + 1], b[3 * j + 1], a[3 * i + 2],
                                b[3 * j + 2]);
}

template <typename R>
__host__ __device__ __forceinline__ void sym_from_voigt(const R s[6], R a[9]) {
    a[0] = s[0]; a[4] = s[1]; a[8] = s[2];
    a[5] = a[7] = s[3];
    a[2] = a[6] = s[4];
    a[1] = a[3] = s[5];
}

template <typename R>
__host__ __device__ __forceinline__ void voigt_from_sym(const R a[9], R s[6]) {
    s[0] = a[0]; s[1] = a[4]; s[2] = a[8];
    s[3] = R(0.5) * (a[5] + a[7]);
    s[4] = R(0.5) * (a[2] + a[6]);
    s[5] = R(0.5) * (a[1] + a[3]);
}

// sqrt(3/2 s:s) of a deviator held in Voigt form
template <typename R>
__host__ __device__ __forceinline__ R mises_voigt(const R s[6]) {
    return sqrt(R(1.5) * fma(R(2), dot3(s[3], s[3], s[4], s[4], s[5], s[5]),
                             dot3(s[0], s[0], s[1], s[1], s[2], s[2])));
}

// Cubic spline with compact support h (q = r/h < 1 for every listed pair):
// W = c (1 - 6q^2 + 6q^3) for q < 1/2, 2c (1-q)^3 beyond; c = 8 / (pi h^3).
template <typename R>
__host__ __device__ __forceinline__ void spline(R r, R inv_h, R wnorm, R& W, R& dW) {
    const R q = r * inv_h;
    const R a = R(1) - q;
    if (q < R(0.5)) {
        W = wnorm * fma(q * q, fma(R(6), q, R(-6)), R(1));
        dW = wnorm * inv_h * (q * fma(R(18), q, R(-12)));
    } else {
        W = wnorm * R(2) * a * a * a;
        dW = wnorm * inv_h * (R(-6) * a * a);
    }
}

// det(I + H) - 1 without forming I + H (keeps J - 1 accurate in float)
template <typename R>
__host__ __device__ __forceinline__ R det_ipH_m1(const R h[9]) {
    const R tr = h[0] + h[4] + h[8];
    const R m2 = mdiff(h[0], h[4], h[1], h[3]) + mdiff(h[0], h[8], h[2], h[6]) +
                 mdiff(h[4], h[8], h[5], h[7]);
    return tr + m2 + det33(h);
}

// Mie-Grueneisen (Sec. 4, eq. pH) as the pressure p (compression positive)
// written in mu = eta - 1; the mean stress is -p.
template <typename R>
__host__ __device__ __forceinline__ R mg_pressure(R pref, R c0, R S, R G0, R mu) {
    const R eta = R(1) + mu;
    const R den = eta - S * mu;
    return pref * c0 * c0 * mu * (eta - R(0.5) * G0 * mu) * rcp_nr(den * den);
}

// Mean stress from Jm1 = J - 1 (eta = 1/J).  Tension with damage uses
// rho0 (1 - D) and eta = (1 - D)/J (decided on the undamaged value) unless
// switched off.
template <typename R>
__host__ __device__ __forceinline__ R mean_stress(const DevSpec& P, R Jm1, R D, R e, bool damaged_branch) {
    const R rho0 = R(P.rho0), c0 = R(P.c0), S = R(P.S_alpha), G0 = R(P.Gamma0);
    const R J = R(1) + Jm1;
    const R eterm = G0 * rho0 * e;
    const R iJ = rcp_nr(J);
    R p = mg_pressure(rho0, c0, S, G0, -Jm1 * iJ) + eterm;
    if (damaged_branch && p < R(0))
        p = mg_pressure(rho0 * (R(1) - D), c0, S, G0, -(D + Jm1) * iJ) + eterm;
    return -p;
}

// Johnson-Cook flow stress, undamaged, isothermal; ln of the normalised rate
// floored at 0.
__host__ __device__ __forceinline__ double jc_rate_factor(const DevSpec& P, double rate) {
    const double rs = rate * P.inv_eps_dot0;
    return rs > 1.0 ? 1.0 + P.C * log(rs) : 1.0;
}

// A + B eps^n, the strain-hardening factor of the Johnson-Cook flow stress
// (A exactly while the point has not yielded)
__host__ __device__ __forceinline__ double jc_hardening(const DevSpec& P, double eps) {
    return eps > 0.0 ? P.A + P.B * pow_el(eps, P.n) : P.A;
}

// Strain-hardening factor h(eps) of the flow stress for the laws Sec. 4
// names: Johnson-Cook A + B eps^n, linear A + B eps, Swift B (e0 + eps)^n,
// Voce A + B (1 - exp(-beta eps)).  kFlow = false compiles Johnson-Cook only.
template <bool kFlow>
__host__ __device__ __forceinline__ double hardening(const DevSpec& P, double eps) {
    if constexpr (kFlow) {
        switch (P.flow) {
            case 1: return P.A + P.B * eps;
            case 2: return P.B * pow_el(P.flow_e0 + eps, P.n);
            case 3: return P.A - P.B * expm1(-P.flow_beta * eps);
            default: break;
        }
    }
    return jc_hardening(P, eps);
}

// dh/deps (the Johnson-Cook slope taken as 0 at eps = 0)
template <bool kFlow>
__host__ __device__ __forceinline__ double hardening_slope(const DevSpec& P, double eps) {
    if constexpr (kFlow) {
        switch (P.flow) {
            case 1: return P.B;
            case 2: return P.B * P.n * pow_el(P.flow_e0 + eps, P.n - 1.0);
            case 3: return P.B * P.flow_beta * exp(-P.flow_beta * eps);
            default: break;
        }
    }
    return eps > 0.0 ? P.B * P.n * pow_el(eps, P.n - 1.0) : 0.0;
}

// h(eps) and dh/deps together, each law's transcendental evaluated once
// (the Johnson-Cook slope taken as 0 at eps = 0)
__host__ __device__ __forceinline__ void hardening_and_slope(const DevSpec& P, double eps,
                                                             double& h, double& hp) {
    switch (P.flow) {
        case 1:
            h = P.A + P.B * eps;
            hp = P.B;
            return;
        case 2: {
            const double x = P.flow_e0 + eps, b = P.B * pow_el(x, P.n);
            h = b;
            hp = P.n * b * rcp_nr(x);
            return;
        }
        case 3: {
            const double em1 = expm1(-P.flow_beta * eps);
            h = P.A - P.B * em1;
            hp = P.B * P.flow_beta * (em1 + 1.0);
            return;
        }
        default: {
            if (eps > 0.0) {
                const double b = P.B * pow_el(eps, P.n);
                h = P.A + b;
                hp = P.n * b * rcp_nr(eps);
            } else {
                h = P.A;
                hp = 0.0;
            }
            return;
        }
    }
}

// Algorithm 1 with the flow stress at the end of the step: the plastic
// increment d solves seq - k3 d = omD sigma_f(eps + d, d / dt) (k3 = 3G(1 - D),
// omD = 1 - D).  The left side falls and the right side rises with d, so the
// root in [0, d_max] (d_max: the increment at the step's-start flow stress) is
// unique; Newton steps are kept inside the shrinking bracket (bisection when
// a step leaves it), at most P.newton_impl (100 by default) iterations.  The iteration ends on a Newton
// step below 1e-8 of d (Newton converges quadratically here, g being smooth
// with |g''| d of the order of |g'|, so the next correction would be below
// about 1e-16 d), on any step below 1e-14 of d or of seq / k3 (the increment
// that would unload the trial stress, which sets the rounding of g: a tiny
// d cannot be resolved to 1e-14 of itself), or on a bracket that narrow.
__host__ __device__ inline double implicit_increment(const DevSpec& P, double k3, double omD,
                                                     double seq, double eps, double d_max,
                                                     int32_t& flags) {
    double lo = 0.0, hi = d_max, d = d_max;
    for (int it = 0; it < P.newton_impl; ++it) {
        const double rs = d * P.inv_dt * P.inv_eps_dot0;
        const bool fast = rs > 1.0 && P.C != 0.0;
        const double rf = fast ? 1.0 + P.C * log(rs) : 1.0;
        double h, hp;
        hardening_and_slope(P, eps + d, h, hp);
        const double g = seq - k3 * d - omD * h * rf;
        if (g > 0.0) lo = d; else hi = d;
        const double drf = fast ? P.C * rcp_nr(d) : 0.0;
        const double dg = -k3 - omD * (hp * rf + h * drf);
        double nd = d - g * rcp_nr(dg);
        const bool newton = nd > lo && nd < hi;
        if (!newton) nd = 0.5 * (lo + hi);
        const double step = fabs(nd - d);
        d = nd;
        if ((newton && step <= 1e-8 * d) || step <= 1e-14 * d || step <= 1e-14 * seq / k3 ||
            hi - lo <= 1e-14 * hi)
            return d;
    }
    flags |= kErrNewton;
    return d;
}

// Largest eigenvalue of a symmetric tensor (closed form of the cubic's roots).
template <typename R>
__host__ __device__ __forceinline__ R max_principal(const R s[6]) {
    const R m = (s[0] + s[1] + s[2]) / R(3);
    const R b0 = s[0] - m, b1 = s[1] - m, b2 = s[2] - m;
    const R off = s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
    const R p = (b0 * b0 + b1 * b1 + b2 * b2 + R(2) * off) / R(6);
    if (!(p > R(0))) return m;
    const R detB = b0 * (b1 * b2 - s[3] * s[3]) - s[5] * (s[5] * b2 - s[3] * s[4]) +
                   s[4] * (s[5] * s[3] - b1 * s[4]);
    R rq = detB / (R(2) * p * sqrt(p));
    rq = rq < R(-1) ? R(-1) : (rq > R(1) ? R(1) : rq);
    const R phi = acos(rq) / R(3);
    return m + R(2) * sqrt(p) * cos(phi);
}

__host__ __device__ __forceinline__ double gtn_fstar(const DevSpec& P, double f) {
    if (f <= P.fc) return f;
    if (f < P.fF) return P.fc + (1.0 / P.q1 - P.fc) / (P.fF - P.fc) * (f - P.fc);
    return 1.0 / P.q1;
}

__host__ __device__ __forceinline__ double gtn_D(const DevSpec& P, double f) {
    if (f >= P.fF) return 1.0;
    const double d = P.q1 * gtn_fstar(P, f);
    return d < 1.0 ? d : 1.0;
}

// cosh y and sinh y from one exponential and its reciprocal (for the y of
// Algorithm 2, |y| well below 700)
__host__ __device__ __forceinline__ void cosh_sinh(double y, double& ch, double& sh) {
    const double e = exp(y), ie = rcp_nr(e);
    ch = 0.5 * (e + ie);
    sh = 0.5 * (e - ie);
}

// GTN return mapping (Algorithm 2), double precision.  In: trial deviator
// (Voigt) and trial mean stress, state (eps_M, its last rate, f), damage D.
// Out: returned deviator and mean stress, updated eps_M, rate, f.
template <bool kFlow>
__host__ __device__ inline void gtn_return(const DevSpec& P, double D, double dt, const double sdt[6],
                                  double smt, double& epsM, double& rate, double& f,
                                  double sd[6], double& sm, int32_t& flags) {
    const double seq = mises_voigt(sdt);
    const double rf = jc_rate_factor(P, rate);
    const double sM0 = hardening<kFlow>(P, epsM) * rf;
    const double fs = gtn_fstar(P, f);
    const double q1 = P.q1, q2 = P.q2, q3 = P.q3;
    bool plastic = false;
    double ss = 0.0;
    // (quotients as products with refined reciprocals, a few ulp from the
    // divisions, as elsewhere in the update)
    const double iseq = rcp_nr(seq), isM0 = rcp_nr(sM0);
    if (seq >= 1e-12 * sM0) {
        ss = smt * iseq;
        const double r = seq * isM0;
        const double a = 1.5 * q2 * ss * r;
        const double cst = 1.0 + q3 * fs * fs;
        // cosh a <= 1 + 0.6 a^2 for |a| <= 1: a trial state that this bound
        // already puts more than 1e-9 inside the yield surface is elastic
        // without the exponential (the exact test below would agree: its
        // rounding is far below the margin)
        const double bound = r * r + 2.0 * q1 * fs * (1.0 + 0.6 * a * a) - cst;
        if (!(fabs(a) <= 1.0 && bound < -1e-9)) {
            const double phi = r * r + 2.0 * q1 * fs * cosh(a) - cst;
            plastic = !(phi < 0.0);
        }
    }
    if (!plastic) {
#pragma unroll
        for (int k = 0; k < 6; ++k) sd[k] = sdt[k];
        sm = smt;
        rate = 0.0;
        return;
    }
    // yield ratio x = sigma_y / sigma_M: Newton from above on the convex,
    // increasing yield function
    double x = seq * isM0 < 1.0 ? seq * isM0 : 1.0;
    const double kx = 1.5 * q2 * ss;
    const double cst = 1.0 + q3 * fs * fs;
    const int cap = P.newton_gtn;
    int it = 0;
    for (; it < cap; ++it) {
        double ch, sh;
        cosh_sinh(kx * x, ch, sh);
        const double dx = -(x * x + 2.0 * q1 * fs * ch - cst) *
                          rcp_nr(2.0 * x + 3.0 * q1 * q2 * fs * ss * sh);
        x += dx;
        if (fabs(dx) <= 1e-14) break;
    }
    if (it == cap) flags |= kErrNewton;
    // matrix plastic strain increment: d = c (seq - x sigma_f(eps_M + d))
    double chx, shx;
    cosh_sinh(kx * x, chx, shx);
    const double c = (x + 1.5 * q1 * q2 * f * ss * shx) * rcp_nr(3.0 * P.G * (1.0 - D) * (1.0 - f));
    double dem = c * (seq - x * sM0);
    for (it = 0; it < cap; ++it) {
        const double e1 = epsM + dem;
        double h1, hp1;   // the hardening factor and its slope, one transcendental
        if constexpr (kFlow) {
            hardening_and_slope(P, e1, h1, hp1);
        } else if (e1 > 0.0) {
            const double b = P.B * pow_el(e1, P.n);
            h1 = P.A + b;
            hp1 = P.n * b * rcp_nr(e1);
        } else {
            h1 = P.A;
            hp1 = 0.0;
        }
        const double hard = hp1 * rf;
        const double sf = h1 * rf;
        const double g = dem - c * (seq - x * sf);
        double nx = dem - g * rcp_nr(1.0 + c * x * hard);
        if (nx < 0.0) nx = 0.5 * dem;
        const double stp = nx - dem;
        dem = nx;
        // converged once the correction is below 1e-14 of c seq, the
        // increment that would unload the trial stress (the rounding of g
        // scales with it; relative to a tiny dem itself the loop would stall)
        if (fabs(stp) <= 1e-14 * c * seq) break;
    }
    if (it == cap) flags |= kErrNewton;
    epsM += dem;
    const double sM = hardening<kFlow>(P, epsM) * rf;
    const double sy = x * sM;
    const double scale = sy * iseq;
#pragma unroll
    for (int k = 0; k < 6; ++k) sd[k] = scale * sdt[k];
    // mean stress returned at constant triaxiality
    sm = smt - ss * (seq - sy);
    const double sMy = sM * rcp_nr(sy);   // sigma_M / sigma_y
    const double alpha = 1.5 * sMy * q1 * q2 * f * shx;
    // omega of the returned stress: 1 - (27 det(s_d) / (2 s_eq^3))^2
    const double detd = sd[0] * (sd[1] * sd[2] - sd[3] * sd[3]) -
                        sd[5] * (sd[5] * sd[2] - sd[3] * sd[4]) +
                        sd[4] * (sd[5] * sd[3] - sd[1] * sd[4]);
    double om = 0.0;
    if (sy > 0.0) {
        const double xi = 13.5 * detd * rcp_nr(sy * sy * sy);
        om = 1.0 - xi * xi;
        om = om < 0.0 ? 0.0 : (om > 1.0 ? 1.0 : om);
    }
    const double isN = rcp_nr(P.sN);
    const double z = (epsM - P.eN) * isN;
    const double AN = P.fN * isN * 0.3989422804014327 * exp(-0.5 * z * z);   // 1/sqrt(2 pi)
    f = f + AN * dem +
        (1.0 - f) * rcp_nr(alpha * ss + 1.0) * sMy * (alpha * (1.0 - f) + f * P.k_omega * om) * dem;
    rate = dem * rcp_nr(dt);
}

// Result of the constitutive update of one particle.
template <typename R>
struct PointOut {
    R H[9];      // F^{n+1} - I
    R sig[6];    // Cauchy stress (Voigt)
    R P[9];      // first Piola-Kirchhoff stress
    double D;    // D^{n+1}
};

// Constitutive and damage update of one particle over one step (Secs. 4-5).
// In: Hn = F^n - I, Fd = dF/dt, sn = sigma^n (Voigt).  Kinematics from dF/dt
// and the midpoint F, Hughes-Winget rotation of the deviator, Mie-Grueneisen
// mean stress, Johnson-Cook radial return (Algorithm 1) or GTN (Algorithm 2),
// Cockcroft-Latham / Johnson-Cook initiation and evolution (Secs. 5.1-5.3),
// failed particles stress free, energy by the trapezoid rule on P,
// P = J sigma F^-T.
// DM >= 0 fixes the damage model at compile time (the other models' code is
// dropped); DM = -1 reads it from the specimen.  kFlow = false compiles the
// Johnson-Cook law with Algorithm 1's explicit hardening only; true reads the
// law and the return from the specimen.
template <typename R, int DM = -1, bool kFlow = true>
__host__ __device__ __forceinline__ void point_update(const DevSpec& P, const R Hn[9], const R Fd[9],
                                             const R sn[6], double& eps, double& rate,
                                             double& dinit, double& wp, double& fv, double& e,
                                             double D, PointOut<R>& o, int32_t& flags) {
    const int model = DM >= 0 ? DM : P.damage;
    // kFlow: the other hardening laws and the implicit return are compiled in
    const R dt = R(P.dt);
#pragma unroll
    for (int k = 0; k < 9; ++k) o.H[k] = fma(dt, Fd[k], Hn[k]);
    if (D >= 1.0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) o.sig[k] = R(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) o.P[k] = R(0);
        o.D = 1.0;
        return;
    }
    // energy per unit mass by the trapezoid rule, dF/dt : (P^n + P^{n+1}) / 2 / rho0:
    // the P^n half now, so F^n and sigma^n need not stay live to the end
    // (P = J sigma F^-T = sigma cof(F))
    R work0 = R(0);
    {
        R S0[9], F0[9], C0[9], P0[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) F0[k] = Hn[k];
        F0[0] += R(1); F0[4] += R(1); F0[8] += R(1);
        sym_from_voigt(sn, S0);
        cof33(F0, C0);
        mm33(S0, C0, P0);
#pragma unroll
        for (int k = 0; k < 9; ++k) work0 = fma(Fd[k], P0[k], work0);
    }
    R Fb[9], Fbi[9], l[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Fb[k] = R(0.5) * (Hn[k] + o.H[k]);
    Fb[0] += R(1); Fb[4] += R(1); Fb[8] += R(1);
    inv33(Fb, Fbi);
    mm33(Fd, Fbi, l);
    const R Jm1 = det_ipH_m1(o.H);
    // rate of deformation (Voigt) and spin
    R d6[6] = {l[0], l[4], l[8], R(0.5) * (l[5] + l[7]), R(0.5) * (l[2] + l[6]),
               R(0.5) * (l[1] + l[3])};
    const R w01 = R(0.5) * (l[1] - l[3]), w02 = R(0.5) * (l[2] - l[6]), w12 = R(0.5) * (l[5] - l[7]);
    // stored deviator, rotated by R = (I - dt/2 w)^-1 (I + dt/2 w)
    const R third = R(1.0 / 3.0);
    const R smn = (sn[0] + sn[1] + sn[2]) * third;
    R Sd[9], sdr[6];
    {
        R s6[6] = {sn[0] - smn, sn[1] - smn, sn[2] - smn, sn[3], sn[4], sn[5]};
        sym_from_voigt(s6, Sd);
    }
    {
        // R = (I - A)^-1 (I + A) for the skew A = dt/2 w, in closed form:
        // with a the axial vector of A (A x = a x x),
        // R = ((1 - a.a) I + 2 A + 2 a a^T) / (1 + a.a)
        const R hd = R(0.5) * dt;
        const R a1 = -hd * w12, a2 = hd * w02, a3 = -hd * w01;
        const R aa = a1 * a1 + a2 * a2 + a3 * a3;
        const R c = rcp_nr(R(1) + aa);
        const R d0 = (R(1) - aa) * c, t2 = R(2) * c;
        const R Rm[9] = {fma(t2 * a1, a1, d0), t2 * fma(a1, a2, -a3), t2 * fma(a1, a3, a2),
                         t2 * fma(a2, a1, a3), fma(t2 * a2, a2, d0), t2 * fma(a2, a3, -a1),
                         t2 * fma(a3, a1, -a2), t2 * fma(a3, a2, a1), fma(t2 * a3, a3, d0)};
        // R S R^T is symmetric: its upper triangle, in Voigt order
        R T[9];
        mm33(Rm, Sd, T);
        constexpr int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            sdr[k] = dot3(T[3 * vi[k]], Rm[3 * vj[k]], T[3 * vi[k] + 1], Rm[3 * vj[k] + 1],
                          T[3 * vi[k] + 2], Rm[3 * vj[k] + 2]);
    }
    // deviatoric strain increment
    const R trd = (d6[0] + d6[1] + d6[2]) * third;
    const R de[6] = {(d6[0] - trd) * dt, (d6[1] - trd) * dt, (d6[2] - trd) * dt,
                     d6[3] * dt, d6[4] * dt, d6[5] * dt};
    const R G = R(P.G);
    const R omD = R(1.0 - D);
    R sd[6], sm;
    double Dn = D;
    if (model == 3) {
        double sdt[6], sdo[6], smo;
#pragma unroll
        for (int k = 0; k < 6; ++k) sdt[k] = double(fma(R(2) * G * omD, de[k], sdr[k]));
        const double smt = double(mean_stress<R>(P, Jm1, R(D), R(e), false));
        gtn_return<kFlow>(P, D, P.dt, sdt, smt, eps, rate, fv, sdo, smo, flags);
#pragma unroll
        for (int k = 0; k < 6; ++k) sd[k] = R(sdo[k]);
        sm = R(smo);
        Dn = gtn_D(P, fv);
    } else {
        sm = mean_stress<R>(P, Jm1, R(D), R(e), true);
        // The trial deviator is formed in the working precision; the radial
        // return from it (the overstress sigma_eq - sigma_f, whose
        // cancellation sets the plastic increment, and the scale factor) and
        // the damage inputs (triaxiality, largest principal stress) are
        // double in both forms: per particle, and what they feed accumulates
        // in double.
        R st[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) st[k] = fma(R(2) * G * omD, de[k], sdr[k]);
        // elastic if sigma_eq < sigma_f, decided on the squares (no root)
        const double t0 = st[0], t1 = st[1], t2 = st[2], t3 = st[3], t4 = st[4], t5 = st[5];
        const double q2 = 1.5 * fma(2.0, dot3(t3, t3, t4, t4, t5, t5), dot3(t0, t0, t1, t1, t2, t2));
        const bool impl = kFlow && P.implicit_return;
        const double h0 = hardening<kFlow>(P, eps);
        const double omDd = 1.0 - D;
        const double sf = h0 * (impl ? 1.0 : jc_rate_factor(P, rate)) * omDd;
        double depd = 0.0;
        double sret = sf;   // equivalent stress after the return
        double sc = 1.0;    // its ratio to the trial value
        if (q2 >= sf * sf) {
            const double seq = sqrt(q2);
            if (impl) {
                const double k3 = 3.0 * P.G * omDd;
                depd = implicit_increment(P, k3, omDd, seq, eps, (seq - omDd * h0) / k3, flags);
                sret = seq - k3 * depd;
            } else {
                depd = (seq - sf) * rcp_nr(3.0 * P.G * omDd);
            }
            sc = sret * rcp_nr(seq);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) sd[k] = R(sc * double(st[k]));
        eps += depd;
        rate = depd * P.inv_dt;
        if (depd > 0.0 && (model == 1 || model == 2)) {
            if (model == 2) {
                // the returned deviator lies on the yield surface: its
                // equivalent stress is sret
                const double sstar = double(sm) * rcp_nr(sret);
                const double ef = (P.D1 + P.D2 * exp(P.D3 * sstar)) *
                                  pow_el(1.0 + rate * P.inv_eps_dot0, P.D4);
                dinit += depd * rcp_nr(ef);
            } else {
                const double smd = double(sm);
                double full6[6] = {sc * double(st[0]) + smd, sc * double(st[1]) + smd,
                                   sc * double(st[2]) + smd, sc * double(st[3]),
                                   sc * double(st[4]), sc * double(st[5])};
                const double s1 = max_principal(full6);
                wp += (s1 > 0.0 ? s1 : 0.0) * depd;
                dinit = wp / P.Wcr;
            }
            double dn = 10.0 * (dinit - 1.0);
            Dn = dn < 0.0 ? 0.0 : (dn > 1.0 ? 1.0 : dn);
        }
    }
    o.D = Dn;
    if (Dn >= 1.0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) o.sig[k] = R(0);
    } else {
        o.sig[0] = sd[0] + sm; o.sig[1] = sd[1] + sm; o.sig[2] = sd[2] + sm;
        o.sig[3] = sd[3]; o.sig[4] = sd[4]; o.sig[5] = sd[5];
    }
    // P^{n+1} = J sigma F^{-T} = sigma cof(F)
    R S1[9], F1[9], C1[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) F1[k] = o.H[k];
    F1[0] += R(1); F1[4] += R(1); F1[8] += R(1);
    sym_from_voigt(o.sig, S1);
    cof33(F1, C1);
    mm33(S1, C1, o.P);
    // the P^{n+1} half of the energy update
    R work1 = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) work1 = fma(Fd[k], o.P[k], work1);
    e += double(P.dt) * double(R(0.5) * (work0 + work1)) * P.inv_rho0;
}

}  // namespace tlsph
