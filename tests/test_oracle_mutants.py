"""The oracle's pins must catch plausible mistakes.

Each case below plants one mistake in a copy of oracle/tlsph_oracle.c (a
dropped term, a wrong sign, factor or index, a transposed operand), builds
it, and runs the CPU pin tests against it in a child process: at least one
pin must fail.  The planted copies live in a temporary directory; the
oracle itself is never modified."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tlsph_oracle.c")
PINS = ["tests/test_oracle_kernel_neighbors.py", "tests/test_oracle_constitutive.py",
        "tests/test_oracle_flow.py", "tests/test_oracle_viscosity.py",
        "tests/test_oracle_graded.py", "tests/test_oracle_contact.py",
        "tests/test_oracle_system.py"]

# (name, text in the oracle, planted replacement)
MUTANTS = [
    ("kernel normalisation", "double c = 8.0 / (M_PI * h * h * h);",
     "double c = 6.0 / (M_PI * h * h * h);"),
    ("kernel slope term", "*dWdr = c / h * (-12.0 * q + 18.0 * q * q);",
     "*dWdr = c / h * (-12.0 * q + 16.0 * q * q);"),
    ("correction matrix without V_j", "Li[3 * a + b] += p->V0[j] * Xij[a] * g[b];",
     "Li[3 * a + b] += Xij[a] * g[b];"),
    ("dF/dt weighted by D_i", "double wgt = p->V0[j] * (1.0 - s->D[j]);",
     "double wgt = p->V0[j] * (1.0 - s->D[i]);"),
    ("nodal force damage weights swapped",
     "acc += ((1.0 - Dj) * Qi[3 * a + b] + (1.0 - Di) * Qj[3 * a + b]) * g[b];",
     "acc += ((1.0 - Di) * Qi[3 * a + b] + (1.0 - Dj) * Qj[3 * a + b]) * g[b];"),
    ("nodal force drops Q_j", "acc += ((1.0 - Dj) * Qi[3 * a + b] + (1.0 - Di) * Qj[3 * a + b]) * g[b];",
     "acc += ((1.0 - Dj) * Qi[3 * a + b]) * g[b];"),
    ("hourglass sign", "double coef = -m->hg_alpha", "double coef = m->hg_alpha"),
    ("hourglass with F_j transposed", "0.5 * (Fi[3 * a + b] + Fj[3 * a + b]) * Xij[b]",
     "0.5 * (Fi[3 * a + b] + Fj[3 * b + a]) * Xij[b]"),
    ("half drift", "for (int a = 0; a < 3; ++a) u[a] += dt * v[a];",
     "for (int a = 0; a < 3; ++a) u[a] += 0.5 * dt * v[a];"),
    ("failed particles keep moving", "if (s->D[i] >= 1.0) v[0] = v[1] = v[2] = 0.0;",
     "if (s->D[i] > 1.0) v[0] = v[1] = v[2] = 0.0;"),
    ("EOS S_alpha sign", "double den = eta - S * mu;", "double den = eta + S * mu;"),
    ("radial return with 2G", "double k3 = 3.0 * G * (1.0 - D);",
     "double k3 = 2.0 * G * (1.0 - D);"),
    ("trial stress without (1 - D)",
     "for (int k = 0; k < 9; ++k) sd_tr[k] = sd_rot[k] + 2.0 * G * (1.0 - D) * deps_d[k];",
     "for (int k = 0; k < 9; ++k) sd_tr[k] = sd_rot[k] + 2.0 * G * deps_d[k];"),
    ("rotation applied transposed", "mul3(R, sd_in, tmp);\n    mul3(tmp, RT, sd_out);",
     "mul3(RT, sd_in, tmp);\n    mul3(tmp, R, sd_out);"),
    ("JC failure strain sign of D3", "exp(m->D3 * sstar)", "exp(-m->D3 * sstar)"),
    ("flow stress rate term", "return 1.0 + m->C * log(rs);", "return 1.0 + m->C * log(rs + 1.0);"),
    ("GTN yield function factor", "cosh(1.5 * m->q2 * sstar * r)", "cosh(1.0 * m->q2 * sstar * r)"),
    ("Voce law sign", "return m->A - m->B * expm1(-m->flow_beta * eps);",
     "return m->A + m->B * expm1(-m->flow_beta * eps);"),
    ("Swift offset dropped", "return m->B * pow(m->flow_e0 + eps, m->n);",
     "return m->B * pow(eps, m->n);"),
    ("implicit return without (1 - D) on the flow stress",
     "double g = seq_tr - k3 * d - omD * h * rf;", "double g = seq_tr - k3 * d - h * rf;"),
    ("implicit return with the rate of the step's start", "double rate = d / dt;",
     "double rate = 0.0 * d / dt;"),
    ("viscosity on separating pairs", "if (vx < 0.0) {", "if (vx > 0.0) {"),
    ("viscosity quadratic term linear", "m->av_q2 * mu * mu) / m->rho0;",
     "m->av_q2 * mu) / m->rho0;"),
    ("viscosity applied with the wrong sign",
     "for (int a = 0; a < 3; ++a) fv[a] += mm * Pi * g[a];",
     "for (int a = 0; a < 3; ++a) fv[a] -= mm * Pi * g[a];"),
    ("viscosity not in the next kick",
     "s->force[3 * i + a] = fi[a] + fhg[a] + s->fvisc[3 * i + a];",
     "s->force[3 * i + a] = fi[a] + fhg[a];"),
    ("pair kernel with the particle's own support",
     "return p->hs ? 0.5 * (p->hs[i] + p->hs[j]) : p->mat[p->spec[i]].h;",
     "return p->hs ? p->hs[i] : p->mat[p->spec[i]].h;"),
    ("neighbour rule with the larger support", "double hij = 0.5 * (hs[i] + hs[j]);",
     "double hij = hs[i] > hs[j] ? hs[i] : hs[j];"),
    ("contact force linear in the overlap", "delta * sqrt(delta);", "delta;"),
    ("contact ignores failure", "if (p->spec[i] == p->spec[j] && s->D[i] < 1.0 && s->D[j] < 1.0 &&",
     "if (p->spec[i] == p->spec[j] &&"),
    ("contact attractive", "for (int a = 0; a < 3; ++a) f[a] -= F * d[a] / r;",
     "for (int a = 0; a < 3; ++a) f[a] += F * d[a] / r;"),
    ("energy from P^{n+1} only", "work += Fdot[k] * 0.5 * (Jn * Pn[k] + P[k]);",
     "work += Fdot[k] * P[k];"),
    ("thermal factor without its exponent",
     "return m->T_star > 0.0 ? 1.0 - pow(m->T_star, m->m) : 1.0;",
     "return m->T_star > 0.0 ? 1.0 - m->T_star : 1.0;"),
    ("failure strain temperature factor sign", "(1.0 + m->D5 * Tstar);", "(1.0 - m->D5 * Tstar);"),
    ("GTN void growth ratio without its 3/2",
     "double alpha = 1.5 * (sM / sy) * m->q1 * m->q2 * f * sinh(arg);",
     "double alpha = 1.0 * (sM / sy) * m->q1 * m->q2 * f * sinh(arg);"),
    ("GTN void growth without 1 / (alpha sigma* + 1)",
     "+ (1.0 - f) / (alpha * sstar + 1.0) * (sM / sy)",
     "+ (1.0 - f) * (sM / sy)"),
    ("GTN shear growth without f", "* (alpha * (1.0 - f) + f * m->k_omega * omega) * dem;",
     "* (alpha * (1.0 - f) + m->k_omega * omega) * dem;"),
]


def build_mutant(tmp, text, repl):
    src = open(SRC).read()
    assert src.count(text) == 1, text
    path = os.path.join(tmp, "mutant.c")
    with open(path, "w") as fh:
        fh.write(src.replace(text, repl))
    sys.path.insert(0, ROOT)
    import oracle
    lib = os.path.join(tmp, "libmutant.so")
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-I", os.path.join(ROOT, "oracle"),
                           "-o", lib, path, "-lm"])
    return lib


# the pin file expected to catch each mistake runs first (the run stops at
# the first failure); the others follow
HOME = {
    'kernel normalisation': 'kernel_neighbors',
    'kernel slope term': 'kernel_neighbors',
    'correction matrix without V_j': 'kernel_neighbors',
    'dF/dt weighted by D_i': 'system',
    'nodal force damage weights swapped': 'system',
    'nodal force drops Q_j': 'system',
    'hourglass sign': 'system',
    'hourglass with F_j transposed': 'system',
    'half drift': 'system',
    'failed particles keep moving': 'system',
    'EOS S_alpha sign': 'constitutive',
    'radial return with 2G': 'constitutive',
    'trial stress without (1 - D)': 'constitutive',
    'rotation applied transposed': 'constitutive',
    'JC failure strain sign of D3': 'constitutive',
    'flow stress rate term': 'constitutive',
    'GTN yield function factor': 'constitutive',
    'Voce law sign': 'flow',
    'Swift offset dropped': 'flow',
    'implicit return without (1 - D) on the flow stress': 'flow',
    "implicit return with the rate of the step's start": 'flow',
    'viscosity on separating pairs': 'viscosity',
    'viscosity quadratic term linear': 'viscosity',
    'viscosity applied with the wrong sign': 'viscosity',
    'viscosity not in the next kick': 'viscosity',
    "pair kernel with the particle's own support": 'graded',
    'neighbour rule with the larger support': 'graded',
    'contact force linear in the overlap': 'contact',
    'contact ignores failure': 'contact',
    'contact attractive': 'contact',
    'energy from P^{n+1} only': 'system',
    'thermal factor without its exponent': 'flow',
    'failure strain temperature factor sign': 'flow',
    'GTN void growth ratio without its 3/2': 'constitutive',
    'GTN void growth without 1 / (alpha sigma* + 1)': 'constitutive',
    'GTN shear growth without f': 'constitutive',
}


@pytest.mark.parametrize("name,text,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, text, repl):
    first = f"tests/test_oracle_{HOME[name]}.py"
    order = [first] + [f for f in PINS if f != first]
    with tempfile.TemporaryDirectory() as tmp:
        lib = build_mutant(tmp, text, repl)
        env = dict(os.environ, TLSPH_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                            "-p", "no:cacheprovider", *order],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, f"no pin caught: {name}\n{r.stdout[-2000:]}"
