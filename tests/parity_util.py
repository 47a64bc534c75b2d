"""Shared helpers of the parity tests: the error measure and field lists.

Error of a field q: max_i |q_i - q_ref_i| / max(max_i |q_ref_i|, floor_q), with
F compared as F - I.  Floors keep fields that are legitimately ~0 from
turning rounding noise into large relative errors.
"""
import numpy as np

FLOORS = {"u": 1e-12, "v": 1e-9, "F": 1e-9, "sig": 1.0, "Q": 1.0, "force": 1e-9,
          "eps_p": 1e-12, "eps_p_rate": 1e-6, "d_init": 1e-12, "w_p": 1.0, "f_void": 1e-12,
          "D": 1e-12, "e": 1e-9, "t": 1e-12, "Linv": 1e-12, "fvisc": 1e-12}

STEP_FIELDS = ("u", "v", "F", "sig", "Q", "force", "eps_p", "eps_p_rate", "d_init", "w_p",
               "f_void", "D", "e", "t", "fvisc")


def rel_err(name, got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if name == "F":
        eye = np.eye(3).ravel()
        got = got - eye
        ref = ref - eye
    den = max(np.abs(ref).max() if ref.size else 0.0, FLOORS.get(name, 1e-12))
    return float(np.abs(got - ref).max() / den) if ref.size else 0.0


def compare(gpu, orc, fields=STEP_FIELDS, skip=()):
    out = {}
    for k in fields:
        if k in skip:
            continue
        out[k] = rel_err(k, gpu.get(k), orc.get(k))
    return out
