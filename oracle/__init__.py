"""ctypes binding of the FP64 CPU oracle (tlsph_oracle.c).

TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it.  It never touches the GPU library and the GPU library never
touches it.

Arrays are host numpy arrays in caller order: vectors (n, 3), tensors (n, 9)
row-major, symmetric tensors (n, 6) Voigt (xx, yy, zz, yz, xz, xy).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TLSPH_ORACLE_LIB points the binding at another build of the same source
# (the mutation test loads deliberately broken copies this way)
LIB_PATH = os.environ.get("TLSPH_ORACLE_LIB") or os.path.join(_HERE, "libtlsph_oracle.so")
SRC = os.path.join(_HERE, "tlsph_oracle.c")

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
          "-Wall", "-Wextra", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Material(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("rho0", "E", "nu", "c0", "S_alpha", "Gamma0",
                                          "A", "B", "n", "C", "eps_dot0")] + \
               [("damage", C.c_int32)] + \
               [(k, C.c_double) for k in ("Wcr", "D1", "D2", "D3", "D4", "D5", "q1", "q2",
                                          "q3", "f0", "fN", "eN", "sN", "fc", "fF",
                                          "k_omega", "h", "dt", "hg_alpha")] + \
               [("has_wall", C.c_int32), ("wall_n", C.c_double * 3), ("wall_d", C.c_double),
                ("flow", C.c_int32), ("implicit_return", C.c_int32), ("flow_e0", C.c_double),
                ("flow_beta", C.c_double), ("av_q1", C.c_double), ("av_q2", C.c_double),
                ("h_per_spacing", C.c_double), ("contact_k", C.c_double),
                ("T_star", C.c_double), ("m", C.c_double)]


class BC(C.Structure):
    _fields_ = [("mask", C.c_int32), ("v_max", C.c_double * 3), ("tau", C.c_double),
                ("grad", C.c_double * 9)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class ProblemC(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_spec", C.c_int32), ("spec", _ip),
                ("mat", C.POINTER(Material)), ("X", _dp), ("V0", _dp), ("bc", _ip),
                ("n_bc", C.c_int32), ("bcs", C.POINTER(BC)), ("row_ptr", _lp), ("col", _ip),
                ("Linv", _dp), ("hs", _dp)]


STATE_FIELDS = ("t", "u", "v", "F", "sig", "eps_p", "eps_p_rate", "d_init", "w_p",
                "f_void", "D", "e", "Q", "force", "fvisc")


class StateC(C.Structure):
    _fields_ = [(k, _dp) for k in STATE_FIELDS]


class PointC(C.Structure):
    _fields_ = [("F", C.c_double * 9), ("sig", C.c_double * 6)] + \
               [(k, C.c_double) for k in ("eps_p", "eps_p_rate", "d_init", "w_p", "f_void",
                                          "D", "e")]


class PointInfo(C.Structure):
    _fields_ = [("dep", C.c_double), ("J", C.c_double), ("yielded", C.c_int32),
                ("newton_x_iters", C.c_int32), ("newton_e_iters", C.c_int32),
                ("newton_failed", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_kernel.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.orc_support_radii.argtypes = [C.c_int64, _dp, _ip, C.POINTER(Material), _dp]
        L.orc_build_neighbors.argtypes = [C.c_int64, _dp, _ip, C.POINTER(Material), _dp, _lp,
                                          _ip, C.c_int64]
        L.orc_build_neighbors.restype = C.c_int64
        L.orc_shape_matrices.argtypes = [C.POINTER(ProblemC), _dp, _dp]
        L.orc_shape_matrices.restype = C.c_int64
        L.orc_init_state.argtypes = [C.POINTER(ProblemC), _dp, C.POINTER(StateC)]
        L.orc_step.argtypes = [C.POINTER(ProblemC), C.POINTER(StateC)]
        L.orc_diagnostics.argtypes = [C.POINTER(ProblemC), C.POINTER(StateC), _dp, _dp]
        L.orc_point_update.argtypes = [C.POINTER(Material), C.c_double, _dp, C.POINTER(PointC),
                                       _dp, C.POINTER(PointInfo)]
        L.orc_mean_stress_eos.argtypes = [C.POINTER(Material), C.c_double, C.c_double,
                                          C.c_double, C.c_int32]
        L.orc_mean_stress_eos.restype = C.c_double
        L.orc_flow_stress.argtypes = [C.POINTER(Material), C.c_double, C.c_double]
        L.orc_flow_stress.restype = C.c_double
        L.orc_principal_max.argtypes = [_dp]
        L.orc_principal_max.restype = C.c_double
        L.orc_omega.argtypes = [_dp]
        L.orc_omega.restype = C.c_double
        L.orc_fstar.argtypes = [C.POINTER(Material), C.c_double]
        L.orc_fstar.restype = C.c_double
        L.orc_hughes_winget.argtypes = [C.c_double, _dp, _dp, _dp]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_get_threads.restype = C.c_int32
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _p(a: np.ndarray, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def material_struct(m: Dict) -> Material:
    s = Material()
    for name, typ in Material._fields_:
        if name == "wall_n":
            s.wall_n = (C.c_double * 3)(*m["wall_n"])
        elif typ is C.c_int32:
            setattr(s, name, int(m[name]))
        else:
            setattr(s, name, float(m[name]))
    return s


def bc_struct(g: Dict) -> BC:
    b = BC()
    b.mask = int(g["mask"])
    b.v_max = (C.c_double * 3)(*g["v_max"])
    b.tau = float(g["tau"])
    b.grad = (C.c_double * 9)(*g["grad"])
    return b


# --------------------------------------------------------------------------
# pieces
# --------------------------------------------------------------------------
def kernel(r: float, h: float):
    W, dW = C.c_double(), C.c_double()
    lib().orc_kernel(r, h, C.byref(W), C.byref(dW))
    return W.value, dW.value


def mean_stress_eos(m: Dict, J: float, D: float = 0.0, e: float = 0.0,
                    damaged_branch: bool = True) -> float:
    ms = material_struct(m)
    return lib().orc_mean_stress_eos(C.byref(ms), J, D, e, int(damaged_branch))


def flow_stress(m: Dict, eps: float, rate: float = 0.0) -> float:
    ms = material_struct(m)
    return lib().orc_flow_stress(C.byref(ms), eps, rate)


def principal_max(sig6) -> float:
    a = np.ascontiguousarray(sig6, np.float64)
    return lib().orc_principal_max(_p(a))


def omega(sig6) -> float:
    a = np.ascontiguousarray(sig6, np.float64)
    return lib().orc_omega(_p(a))


def fstar(m: Dict, f: float) -> float:
    ms = material_struct(m)
    return lib().orc_fstar(C.byref(ms), f)


def hughes_winget(dt: float, w: np.ndarray, sd: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w, np.float64).ravel()
    sd = np.ascontiguousarray(sd, np.float64).ravel()
    out = np.zeros(9)
    lib().orc_hughes_winget(dt, _p(w), _p(sd), _p(out))
    return out.reshape(3, 3)


class Point:
    """One material point driven by a prescribed dF/dt (constitutive pins)."""

    def __init__(self, m: Dict, **init):
        self.m = m
        self.ms = material_struct(m)
        self.pt = PointC()
        for k in range(9):
            self.pt.F[k] = 1.0 if k % 4 == 0 else 0.0
        self.pt.f_void = m.get("f0", 0.0)
        self.pt.D = 0.0
        for k, v in init.items():
            if k in ("F", "sig"):
                arr = getattr(self.pt, k)
                for i, x in enumerate(np.ravel(v)):
                    arr[i] = float(x)
            else:
                setattr(self.pt, k, float(v))
        self.P = np.zeros(9)
        self.info = PointInfo()

    def update(self, Fdot, dt: Optional[float] = None) -> "Point":
        fd = np.ascontiguousarray(Fdot, np.float64).ravel()
        lib().orc_point_update(C.byref(self.ms), self.m["dt"] if dt is None else dt, _p(fd),
                               C.byref(self.pt), _p(self.P), C.byref(self.info))
        return self

    def __getattr__(self, k):
        if k in ("F", "sig"):
            return np.array(getattr(self.pt, k)[:])
        if k in ("eps_p", "eps_p_rate", "d_init", "w_p", "f_void", "D", "e"):
            return getattr(self.pt, k)
        raise AttributeError(k)


# --------------------------------------------------------------------------
# whole problem
# --------------------------------------------------------------------------
def support_radii(V0: np.ndarray, spec: np.ndarray, materials) -> np.ndarray:
    V0 = np.ascontiguousarray(V0, np.float64)
    spec = np.ascontiguousarray(spec, np.int32)
    mats = (Material * len(materials))(*[material_struct(m) for m in materials])
    hs = np.zeros(V0.shape[0])
    lib().orc_support_radii(V0.shape[0], _p(V0), _p(spec, C.c_int32), mats, _p(hs))
    return hs


def neighbors(X: np.ndarray, spec: np.ndarray, materials, hs=None) -> tuple:
    """Reference neighbour lists; hs: per-particle support radii (None: each
    specimen's h)."""
    X = np.ascontiguousarray(X, np.float64)
    spec = np.ascontiguousarray(spec, np.int32)
    mats = (Material * len(materials))(*[material_struct(m) for m in materials])
    hp = None if hs is None else _p(np.ascontiguousarray(hs, np.float64))
    n = X.shape[0]
    row_ptr = np.zeros(n + 1, np.int64)
    nnz = lib().orc_build_neighbors(n, _p(X), _p(spec, C.c_int32), mats, hp,
                                    _p(row_ptr, C.c_int64), None, 0)
    col = np.zeros(max(nnz, 1), np.int32)
    lib().orc_build_neighbors(n, _p(X), _p(spec, C.c_int32), mats, hp, _p(row_ptr, C.c_int64),
                              _p(col, C.c_int32), nnz)
    return row_ptr, col[:nnz]


class OracleError(RuntimeError):
    pass


class Sim:
    """The oracle run of one Problem (see paper_1901_07374_amd.inputs)."""

    def __init__(self, prob, v_init: Optional[np.ndarray] = None):
        self.prob = prob
        n = prob.n
        self.X = np.ascontiguousarray(prob.X, np.float64)
        self.V0 = np.ascontiguousarray(prob.V0, np.float64)
        self.spec = np.ascontiguousarray(prob.spec_id(), np.int32)
        self.bc = np.ascontiguousarray(prob.bc_group, np.int32)
        self.mats = (Material * prob.n_spec)(*[material_struct(m) for m in prob.materials])
        nb = max(len(prob.bc_groups), 1)
        self.bcs = (BC * nb)(*[bc_struct(g) for g in prob.bc_groups])
        self.hs = support_radii(self.V0, self.spec, prob.materials)
        self.row_ptr, self.col = neighbors(self.X, self.spec, prob.materials, self.hs)
        if self.col.size == 0:
            self.col = np.zeros(1, np.int32)
        self.L = np.zeros((n, 9))
        self.Linv = np.zeros((n, 9))
        self.pc = ProblemC(n, prob.n_spec, _p(self.spec, C.c_int32), self.mats, _p(self.X),
                           _p(self.V0), _p(self.bc, C.c_int32), len(prob.bc_groups), self.bcs,
                           _p(self.row_ptr, C.c_int64), _p(self.col, C.c_int32), _p(self.Linv),
                           _p(self.hs))
        bad = lib().orc_shape_matrices(C.byref(self.pc), _p(self.L), _p(self.Linv))
        if bad >= 0:
            raise OracleError(f"singular correction matrix at particle {bad}")
        shapes = dict(t=(prob.n_spec,), u=(n, 3), v=(n, 3), F=(n, 9), sig=(n, 6), Q=(n, 9),
                      force=(n, 3), fvisc=(n, 3))
        self.state = {k: np.zeros(shapes.get(k, (n,))) for k in STATE_FIELDS}
        self.sc = StateC(*[_p(self.state[k]) for k in STATE_FIELDS])
        vi = np.ascontiguousarray(prob.v_init if v_init is None else v_init, np.float64)
        lib().orc_init_state(C.byref(self.pc), _p(vi), C.byref(self.sc))

    def set_bc_groups(self, groups):
        self.prob.bc_groups = list(groups)
        self.bcs = (BC * max(len(groups), 1))(*[bc_struct(g) for g in groups])
        self.pc.bcs = self.bcs
        self.pc.n_bc = len(groups)

    def step(self, k: int = 1):
        for _ in range(k):
            lib().orc_step(C.byref(self.pc), C.byref(self.sc))

    def diagnostics(self):
        """(spec_diag (n_spec, 8), bc_diag (n_bc, 8)) of the current state:
        kinetic and internal energy, failed count, max D, time per specimen;
        summed nodal force, mean displacement and count per group."""
        sd = np.zeros((self.prob.n_spec, 8))
        bd = np.zeros((max(len(self.prob.bc_groups), 1), 8))
        lib().orc_diagnostics(C.byref(self.pc), C.byref(self.sc), _p(sd), _p(bd))
        return sd, bd[: len(self.prob.bc_groups)]

    def get(self, name: str) -> np.ndarray:
        return self.state[name].copy()

    def set(self, name: str, value):
        self.state[name][...] = value

    def set_state(self, st: Dict[str, np.ndarray]):
        for k, v in st.items():
            self.set(k, v)

    def neighbor_sets(self):
        return [self.col[self.row_ptr[i]:self.row_ptr[i + 1]] for i in range(self.prob.n)]
