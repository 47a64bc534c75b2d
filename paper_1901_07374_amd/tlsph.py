"""Python binding of libtlsph (the C ABI of include/tlsph.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libtlsph.so.  PyTorch provides device memory (the workspace and the
per-field staging tensors) and the stream.  If the library is not built, or
no GPU is present, construction fails loudly: there is no fallback path.

Field arrays cross the boundary component-major in caller order
(double[ncomp][n]); this wrapper presents them as (n, ncomp) tensors.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtlsph.so")

FP64, MIXED = 0, 1
STORE_FORCE, USE_GRAPHS, CHECK_FINITE, NO_STAGING = 1, 2, 4, 8

FIELDS = {"X": (0, 3), "u": (1, 3), "v": (2, 3), "F": (3, 9), "sig": (4, 6), "eps_p": (5, 1),
          "eps_p_rate": (6, 1), "d_init": (7, 1), "w_p": (8, 1), "f_void": (9, 1), "D": (10, 1),
          "e": (11, 1), "force": (12, 3), "Q": (13, 9), "t": (14, 0), "Linv": (15, 9),
          "fvisc": (16, 3), "H": (17, 9)}

STATUS = {0: "ok", 1: "invalid argument", 2: "bad call order", 3: "HIP runtime error",
          4: "singular correction matrix", 5: "non-finite state",
          6: "neighbour capacity exceeded", 7: "unsupported configuration"}


class TLSPHError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}" + (f" ({detail})" if detail else ""))


class Specimen(C.Structure):
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
                ("T_star", C.c_double), ("m", C.c_double), ("newton_max_iter", C.c_int32)]


class BCGroup(C.Structure):
    _fields_ = [("mask", C.c_int32), ("v_max", C.c_double * 3), ("tau", C.c_double),
                ("grad", C.c_double * 9)]


class StopRule(C.Structure):
    _fields_ = [("step_cap", C.c_int64), ("group", C.c_int32), ("axis", C.c_int32),
                ("sign", C.c_double), ("drop", C.c_double), ("min_peak", C.c_double)]


# why a specimen stopped under run control
RUNNING, STOPPED_AT_CAP, FAILED = 0, 1, 2

_vp = C.c_void_p
_lib = None


def library_path() -> str:
    return LIB_PATH


def lib():
    """Load libtlsph.so (built by paper_1901_07374_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1901_07374_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.tlsph_workspace_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int,
                                            C.POINTER(C.c_size_t)]
        L.tlsph_create.argtypes = [C.c_int64, C.c_int32, _vp, C.POINTER(Specimen), C.c_int32,
                                   C.POINTER(BCGroup), C.c_int, C.c_int32, C.c_uint32, _vp,
                                   C.c_size_t, _vp, C.POINTER(_vp)]
        L.tlsph_build_neighbors.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.tlsph_step.argtypes = [_vp, C.c_int32, _vp]
        L.tlsph_set_contact.argtypes = [_vp, C.c_int32, C.c_double]
        L.tlsph_get_state.argtypes = [_vp, C.c_int, _vp, C.c_size_t, _vp]
        L.tlsph_set_state.argtypes = [_vp, C.c_int, _vp, C.c_size_t, _vp]
        L.tlsph_neighbor_count.argtypes = [_vp, C.POINTER(C.c_int64)]
        L.tlsph_get_neighbors.argtypes = [_vp, _vp, _vp, _vp]
        L.tlsph_get_diagnostics.argtypes = [_vp, _vp, _vp, _vp]
        L.tlsph_get_diagnostics_static.argtypes = [_vp, _vp, _vp, _vp]
        L.tlsph_set_bc_groups.argtypes = [_vp, C.c_int32, C.POINTER(BCGroup), _vp]
        L.tlsph_autotune.argtypes = [_vp, _vp]
        L.tlsph_enable_kernel_timing.argtypes = [_vp, C.c_int32]
        L.tlsph_kernel_times.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.tlsph_info.argtypes = [_vp, C.POINTER(C.c_int64), _vp]
        L.tlsph_set_launch_shape.argtypes = [_vp, C.POINTER(C.c_int32), _vp]
        L.tlsph_set_run_control.argtypes = [_vp, C.POINTER(StopRule), _vp]
        L.tlsph_get_run_status.argtypes = [_vp, _vp, _vp, _vp, C.POINTER(C.c_int32), _vp]
        L.tlsph_run.argtypes = [_vp, C.c_int64, C.c_int32, C.POINTER(C.c_int64), _vp]
        L.tlsph_destroy.argtypes = [_vp]
        L.tlsph_destroy.restype = None
        L.tlsph_status_string.argtypes = [C.c_int]
        L.tlsph_status_string.restype = C.c_char_p
        L.tlsph_last_error.argtypes = [_vp]
        L.tlsph_last_error.restype = C.c_char_p
        for name in ("tlsph_workspace_bytes", "tlsph_create", "tlsph_build_neighbors",
                     "tlsph_step", "tlsph_get_state", "tlsph_set_state", "tlsph_neighbor_count",
                     "tlsph_get_neighbors", "tlsph_get_diagnostics",
                     "tlsph_get_diagnostics_static", "tlsph_set_bc_groups",
                     "tlsph_autotune", "tlsph_enable_kernel_timing", "tlsph_kernel_times",
                     "tlsph_info", "tlsph_set_launch_shape"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def specimen_struct(m: Dict) -> Specimen:
    s = Specimen()
    for name, typ in Specimen._fields_:
        if name == "wall_n":
            s.wall_n = (C.c_double * 3)(*m["wall_n"])
        elif typ is C.c_int32:
            setattr(s, name, int(m.get(name, 0)))
        else:
            setattr(s, name, float(m[name]))
    return s


def bc_struct(g: Dict) -> BCGroup:
    b = BCGroup()
    b.mask = int(g["mask"])
    b.v_max = (C.c_double * 3)(*g["v_max"])
    b.tau = float(g["tau"])
    b.grad = (C.c_double * 9)(*g["grad"])
    return b


def workspace_bytes(n: int, n_spec: int, n_bc: int, k_cap: int, precision: int) -> int:
    out = C.c_size_t()
    st = lib().tlsph_workspace_bytes(n, n_spec, n_bc, k_cap, precision, C.byref(out))
    if st:
        raise TLSPHError(st, "tlsph_workspace_bytes")
    return int(out.value)


class Sim:
    """One context over a Problem (see paper_1901_07374_amd.inputs)."""

    def __init__(self, prob, precision: int = FP64, k_cap: int = 32, flags: int = 0,
                 device: str = "cuda", stream=None, build: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libtlsph needs a HIP device; none is visible")
        self.torch = torch
        self.prob = prob
        self.n = prob.n
        self.n_spec = prob.n_spec
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lib()
        self.n_bc = len(prob.bc_groups)
        nbytes = workspace_bytes(self.n, self.n_spec, self.n_bc, k_cap, precision)
        # 256-byte aligned workspace from the torch caching allocator
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._specs = (Specimen * self.n_spec)(*[specimen_struct(m) for m in prob.materials])
        nb = max(self.n_bc, 1)
        self._bcs = (BCGroup * nb)(*[bc_struct(g) for g in prob.bc_groups])
        self._offs = np.ascontiguousarray(prob.spec_offsets, np.int64)
        ctx = _vp()
        st = L.tlsph_create(self.n, self.n_spec, self._offs.ctypes.data, self._specs, self.n_bc,
                            self._bcs, precision, k_cap, flags, self._ws_ptr, nbytes,
                            self._sp(), C.byref(ctx))
        if st:
            raise TLSPHError(st, "tlsph_create")
        self.ctx = ctx
        if build:
            self.build()

    def _sp(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _check(self, st: int, where: str):
        if st:
            raise TLSPHError(st, where, lib().tlsph_last_error(self.ctx).decode())

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and _lib is not None:
            _lib.tlsph_destroy(ctx)
            self.ctx = None

    # ------------------------------------------------------------------
    def build(self):
        t = self.torch
        d = self.device
        X = t.as_tensor(np.ascontiguousarray(self.prob.X.T), dtype=t.float64).to(d).contiguous()
        V0 = t.as_tensor(self.prob.V0, dtype=t.float64).to(d).contiguous()
        bc = t.as_tensor(self.prob.bc_group, dtype=t.int32).to(d).contiguous()
        self._check(lib().tlsph_build_neighbors(self.ctx, X.data_ptr(), V0.data_ptr(),
                                                bc.data_ptr(), self._sp()), "tlsph_build_neighbors")
        if np.any(self.prob.v_init != 0.0):
            self.set("v", self.prob.v_init)

    def step(self, k: int = 1):
        self._check(lib().tlsph_step(self.ctx, int(k), self._sp()), "tlsph_step")

    def get_tensor(self, name: str):
        """Field as a device tensor, (n, ncomp) (or (n,), or (n_spec,) for t)."""
        t = self.torch
        fid, comps = FIELDS[name]
        if name == "t":
            out = t.empty(self.n_spec, dtype=t.float64, device=self.device)
            nbytes = self.n_spec * 8
        else:
            out = t.empty((comps, self.n), dtype=t.float64, device=self.device)
            nbytes = comps * self.n * 8
        self._check(lib().tlsph_get_state(self.ctx, fid, out.data_ptr(), nbytes, self._sp()),
                    f"tlsph_get_state({name})")
        if name == "t":
            return out
        return out[0] if comps == 1 else out.t()

    def get(self, name: str) -> np.ndarray:
        x = self.get_tensor(name)
        self.stream.synchronize()
        return x.cpu().numpy().copy()

    def set(self, name: str, value):
        t = self.torch
        fid, comps = FIELDS[name]
        a = np.asarray(value, np.float64)
        if name == "t":
            a = a.reshape(self.n_spec)
        elif comps == 1:
            a = a.reshape(1, self.n)
        else:
            a = a.reshape(self.n, comps).T
        src = t.as_tensor(np.ascontiguousarray(a), dtype=t.float64).to(self.device)
        self._check(lib().tlsph_set_state(self.ctx, fid, src.data_ptr(), src.numel() * 8,
                                          self._sp()), f"tlsph_set_state({name})")
        self.stream.synchronize()

    def set_state(self, st: Dict[str, np.ndarray]):
        for k, v in st.items():
            self.set(k, v)

    def set_tensor(self, name: str, x):
        """Overwrite a field from a device tensor shaped as get_tensor returns
        it (stream-ordered, no host copy)."""
        fid, comps = FIELDS[name]
        if name == "t" or comps == 1:
            src = x.contiguous()
        else:
            src = x.t().contiguous()
        self._check(lib().tlsph_set_state(self.ctx, fid, src.data_ptr(), src.numel() * 8,
                                          self._sp()), f"tlsph_set_state({name})")
        self.stream.synchronize()

    # every field that makes up the evolving state (F through H = F - I, so a
    # context of the same precision continues bit for bit)
    STATE = ("u", "v", "H", "sig", "eps_p", "eps_p_rate", "d_init", "w_p", "f_void", "D", "e",
             "Q", "fvisc", "t")

    def copy_state_from(self, other: "Sim"):
        """Take over the state of another context over the same problem
        (device to device); across precisions the stored float fields are
        rounded or widened."""
        for k in self.STATE:
            x = other.get_tensor(k)
            other.stream.synchronize()
            self.set_tensor(k, x)

    def neighbors(self):
        t = self.torch
        nnz = C.c_int64()
        self._check(lib().tlsph_neighbor_count(self.ctx, C.byref(nnz)), "tlsph_neighbor_count")
        rp = t.empty(self.n + 1, dtype=t.int64, device=self.device)
        col = t.empty(max(nnz.value, 1), dtype=t.int32, device=self.device)
        self._check(lib().tlsph_get_neighbors(self.ctx, rp.data_ptr(), col.data_ptr(), self._sp()),
                    "tlsph_get_neighbors")
        self.stream.synchronize()
        return rp.cpu().numpy(), col.cpu().numpy()[: nnz.value]

    def diagnostics(self):
        t = self.torch
        sd = t.empty((self.n_spec, 8), dtype=t.float64, device=self.device)
        bd = t.empty((max(self.n_bc, 1), 8), dtype=t.float64, device=self.device)
        self._check(lib().tlsph_get_diagnostics(self.ctx, sd.data_ptr(),
                                                bd.data_ptr() if self.n_bc else None, self._sp()),
                    "tlsph_get_diagnostics")
        self.stream.synchronize()
        return sd.cpu().numpy(), bd.cpu().numpy()[: self.n_bc]

    def set_bc_groups(self, groups: Sequence[Dict]):
        arr = (BCGroup * max(len(groups), 1))(*[bc_struct(g) for g in groups])
        self._check(lib().tlsph_set_bc_groups(self.ctx, len(groups), arr, self._sp()),
                    "tlsph_set_bc_groups")
        self._keep_bcs = arr

    def autotune(self):
        self._check(lib().tlsph_autotune(self.ctx, self._sp()), "tlsph_autotune")

    def enable_kernel_timing(self, stride: int = 1):
        """Time both step kernels of every stride-th step (0: off)."""
        self._check(lib().tlsph_enable_kernel_timing(self.ctx, int(stride)), "enable_kernel_timing")

    def kernel_times(self):
        ms = (C.c_double * 2)()
        cnt = (C.c_int64 * 2)()
        self._check(lib().tlsph_kernel_times(self.ctx, ms, cnt), "tlsph_kernel_times")
        return {"force_pass": (ms[0], cnt[0]), "deformation_pass": (ms[1], cnt[1])}

    def info(self) -> Dict[str, int]:
        out = (C.c_int64 * 9)()
        self._check(lib().tlsph_info(self.ctx, out, self._sp()), "tlsph_info")
        return dict(block_force=abs(out[0]), staged=out[0] < 0, block_deformation=out[1],
                    nnz=out[2], slots=out[3], n=out[4], flags=out[5],
                    lanes_per_particle=out[6], lds_bytes=out[7], tile=out[8])

    def set_contact(self, every: int = 1, skin: float = 0.0):
        """Rebuild the penalty-contact candidate lists every `every` steps
        with the given skin (valid while no particle moves more than
        skin / 2 between rebuilds; flagged otherwise)."""
        self._check(lib().tlsph_set_contact(self.ctx, int(every), float(skin)),
                    "tlsph_set_contact")

    def set_run_control(self, rules: Optional[Sequence[Dict]]):
        """Per-specimen stop rules (dicts with step_cap, and for failure
        group, axis, sign, drop, min_peak), or None to switch run control
        off."""
        if rules is None:
            self._check(lib().tlsph_set_run_control(self.ctx, None, self._sp()),
                        "tlsph_set_run_control")
            return
        arr = (StopRule * self.n_spec)()
        for q, r in enumerate(rules):
            arr[q] = StopRule(int(r.get("step_cap", 0)), int(r.get("group", -1)),
                              int(r.get("axis", 0)), float(r.get("sign", 1.0)),
                              float(r.get("drop", 0.5)), float(r.get("min_peak", 0.0)))
        self._check(lib().tlsph_set_run_control(self.ctx, arr, self._sp()),
                    "tlsph_set_run_control")

    def run_status(self) -> Dict[str, np.ndarray]:
        why = np.zeros(self.n_spec, np.int32)
        steps = np.zeros(self.n_spec, np.int64)
        peak = np.zeros(self.n_spec, np.float64)
        nr = C.c_int32(0)
        self._check(lib().tlsph_get_run_status(self.ctx, why.ctypes.data, steps.ctypes.data,
                                               peak.ctypes.data, C.byref(nr), self._sp()),
                    "tlsph_get_run_status")
        return {"why": why, "steps": steps, "peak": peak, "running": int(nr.value)}

    def run(self, max_steps: int, check_every: int = 100) -> int:
        """Step until every specimen has stopped (or max_steps); the steps run."""
        done = C.c_int64(0)
        self._check(lib().tlsph_run(self.ctx, int(max_steps), int(check_every), C.byref(done),
                                    self._sp()), "tlsph_run")
        return int(done.value)

    def set_launch_shape(self, staged: bool, lanes: int, block_force: int = 256,
                         block_deformation: int = 256, tile: int = 0):
        shape = (C.c_int32 * 5)(int(staged), int(lanes), int(block_force),
                                int(block_deformation), int(tile))
        self._check(lib().tlsph_set_launch_shape(self.ctx, shape, self._sp()),
                    "tlsph_set_launch_shape")