"""Seeded synthetic specimens for the TLSPH damage step.

This module only lays out particles and fills parameter tables. It holds none
of the method's arithmetic: both the FP64 CPU oracle and the GPU library
consume what it returns, and neither is imported here.

Workload structure follows the paper's case study (Sec. 6): a simple cubic
lattice of particles, the axial velocity ramp v_max (1 - exp(-t)) on the end
rows, Weldox-like steel. Geometry and sizes are synthetic stand-ins for the
specimens of the paper's Fig. 3, whose drawings and experimental data are not
available; every generator is seeded so the same arrays reach both sides.

Units are SI throughout (m, kg, s, Pa).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

SEED_BASE = 190107374

# damage model identifiers (same numbering on both sides of the boundary)
DMG_NONE, DMG_CL, DMG_JC, DMG_GTN = 0, 1, 2, 3
# strain-hardening laws of the flow stress: Johnson-Cook A + B eps^n, linear
# A + B eps, Swift B (flow_e0 + eps)^n, Voce A + B (1 - exp(-flow_beta eps))
FLOW_JC, FLOW_LINEAR, FLOW_SWIFT, FLOW_VOCE = 0, 1, 2, 3

# Field order of one per-specimen parameter record.
MATERIAL_KEYS = (
    "rho0", "E", "nu", "c0", "S_alpha", "Gamma0",
    "A", "B", "n", "C", "eps_dot0",
    "damage", "Wcr", "D1", "D2", "D3", "D4", "D5",
    "q1", "q2", "q3", "f0", "fN", "eN", "sN", "fc", "fF", "k_omega",
    "h", "dt", "hg_alpha", "has_wall", "wall_n", "wall_d",
    "flow", "implicit_return", "flow_e0", "flow_beta", "av_q1", "av_q2", "h_per_spacing",
    "contact_k", "T_star", "m", "newton_max_iter",
)

# Steel used by every synthetic workload (rho, E, nu and the Johnson-Cook
# flow constants are the ones the benchmark configurations name).  The bulk
# sound speed follows the value printed in Table 1 of the paper, which is
# reproduced by c0 = sqrt(E / (3 (1 - 2 nu)) / rho0).
STEEL = dict(rho0=7850.0, E=200e9, nu=0.3, S_alpha=1.5, Gamma0=0.0,
             A=792e6, B=510e6, n=0.26, C=0.014, eps_dot0=1.0)
JC_DAMAGE = dict(D1=0.05, D2=3.44, D3=-2.12, D4=0.002, D5=0.61)
GTN = dict(q1=1.5, q2=1.0, q3=2.25, f0=0.001, fN=0.04, eN=0.3, sN=0.1,
           fc=0.15, fF=0.25, k_omega=3.5)


def bulk_sound_speed(E: float, nu: float, rho0: float) -> float:
    """Input recipe for c0 (material data, not a step of the method)."""
    return math.sqrt(E / (3.0 * (1.0 - 2.0 * nu)) / rho0)


def material(dx: float, damage: int = DMG_NONE, **over) -> Dict:
    """One specimen's parameter record with h = 1.5 dx and dt = 0.3 dx / c0."""
    m = dict(STEEL)
    m.update(dict(damage=damage, Wcr=0.0, D1=0.0, D2=0.0, D3=0.0, D4=0.0, D5=0.0,
                  q1=1.0, q2=1.0, q3=1.0, f0=0.0, fN=0.0, eN=0.0, sN=1.0,
                  fc=1.0, fF=1.0, k_omega=0.0, hg_alpha=1.0, has_wall=0,
                  wall_n=(0.0, 0.0, 1.0), wall_d=0.0, flow=FLOW_JC, implicit_return=0,
                  flow_e0=0.0, flow_beta=0.0, av_q1=0.0, av_q2=0.0, h_per_spacing=0.0,
                  contact_k=0.0, T_star=0.0, m=1.0, newton_max_iter=0))
    if damage == DMG_JC:
        m.update(JC_DAMAGE)
    if damage == DMG_GTN:
        m.update(GTN)
    m.update(over)
    if "c0" not in over:
        m["c0"] = bulk_sound_speed(m["E"], m["nu"], m["rho0"])
    if "h" not in over:
        m["h"] = 1.5 * dx
    if "dt" not in over:
        m["dt"] = 0.3 * dx / m["c0"]
    return m


def bc_group(mask: int, v_max=(0.0, 0.0, 0.0), tau: float = 0.0, grad=None) -> Dict:
    """Prescribed-velocity group: component c (bit c of mask) follows
    v_max[c] (1 - exp(-t / tau)) + sum_b grad[3c+b] X_b  (tau = 0: constant)."""
    return dict(mask=int(mask), v_max=tuple(float(x) for x in v_max), tau=float(tau),
                grad=tuple(float(x) for x in (grad if grad is not None else (0.0,) * 9)))


@dataclasses.dataclass
class Problem:
    """Particles of one or more specimens, contiguous per specimen."""
    name: str
    X: np.ndarray             # (n, 3) f64 reference positions
    V0: np.ndarray            # (n,)   f64 reference volumes
    spec_offsets: np.ndarray  # (n_spec + 1,) int64
    materials: List[Dict]     # one record per specimen (MATERIAL_KEYS)
    bc_group: np.ndarray      # (n,) int32, -1 = free
    bc_groups: List[Dict]     # prescribed-velocity groups
    v_init: np.ndarray        # (n, 3) f64 initial velocity
    steps: int = 100          # steps the workload is quoted for
    dx: Optional[np.ndarray] = None  # (n_spec,) lattice spacing

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_spec(self) -> int:
        return len(self.materials)

    def spec_id(self) -> np.ndarray:
        sid = np.empty(self.n, np.int32)
        for s in range(self.n_spec):
            sid[self.spec_offsets[s]:self.spec_offsets[s + 1]] = s
        return sid


def _jitter(rng, pts: np.ndarray, dx: float, jitter: float) -> np.ndarray:
    if jitter <= 0.0:
        return pts.copy()
    return pts + rng.uniform(-jitter * dx, jitter * dx, size=pts.shape)


def _lattice(nx: int, ny: int, nz: int):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


# ----------------------------------------------------------------------------
# c1: cube in uniaxial tension
# ----------------------------------------------------------------------------
def cube(nside: int = 10, dx: float = 1e-3, jitter: float = 0.05, v: float = 1.0,
         damage: int = DMG_NONE, seed: int = SEED_BASE + 0, **mat_over) -> Problem:
    rng = np.random.default_rng(seed)
    i, j, k = _lattice(nside, nside, nside)
    lat = np.stack([(i + 0.5) * dx, (j + 0.5) * dx, (k + 0.5) * dx], axis=1)
    X = _jitter(rng, lat, dx, jitter)
    n = X.shape[0]
    bc = np.full(n, -1, np.int32)
    bc[k < 2] = 0
    bc[k >= nside - 2] = 1
    groups = [bc_group(4, (0.0, 0.0, -v)), bc_group(4, (0.0, 0.0, v))]
    return Problem("cube", X, np.full(n, dx ** 3), np.array([0, n], np.int64),
                   [material(dx, damage, **mat_over)], bc, groups,
                   np.zeros((n, 3)), steps=100, dx=np.array([dx]))


# ----------------------------------------------------------------------------
# c2 / c5: notched round bar (axis z), 90 degree V-notch at mid-length
# ----------------------------------------------------------------------------
BAR_R, BAR_L, NOTCH_DEPTH = 5e-3, 40e-3, 1e-3


def notched_bar_volume(R=BAR_R, L=BAR_L, d=NOTCH_DEPTH) -> float:
    """Solid volume of the notched bar (Pappus for the triangular groove)."""
    return math.pi * R * R * L - 2.0 * math.pi * (R - d / 3.0) * d * d


def _notched_bar_points(dx, R=BAR_R, L=BAR_L, d=NOTCH_DEPTH):
    nr = int(math.ceil(2 * R / dx))
    nz = int(round(L / dx))
    i, j, k = _lattice(nr, nr, nz)
    x = (i + 0.5) * dx - nr * dx / 2
    y = (j + 0.5) * dx - nr * dx / 2
    z = (k + 0.5) * dx
    r = np.sqrt(x * x + y * y)
    zc = np.abs(z - L / 2)
    rmax = np.where(zc < d, R - d + zc, R)
    keep = r < rmax
    return np.stack([x[keep], y[keep], z[keep]], axis=1), k[keep], nz


def notched_bar(dx: float = 0.25e-3, jitter: float = 0.03, v_max: float = 10.0,
                tau: float = 1e-3, damage: int = DMG_JC, seed: int = SEED_BASE + 1,
                steps: int = 43000, **mat_over) -> Problem:
    rng = np.random.default_rng(seed)
    lat, k, nz = _notched_bar_points(dx)
    X = _jitter(rng, lat, dx, jitter)
    n = X.shape[0]
    bc = np.full(n, -1, np.int32)
    bc[k < 2] = 0
    bc[k >= nz - 2] = 1
    groups = [bc_group(4, (0.0, 0.0, -v_max), tau), bc_group(4, (0.0, 0.0, v_max), tau)]
    return Problem("notched_bar", X, np.full(n, dx ** 3), np.array([0, n], np.int64),
                   [material(dx, damage, **mat_over)], bc, groups, np.zeros((n, 3)),
                   steps=steps, dx=np.array([dx]))


# ----------------------------------------------------------------------------
# graded notched bar: a round bar with a semicircular notch (radius rho) at
# mid-length, the particle spacing refined towards the notch plane in axial
# zones (finest first); each zone is a cubic lattice of its own spacing, so
# the lattices meet unconformingly at the zone boundaries.  V_i = dx^3 of the
# particle's zone and the support radius is 1.75 times the local spacing.
# ----------------------------------------------------------------------------
def graded_notched_bar(R: float = 5e-3, L: float = 7e-3, rho: float = 0.4e-3,
                       spacings=(0.1e-3, 0.2e-3, 0.4e-3, 0.8e-3),
                       bounds=(0.5e-3, 1.5e-3, 2.5e-3), jitter: float = 0.03,
                       v_max: float = 10.0, tau: float = 1e-3, damage: int = DMG_JC,
                       seed: int = SEED_BASE + 6, steps: int = 2000, **mat_over) -> Problem:
    """Zones |z| < bounds[0] at spacings[0], ..., the last up to L / 2; the
    prescribed-velocity grips are the particles of the coarsest zone.  The
    support is 1.75 times the local spacing: at 1.5 the particles next to a
    zone boundary keep too few neighbours (down to four) for a stable
    correction matrix."""
    rng = np.random.default_rng(seed)
    edges = [0.0, *bounds, L / 2]
    pts, vol, zone = [], [], []
    for q, dx in enumerate(spacings):
        z0, z1 = edges[q], edges[q + 1]
        nz = max(1, int(round((z1 - z0) / dx)))
        nr = int(math.ceil(2 * R / dx))
        i, j, k = _lattice(nr, nr, nz)
        x = (i + 0.5) * dx - nr * dx / 2
        y = (j + 0.5) * dx - nr * dx / 2
        z = z0 + (k + 0.5) * (z1 - z0) / nz
        r = np.sqrt(x * x + y * y)
        for sgn in (1.0, -1.0):
            zz = sgn * z
            az = np.abs(zz)
            rmax = np.where(az < rho, R - np.sqrt(np.maximum(rho * rho - az * az, 0.0)), R)
            keep = r < rmax
            lat = np.stack([x[keep], y[keep], zz[keep]], axis=1)
            pts.append(_jitter(rng, lat, dx, jitter))
            vol.append(np.full(lat.shape[0], dx ** 3))
            zone.append(np.full(lat.shape[0], q))
    X = np.concatenate(pts)
    V0 = np.concatenate(vol)
    zone = np.concatenate(zone)
    n = X.shape[0]
    bc = np.full(n, -1, np.int32)
    last = len(spacings) - 1
    bc[(zone == last) & (X[:, 2] < 0)] = 0
    bc[(zone == last) & (X[:, 2] > 0)] = 1
    groups = [bc_group(4, (0.0, 0.0, -v_max), tau), bc_group(4, (0.0, 0.0, v_max), tau)]
    dxm = min(spacings)
    m = material(dxm, damage, **dict(dict(h_per_spacing=1.75), **mat_over))
    m["h"] = 1.5 * max(spacings)
    return Problem("graded_notched_bar", X, V0, np.array([0, n], np.int64), [m], bc, groups,
                   np.zeros((n, 3)), steps=steps, dx=np.array([dxm]))


# ----------------------------------------------------------------------------
# two bars meeting head on (two specimens): they interact only through the
# penalty contact; bar 0 below z = -gap/2 moving up, bar 1 above gap/2 moving
# down, each at v0
# ----------------------------------------------------------------------------
def bar_collision(dx: float = 0.2e-3, R: float = 2.5e-3, L: float = 10e-3, gap: float = 0.1e-3,
                  v0: float = 100.0, jitter: float = 0.03, damage: int = DMG_CL,
                  Wcr: float = 300e6, contact_k: float = 1.0, seed: int = SEED_BASE + 7,
                  steps: int = 2000, **mat_over) -> Problem:
    rng = np.random.default_rng(seed)
    nr = int(math.ceil(2 * R / dx))
    nz = int(round(L / dx))
    i, j, k = _lattice(nr, nr, nz)
    x = (i + 0.5) * dx - nr * dx / 2
    y = (j + 0.5) * dx - nr * dx / 2
    z = (k + 0.5) * dx
    keep = np.sqrt(x * x + y * y) < R
    lat = np.stack([x[keep], y[keep], z[keep]], axis=1)
    lo = lat.copy()
    lo[:, 2] = -gap / 2 - lo[:, 2]
    hi = lat.copy()
    hi[:, 2] = gap / 2 + hi[:, 2]
    X = np.concatenate([_jitter(rng, lo, dx, jitter), _jitter(rng, hi, dx, jitter)])
    n0 = lo.shape[0]
    n = X.shape[0]
    v = np.zeros((n, 3))
    v[:n0, 2] = v0
    v[n0:, 2] = -v0
    m = material(dx, damage, **dict(dict(Wcr=Wcr, contact_k=contact_k), **mat_over))
    return Problem("bar_collision", X, np.full(n, dx ** 3), np.array([0, n0, n], np.int64),
                   [m, dict(m)], np.full(n, -1, np.int32), [], v, steps=steps,
                   dx=np.array([dx, dx]))


# ----------------------------------------------------------------------------
# c3: Taylor impact bar against a rigid wall at z = 0
# ----------------------------------------------------------------------------
def taylor_bar(dx: float = 0.105e-3, R: float = 3.8e-3, L: float = 25.4e-3,
               jitter: float = 0.03, v0: float = 200.0, Wcr: float = 300e6,
               seed: int = SEED_BASE + 2, steps: int = 5000) -> Problem:
    rng = np.random.default_rng(seed)
    nr = int(math.ceil(2 * R / dx))
    nz = int(round(L / dx))
    i, j, k = _lattice(nr, nr, nz)
    x = (i + 0.5) * dx - nr * dx / 2
    y = (j + 0.5) * dx - nr * dx / 2
    z = (k + 0.5) * dx
    keep = x * x + y * y < R * R
    lat = np.stack([x[keep], y[keep], z[keep]], axis=1)
    X = _jitter(rng, lat, dx, jitter)
    n = X.shape[0]
    v = np.zeros((n, 3))
    v[:, 2] = -v0
    mat = material(dx, DMG_CL, Wcr=Wcr, has_wall=1, wall_n=(0.0, 0.0, 1.0), wall_d=0.0)
    return Problem("taylor_bar", X, np.full(n, dx ** 3), np.array([0, n], np.int64),
                   [mat], np.full(n, -1, np.int32), [], v, steps=steps, dx=np.array([dx]))


# ----------------------------------------------------------------------------
# c4: GTN plate with a central hole, plane-strain-like tension along x
# ----------------------------------------------------------------------------
def holed_plate(dx: float = 0.125e-3, W: float = 100e-3, H: float = 40e-3, T: float = 2e-3,
                hole_d: float = 5e-3, jitter: float = 0.03, v_max: float = 10.0,
                tau: float = 1e-3, seed: int = SEED_BASE + 3, steps: int = 2000) -> Problem:
    rng = np.random.default_rng(seed)
    nx, ny, nz = int(round(W / dx)), int(round(H / dx)), int(round(T / dx))
    i, j, k = _lattice(nx, ny, nz)
    x = (i + 0.5) * dx - W / 2
    y = (j + 0.5) * dx - H / 2
    z = (k + 0.5) * dx
    keep = x * x + y * y >= (hole_d / 2) ** 2
    lat = np.stack([x[keep], y[keep], z[keep]], axis=1)
    ii = i[keep]
    X = _jitter(rng, lat, dx, jitter)
    n = X.shape[0]
    bc = np.full(n, 2, np.int32)
    bc[ii < 2] = 0
    bc[ii >= nx - 2] = 1
    groups = [bc_group(1 | 4, (-v_max, 0.0, 0.0), tau), bc_group(1 | 4, (v_max, 0.0, 0.0), tau),
              bc_group(4, (0.0, 0.0, 0.0))]
    return Problem("holed_plate", X, np.full(n, dx ** 3), np.array([0, n], np.int64),
                   [material(dx, DMG_GTN)], bc, groups, np.zeros((n, 3)), steps=steps,
                   dx=np.array([dx]))


# ----------------------------------------------------------------------------
# c5: batch of notched bars with uneven particle counts and material scatter
# ----------------------------------------------------------------------------
def batch_counts(n_spec: int = 256, lo: int = 2000, hi: int = 60000) -> np.ndarray:
    return np.random.default_rng(SEED_BASE + 5).integers(lo, hi + 1, n_spec)


def bar_batch(n_spec: int = 256, lo: int = 2000, hi: int = 60000, jitter: float = 0.03,
              v_max: float = 10.0, tau: float = 1e-3, steps: int = 200,
              counts: Optional[np.ndarray] = None) -> Problem:
    if counts is None:
        counts = batch_counts(n_spec, lo, hi)
    vol = notched_bar_volume()
    Xs, bcs, mats, offs, dxs = [], [], [], [0], []
    for s, ns in enumerate(counts):
        rng = np.random.default_rng([SEED_BASE + 5, s])
        dx = (vol / float(ns)) ** (1.0 / 3.0)
        lat, k, nz = _notched_bar_points(dx)
        X = _jitter(rng, lat, dx, jitter)
        b = np.full(X.shape[0], -1, np.int32)
        b[k < 2] = 2 * s
        b[k >= nz - 2] = 2 * s + 1
        scat = rng.uniform(0.8, 1.2, size=6)
        mats.append(material(dx, DMG_JC, A=STEEL["A"] * scat[0], B=STEEL["B"] * scat[1],
                             n=STEEL["n"] * scat[2], D1=JC_DAMAGE["D1"] * scat[3],
                             D2=JC_DAMAGE["D2"] * scat[4], D3=JC_DAMAGE["D3"] * scat[5]))
        Xs.append(X)
        bcs.append(b)
        offs.append(offs[-1] + X.shape[0])
        dxs.append(dx)
    X = np.concatenate(Xs)
    groups = []
    for s in range(len(counts)):
        groups.append(bc_group(4, (0.0, 0.0, -v_max), tau))
        groups.append(bc_group(4, (0.0, 0.0, v_max), tau))
    V0 = np.concatenate([np.full(x.shape[0], d ** 3) for x, d in zip(Xs, dxs)])
    return Problem("bar_batch", X, V0, np.array(offs, np.int64), mats,
                   np.concatenate(bcs), groups, np.zeros((X.shape[0], 3)), steps=steps,
                   dx=np.array(dxs))


# ----------------------------------------------------------------------------
# variants of the generators above that the benchmark times and the full-size
# tests check
# ----------------------------------------------------------------------------
# Voce hardening fitted near the Johnson-Cook curve, implicit return
VOCE_IMPLICIT = dict(flow=FLOW_VOCE, A=792e6, B=510e6, flow_beta=5.0, implicit_return=1)
# artificial particle-velocity damping coefficients (Q1, Q2)
DAMPING = dict(av_q1=1.0, av_q2=2.0)


def with_materials(p: Problem, **over) -> Problem:
    """The problem with every specimen's parameters overridden."""
    mats = [dict(m, **over) for m in p.materials]
    return Problem(p.name, p.X, p.V0, p.spec_offsets, mats, p.bc_group, p.bc_groups, p.v_init,
                   p.steps, p.dx)


def bar_collision_395k() -> Problem:
    """Two bars (R 2.5 mm, 10 mm long, dx 0.1 mm, 395 200 particles) 0.05 mm
    apart, meeting head on at 100 m/s each."""
    return bar_collision(dx=0.1e-3, R=2.5e-3, L=10e-3, gap=0.05e-3, v0=100.0)


def subset(p: Problem, specs) -> Problem:
    """The given specimens of a batch as a problem of their own (group ids remapped)."""
    specs = list(specs)
    Xs, V0s, bcs, offs, groups, mats, dxs = [], [], [], [0], [], [], []
    for s in specs:
        a, b = int(p.spec_offsets[s]), int(p.spec_offsets[s + 1])
        Xs.append(p.X[a:b])
        V0s.append(p.V0[a:b])
        old = p.bc_group[a:b]
        new = np.full(b - a, -1, np.int32)
        for g in sorted(set(old[old >= 0].tolist())):
            new[old == g] = len(groups)
            groups.append(p.bc_groups[g])
        bcs.append(new)
        offs.append(offs[-1] + (b - a))
        mats.append(p.materials[s])
        dxs.append(p.dx[s] if p.dx is not None else 0.0)
    vi = np.concatenate([p.v_init[p.spec_offsets[s]:p.spec_offsets[s + 1]] for s in specs])
    return Problem(p.name + "_subset", np.concatenate(Xs), np.concatenate(V0s),
                   np.array(offs, np.int64), mats, np.concatenate(bcs), groups, vi,
                   steps=p.steps, dx=np.array(dxs))


# ----------------------------------------------------------------------------
# Random per-particle states for one-step parity from an injected state
# ----------------------------------------------------------------------------
def random_state(p: Problem, seed: int, v_scale: float = 2.0, u_scale: float = 2e-6,
                 sig_scale: float = 700e6, frac_failed: float = 0.05,
                 frac_undamaged: float = 0.4) -> Dict[str, np.ndarray]:
    """Seeded random state covering elastic, yielding, damaged and failed
    particles. Arrays are in caller order with the oracle's shapes:
    vectors (n,3), tensors (n,9) row-major, symmetric tensors (n,6) Voigt
    (xx, yy, zz, yz, xz, xy)."""
    rng = np.random.default_rng(seed)
    n = p.n
    st = {}
    st["u"] = rng.uniform(-u_scale, u_scale, (n, 3))
    st["v"] = rng.uniform(-v_scale, v_scale, (n, 3))
    F = np.tile(np.eye(3).ravel(), (n, 1)) + rng.uniform(-0.02, 0.02, (n, 9))
    st["F"] = F
    st["sig"] = rng.uniform(-sig_scale, sig_scale, (n, 6))
    st["eps_p"] = rng.uniform(0.0, 0.6, n)
    st["eps_p_rate"] = np.where(rng.uniform(size=n) < 0.5, 0.0, rng.uniform(0.0, 2e3, n))
    D = rng.uniform(0.0, 0.95, n)
    r = rng.uniform(size=n)
    D[r < frac_undamaged] = 0.0
    D[r > 1.0 - frac_failed] = 1.0
    st["D"] = D
    st["d_init"] = rng.uniform(0.8, 1.11, n)
    st["w_p"] = rng.uniform(0.0, 400e6, n)
    st["f_void"] = rng.uniform(0.0005, 0.27, n)
    st["e"] = rng.uniform(0.0, 50.0, n)
    st["Q"] = rng.uniform(-sig_scale, sig_scale, (n, 9))
    return st
