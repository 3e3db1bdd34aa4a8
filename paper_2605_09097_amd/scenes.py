"""Seeded synthetic scenes for OS-MPM runs.

This module only produces *inputs*: particle positions and initial state,
material tables, grid descriptors on an integer lattice, boundary-layer and
scene-BC markers, and the per-frame boundary-condition parameters.  It holds
none of the method's arithmetic, so the GPU library and the CPU oracle can
both be fed from it.

Geometry follows the paper's numerical examples (Sec. 4): the elastic
inclusion of Sec. 4.3 (matrix square with a circular inclusion, a coarse
domain carrying the matrix outside r = 0.1 and a fine domain carrying the
disc r <= 0.15, overlap 0.1 <= r <= 0.15), the cantilever of Sec. 4.1 split
longitudinally, and a 2D Hertz-type contact of Sec. 4.2 (a half cylinder
pressed onto a block).  Particles sit at the centres of k x k sub-cells of
each grid cell, jittered by up to +-0.1 dx per component; a particle is kept
when its unjittered centre lies in the material region.  Random numbers come
from SplitMix64 (Steele, Lea & Flood 2014) evaluated at counters, so every
scene is a pure function of its seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple, Union

import numpy as np

BC_FIX, BC_TRANSLATE, BC_ROTATE = 0, 1, 2
FLAG_BOUNDARY = 1  # bit 0: Schwarz boundary-layer particle; bit 1+g: scene group g

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state seed + (c + 1) * golden, for each counter c."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, counters) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def stream_seed(seed: int, key: int) -> int:
    """Independent stream per (seed, key): one SplitMix64 draw of the pair."""
    return int(splitmix64(seed * 1000003 + key, np.array([0], dtype=np.uint64))[0])


@dataclass
class DomainSpec:
    """One subdomain: grid on the lattice x_i = (origin_q + i dx_q) h0, particles,
    materials and scene-BC groups (kind, component mask; parameters per frame)."""

    dim: int
    h0: float
    origin_q: List[int]
    dx_q: int
    n_nodes: List[int]
    x: np.ndarray
    v: np.ndarray
    B: np.ndarray
    F: np.ndarray
    mass: np.ndarray
    vol: np.ndarray
    mat: np.ndarray
    flags: np.ndarray
    E: np.ndarray
    nu: np.ndarray
    bc_kind: List[int] = field(default_factory=list)
    bc_mask: List[int] = field(default_factory=list)
    m_ref: float = 1.0
    tau: float = 0.0
    ppc1d: Union[int, Tuple[int, ...]] = 2  # particles per cell, per axis or the same on every axis
    tau_y: Optional[np.ndarray] = None  # von Mises yield stress per material (None: elastic)

    @property
    def dx(self) -> float:
        return self.dx_q * self.h0

    @property
    def n_particles(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "DomainSpec":
        c = DomainSpec(**{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in self.__dict__.items()})
        c.origin_q = list(self.origin_q)
        c.n_nodes = list(self.n_nodes)
        c.bc_kind = list(self.bc_kind)
        c.bc_mask = list(self.bc_mask)
        if self.tau_y is not None:
            c.tau_y = np.array(self.tau_y, dtype=np.float64)
        return c


@dataclass
class Scene:
    """A coarse/fine pair (S may be None for a single-domain run) and its
    time stepping.  bc_params(frame) returns (params_B, params_S), arrays of
    shape (n_groups, 8) with the per-frame scene-BC parameters."""

    name: str
    B: DomainSpec
    S: Optional[DomainSpec]
    dT: float
    M: int
    n_frames: int
    bc_params: Callable[[int], tuple]
    eps_tol: float = 0.0
    meta: dict = field(default_factory=dict)


def _per_axis(ppc1d, dim):
    """Particles per cell along each axis: an int means the same count on
    every axis, a sequence gives one count per axis."""
    if isinstance(ppc1d, (int, np.integer)):
        return (int(ppc1d),) * dim
    out = tuple(int(k) for k in ppc1d)
    if len(out) != dim or min(out) < 1:
        raise ValueError("ppc1d needs %d positive counts" % dim)
    return out


def _sample(dim, inv_dx, lo_cell, hi_cell, ppc1d, region, seed, key, jitter=0.1):
    """Sub-cell centres of cells lo_cell..hi_cell-1 (per axis) kept by region(),
    then jittered.  ppc1d is the count per axis (int or one per axis).
    Returns positions (n, dim) and the unjittered centres."""
    dx = 1.0 / inv_dx
    ppc = _per_axis(ppc1d, dim)
    axes = [np.arange(lo_cell[a], hi_cell[a]) for a in range(dim)]
    subs = [(np.arange(ppc[a]) + 0.5) / ppc[a] for a in range(dim)]
    grids = np.meshgrid(*[(axes[a][:, None] + subs[a][None, :]).ravel() for a in range(dim)], indexing="ij")
    centres = np.stack([g.ravel() for g in grids], axis=1) * dx
    keep = region(centres)
    centres = centres[keep]
    n = centres.shape[0]
    s = stream_seed(seed, key)
    cnt = np.arange(n * dim, dtype=np.uint64)
    jit = (uniform01(s, cnt).reshape(n, dim) * 2.0 - 1.0) * (jitter * dx)
    return centres + jit, centres


def _domain(dim, h0, origin_q, dx_q, n_nodes, x, mat, E, nu, rho, ppc1d, flags, bc_kind, bc_mask,
            m_ref, tau_rel, F0=None):
    n = x.shape[0]
    dx = dx_q * h0
    vol = np.full(n, dx ** dim / math.prod(_per_axis(ppc1d, dim)))
    mass = rho * vol
    F = np.broadcast_to(np.eye(dim), (n, dim, dim)).copy()
    if F0 is not None:
        F[:] = F0
    return DomainSpec(dim=dim, h0=h0, origin_q=list(origin_q), dx_q=int(dx_q), n_nodes=list(n_nodes),
                      x=x, v=np.zeros((n, dim)), B=np.zeros((n, dim, dim)), F=F, mass=mass, vol=vol,
                      mat=mat.astype(np.int32), flags=flags.astype(np.uint8),
                      E=np.asarray(E, dtype=np.float64), nu=np.asarray(nu, dtype=np.float64),
                      bc_kind=list(bc_kind), bc_mask=list(bc_mask), m_ref=m_ref,
                      tau=tau_rel * float(mass.mean()) if n else 0.0, ppc1d=ppc1d)


def inclusion_scene(inv_dx_B=20, inv_dx_S=50, ppc1d=2, r_inc=0.05, E_matrix=1e4, E_inc=1e5,
                    nu=0.3, rho=1000.0, seed=0, dT=1e-3, M=2, n_frames=50, top_disp=0.01,
                    ramp_frames=50, tau_rel=1e-3, eps_tol_rel=1e-9, delta=0.0, loaded=True,
                    clamped=False, name="inclusion"):
    """2D elastic inclusion (Sec. 4.3 geometry).  Coarse grid on [0,1]^2 holding
    the matrix square [0.1,0.9]^2 outside r = 0.1; fine grid on [0.3,0.7]^2
    holding the matrix annulus r_inc < r <= 0.15 and the inclusion r <= r_inc.

    loaded=True: bottom layer clamped, top layer driven down in y (roller in x)
    by top_disp ramped linearly over ramp_frames frames.  clamped=True (with
    loaded=False): the outer particle layer of all four edges is fixed.
    delta > 0 gives the inclusion the eigenstrain F0 = (1 - delta) I of
    Sec. 4.3.
    """
    lat = math.lcm(inv_dx_B, inv_dx_S, 10)
    h0 = 1.0 / lat
    dxq_B, dxq_S = lat // inv_dx_B, lat // inv_dx_S
    c = np.array([0.5, 0.5])
    spB, spS = 1.0 / (inv_dx_B * ppc1d), 1.0 / (inv_dx_S * ppc1d)

    def regB(p):
        r = np.linalg.norm(p - c, axis=1)
        return (p[:, 0] >= 0.1) & (p[:, 0] <= 0.9) & (p[:, 1] >= 0.1) & (p[:, 1] <= 0.9) & (r > 0.1)

    def regS(p):
        return np.linalg.norm(p - c, axis=1) <= 0.15

    nB = inv_dx_B + 1
    xB, _ = _sample(2, inv_dx_B, [0, 0], [inv_dx_B, inv_dx_B], ppc1d, regB, seed, 1)
    s0 = int(round(0.3 * inv_dx_S))
    s1 = int(round(0.7 * inv_dx_S))
    xS, _ = _sample(2, inv_dx_S, [s0, s0], [s1, s1], ppc1d, regS, seed, 2)
    nS = s1 - s0 + 1
    rB = np.linalg.norm(xB - c, axis=1)
    rS = np.linalg.norm(xS - c, axis=1)
    flagsB = np.where(rB < 0.1 + spB, FLAG_BOUNDARY, 0)
    flagsS = np.where(rS > 0.15 - spS, FLAG_BOUNDARY, 0)
    bc_kind, bc_mask = [], []
    if loaded:
        flagsB = flagsB | np.where(xB[:, 1] < 0.1 + spB, 2, 0) | np.where(xB[:, 1] > 0.9 - spB, 4, 0)
        bc_kind, bc_mask = [BC_FIX, BC_TRANSLATE], [0b11, 0b10]
    elif clamped:
        flagsB = flagsB | np.where(_outer_layer(xB, spB), 2, 0)
        bc_kind, bc_mask = [BC_FIX], [0b11]
    matS = (rS <= r_inc).astype(np.int32)
    m_ref = rho / (inv_dx_B ** 2 * ppc1d ** 2)
    F0S = None
    if delta:
        F0S = np.where((matS == 1)[:, None, None], (1.0 - delta) * np.eye(2), np.eye(2))
    B = _domain(2, h0, [0, 0], dxq_B, [nB, nB], xB, np.zeros(len(xB), np.int32), [E_matrix], [nu], rho,
                ppc1d, flagsB, bc_kind, bc_mask, m_ref, tau_rel)
    S = _domain(2, h0, [s0 * dxq_S, s0 * dxq_S], dxq_S, [nS, nS], xS, matS, [E_matrix, E_inc], [nu, nu],
                rho, ppc1d, flagsS, [], [], m_ref, tau_rel, F0=F0S)

    def bc_params(frame):
        pB = np.zeros((max(len(bc_kind), 1), 8))
        if loaded:
            ds = top_disp / ramp_frames if frame < ramp_frames else 0.0
            pB[1, 1] = -ds / dT
        return pB, np.zeros((1, 8))

    return Scene(name=name, B=B, S=S, dT=dT, M=M, n_frames=n_frames, bc_params=bc_params,
                 eps_tol=eps_tol_rel * float(S.mass.mean()),
                 meta={"inv_dx_B": inv_dx_B, "inv_dx_S": inv_dx_S, "r_inc": r_inc, "E_inc": E_inc,
                       "E_matrix": E_matrix, "nu": nu, "ppc1d": ppc1d, "top_disp": top_disp if loaded else 0.0,
                       "ramp_frames": ramp_frames})


@dataclass
class MultiScene:
    """One coarse domain and several disjoint fine domains.  S_union holds the
    fine domains' particles together on one fine grid of the same lattice (a
    single fine domain equivalent to the set).  bc_params(frame) returns
    (params_B, [params_S...])."""

    name: str
    B: DomainSpec
    S: List[DomainSpec]
    S_union: DomainSpec
    dT: float
    M: int
    n_frames: int
    bc_params: Callable[[int], tuple]
    eps_tol: float = 0.0
    meta: dict = field(default_factory=dict)


def two_inclusion_scene(inv_dx_B=20, inv_dx_S=50, ppc1d=2, r_inc=0.04, E_matrix=1e4, E_inc=1e5, nu=0.3,
                        rho=1000.0, seed=0, dT=1e-3, M=2, n_frames=50, top_disp=0.01, ramp_frames=50,
                        tau_rel=1e-3, eps_tol_rel=1e-9, delta=0.0, centres=((0.3, 0.5), (0.7, 0.5)),
                        name="two_inclusions"):
    """Two refined regions in one matrix (several refined subdomains, named as
    future work in the conclusion): the matrix square [0.1,0.9]^2 with
    inclusions r <= r_inc around the two centres (default c1 = (0.3, 0.5),
    c2 = (0.7, 0.5)).  Fine domain i holds the material within r = 0.12 of
    c_i on the box c_i +- 0.16; the coarse domain the matrix outside r = 0.08
    of both centres.  With the default centres the fine regions are 0.16
    apart and meet only the coarse domain; centres closer than 0.24 make the
    fine regions overlap each other (both carry the material of the lens
    between them).  S_union is one fine domain over both regions (their
    particles concatenated when disjoint, the union region sampled once when
    they overlap).  Loaded like inclusion_scene (bottom clamped, top driven
    down)."""
    lat = math.lcm(inv_dx_B, inv_dx_S, 10)
    h0 = 1.0 / lat
    dxq_B, dxq_S = lat // inv_dx_B, lat // inv_dx_S
    cs = [np.array(c, dtype=np.float64) for c in centres]
    R_f, R_h = 0.12, 0.08
    spB, spS = 1.0 / (inv_dx_B * ppc1d), 1.0 / (inv_dx_S * ppc1d)

    def rmin(p):
        return np.minimum(np.linalg.norm(p - cs[0], axis=1), np.linalg.norm(p - cs[1], axis=1))

    def regB(p):
        return (p[:, 0] >= 0.1) & (p[:, 0] <= 0.9) & (p[:, 1] >= 0.1) & (p[:, 1] <= 0.9) & (rmin(p) > R_h)

    nB = inv_dx_B + 1
    xB, _ = _sample(2, inv_dx_B, [0, 0], [inv_dx_B, inv_dx_B], ppc1d, regB, seed, 1)
    flagsB = np.where(rmin(xB) < R_h + spB, FLAG_BOUNDARY, 0)
    flagsB = flagsB | np.where(xB[:, 1] < 0.1 + spB, 2, 0) | np.where(xB[:, 1] > 0.9 - spB, 4, 0)
    bc_kind, bc_mask = [BC_FIX, BC_TRANSLATE], [0b11, 0b10]
    m_ref = rho / (inv_dx_B ** 2 * ppc1d ** 2)
    B = _domain(2, h0, [0, 0], dxq_B, [nB, nB], xB, np.zeros(len(xB), np.int32), [E_matrix], [nu], rho,
                ppc1d, flagsB, bc_kind, bc_mask, m_ref, tau_rel)
    Ss, parts = [], []
    for i, c in enumerate(cs):
        lo = [int(math.floor((c[a] - 0.16) * inv_dx_S + 1e-9)) for a in range(2)]
        hi = [int(math.ceil((c[a] + 0.16) * inv_dx_S - 1e-9)) for a in range(2)]
        xS, _ = _sample(2, inv_dx_S, lo, hi, ppc1d, lambda p, c=c: np.linalg.norm(p - c, axis=1) <= R_f, seed, 2 + i)
        r = np.linalg.norm(xS - c, axis=1)
        flags = np.where(r > R_f - spS, FLAG_BOUNDARY, 0)
        mat = (r <= r_inc).astype(np.int32)
        F0 = np.where((mat == 1)[:, None, None], (1.0 - delta) * np.eye(2), np.eye(2)) if delta else None
        Ss.append(_domain(2, h0, [lo[0] * dxq_S, lo[1] * dxq_S], dxq_S, [hi[0] - lo[0] + 1, hi[1] - lo[1] + 1], xS,
                          mat, [E_matrix, E_inc], [nu, nu], rho, ppc1d, flags, [], [], m_ref, tau_rel, F0=F0))
        parts.append((xS, mat, flags))
    ulo = [int(math.floor((min(c[a] for c in cs) - 0.16) * inv_dx_S + 1e-9)) for a in range(2)]
    uhi = [int(math.ceil((max(c[a] for c in cs) + 0.16) * inv_dx_S - 1e-9)) for a in range(2)]
    if np.linalg.norm(cs[0] - cs[1]) >= 2 * R_f:
        xU = np.concatenate([q[0] for q in parts])
        matU = np.concatenate([q[1] for q in parts])
        flU = np.concatenate([q[2] for q in parts])
    else:
        xU, _ = _sample(2, inv_dx_S, ulo, uhi, ppc1d, lambda p: rmin(p) <= R_f, seed, 4)
        matU = (rmin(xU) <= r_inc).astype(np.int32)
        flU = np.where(rmin(xU) > R_f - spS, FLAG_BOUNDARY, 0)
    F0U = np.where((matU == 1)[:, None, None], (1.0 - delta) * np.eye(2), np.eye(2)) if delta else None
    U = _domain(2, h0, [ulo[0] * dxq_S, ulo[1] * dxq_S], dxq_S, [uhi[0] - ulo[0] + 1, uhi[1] - ulo[1] + 1], xU,
                matU, [E_matrix, E_inc], [nu, nu], rho, ppc1d, flU, [], [], m_ref, tau_rel, F0=F0U)
    # one fixed-point threshold and regulariser for all fine domains (those of the union)
    for S_ in Ss:
        S_.tau = U.tau

    def bc_params(frame):
        pB = np.zeros((2, 8))
        ds = top_disp / ramp_frames if frame < ramp_frames else 0.0
        pB[1, 1] = -ds / dT
        return pB, [np.zeros((1, 8)) for _ in Ss]

    return MultiScene(name=name, B=B, S=Ss, S_union=U, dT=dT, M=M, n_frames=n_frames, bc_params=bc_params,
                      eps_tol=eps_tol_rel * float(U.mass.mean()),
                      meta={"inv_dx_B": inv_dx_B, "inv_dx_S": inv_dx_S, "r_inc": r_inc, "E_inc": E_inc,
                            "E_matrix": E_matrix, "nu": nu, "ppc1d": ppc1d, "top_disp": top_disp,
                            "ramp_frames": ramp_frames})


def _outer_layer(x, sp):
    """Particles within one particle spacing of the edges of [0.1, 0.9]^2."""
    return (x[:, 0] < 0.1 + sp) | (x[:, 0] > 0.9 - sp) | (x[:, 1] < 0.1 + sp) | (x[:, 1] > 0.9 - sp)


def inclusion_single(inv_dx=50, ppc1d=2, r_inc=0.05, E_matrix=1e4, E_inc=1e5, nu=0.3, rho=1000.0,
                     seed=0, dt=1e-3, n_frames=50, top_disp=0.01, ramp_frames=50, delta=0.0,
                     loaded=True, clamped=False, tau_rel=1e-3):
    """Single-domain reference of the inclusion: the whole square [0.1,0.9]^2 on
    one grid (loaded / clamped outer boundary as in inclusion_scene)."""
    lat = math.lcm(inv_dx, 10)
    h0 = 1.0 / lat
    dxq = lat // inv_dx
    c = np.array([0.5, 0.5])
    sp = 1.0 / (inv_dx * ppc1d)

    def reg(p):
        return (p[:, 0] >= 0.1) & (p[:, 0] <= 0.9) & (p[:, 1] >= 0.1) & (p[:, 1] <= 0.9)

    x, _ = _sample(2, inv_dx, [0, 0], [inv_dx, inv_dx], ppc1d, reg, seed, 3)
    r = np.linalg.norm(x - c, axis=1)
    mat = (r <= r_inc).astype(np.int32)
    flags = np.zeros(len(x), np.int64)
    bc_kind, bc_mask = [], []
    if loaded:
        flags = flags | np.where(x[:, 1] < 0.1 + sp, 2, 0) | np.where(x[:, 1] > 0.9 - sp, 4, 0)
        bc_kind, bc_mask = [BC_FIX, BC_TRANSLATE], [0b11, 0b10]
    elif clamped:
        flags = flags | np.where(_outer_layer(x, sp), 2, 0)
        bc_kind, bc_mask = [BC_FIX], [0b11]
    F0 = None
    if delta:
        F0 = np.where((mat == 1)[:, None, None], (1.0 - delta) * np.eye(2), np.eye(2))
    D = _domain(2, h0, [0, 0], dxq, [inv_dx + 1, inv_dx + 1], x, mat, [E_matrix, E_inc], [nu, nu], rho,
                ppc1d, flags, bc_kind, bc_mask, rho / (inv_dx ** 2 * ppc1d ** 2), tau_rel, F0=F0)

    def bc_params(frame):
        p = np.zeros((max(len(bc_kind), 1), 8))
        if loaded:
            ds = top_disp / ramp_frames if frame < ramp_frames else 0.0
            p[1, 1] = -ds / dt
        return p, None

    return Scene(name="inclusion_single", B=D, S=None, dT=dt, M=1, n_frames=n_frames,
                 bc_params=bc_params)


def cantilever_scene(inv_dx=40, ppc1d=3, E=1e5, nu=0.4, rho=1000.0, gravity=-9.81, seed=0, dt=2e-3,
                     n_frames=100, split=True, x0=0.05, x1=0.90, y0=0.40, thick=0.02,
                     left=(0.05, 0.45), right=(0.39, 0.90), tau_rel=1e-3, eps_tol_rel=1e-9):
    """Gravity cantilever of Sec. 4.1: a beam [x0, x1] x [y0, y0 + thick]
    clamped at x = x0.  split=True gives the two overlapping subdomains
    Omega_L = [0.05, 0.45] (coarse role) and Omega_R = [0.39, 0.90] (fine role)
    at identical resolution; split=False the single-domain beam."""
    lat = math.lcm(inv_dx, 100)
    h0 = 1.0 / lat
    dxq = lat // inv_dx
    sp = 1.0 / (inv_dx * ppc1d)
    nodes = [inv_dx + 1, inv_dx + 1]

    def reg(lo, hi):
        return lambda p: (p[:, 0] >= lo) & (p[:, 0] <= hi) & (p[:, 1] >= y0) & (p[:, 1] <= y0 + thick)

    m_ref = rho / (inv_dx ** 2 * ppc1d ** 2)
    if not split:
        x, _ = _sample(2, inv_dx, [0, 0], [inv_dx, inv_dx], ppc1d, reg(x0, x1), seed, 4, jitter=0.0)
        flags = np.where(x[:, 0] < x0 + sp, 2, 0)
        D = _domain(2, h0, [0, 0], dxq, nodes, x, np.zeros(len(x), np.int32), [E], [nu], rho, ppc1d,
                    flags, [BC_FIX], [0b11], m_ref, tau_rel)
        return Scene(name="cantilever_single", B=D, S=None, dT=dt, M=1, n_frames=n_frames,
                     bc_params=lambda f: (np.zeros((1, 8)), None), meta={"gravity": gravity})
    xL, _ = _sample(2, inv_dx, [0, 0], [inv_dx, inv_dx], ppc1d, reg(*left), seed, 4, jitter=0.0)
    xR, _ = _sample(2, inv_dx, [0, 0], [inv_dx, inv_dx], ppc1d, reg(*right), seed, 5, jitter=0.0)
    flL = np.where(xL[:, 0] < x0 + sp, 2, 0) | np.where(xL[:, 0] > left[1] - sp, FLAG_BOUNDARY, 0)
    flR = np.where(xR[:, 0] < right[0] + sp, FLAG_BOUNDARY, 0)
    L = _domain(2, h0, [0, 0], dxq, nodes, xL, np.zeros(len(xL), np.int32), [E], [nu], rho, ppc1d, flL,
                [BC_FIX], [0b11], m_ref, tau_rel)
    R = _domain(2, h0, [0, 0], dxq, nodes, xR, np.zeros(len(xR), np.int32), [E], [nu], rho, ppc1d, flR,
                [], [], m_ref, tau_rel)
    return Scene(name="cantilever_dual", B=L, S=R, dT=dt, M=1, n_frames=n_frames,
                 bc_params=lambda f: (np.zeros((1, 8)), np.zeros((1, 8))),
                 eps_tol=eps_tol_rel * float(R.mass.mean()), meta={"gravity": gravity})


def hertz_scene(inv_dx_B=32, inv_dx_S=128, ppc1d=2, R=0.5, E_cyl=1e5, E_block=1e6, nu=0.3, rho=1000.0,
                seed=0, dT=1e-3, M=4, n_frames=100, plate_disp=0.005, ramp_frames=None, tau_rel=1e-3,
                eps_tol_rel=1e-9, fine_box=((1.7, 2.3), (0.85, 1.15)), band=0.05):
    """2D Hertz-type contact (Sec. 4.2 setting): an elastic half-cylinder of
    radius R centred at (2, 1.5) (its lower half) resting on a block [0,4]x[0,1],
    pressed down by a rigid plate on its flat top face.  The fine domain carries
    all material inside fine_box; the coarse domain carries all material outside
    fine_box shrunk by band (overlap band of width band)."""
    lat = math.lcm(inv_dx_B, inv_dx_S, 100)
    h0 = 1.0 / lat
    ramp_frames = ramp_frames or n_frames
    c = np.array([2.0, 1.5])
    (fx0, fx1), (fy0, fy1) = fine_box

    def material(p):
        block = (p[:, 0] >= 0.0) & (p[:, 0] <= 4.0) & (p[:, 1] >= 0.0) & (p[:, 1] <= 1.0)
        cyl = (np.linalg.norm(p - c, axis=1) <= R) & (p[:, 1] <= c[1]) & (p[:, 1] > 1.0)
        return block | cyl

    def in_box(p, shrink):
        return ((p[:, 0] >= fx0 + shrink) & (p[:, 0] <= fx1 - shrink) & (p[:, 1] >= fy0 + shrink)
                & (p[:, 1] <= fy1 - shrink))

    regB = lambda p: material(p) & ~in_box(p, band)
    regS = lambda p: material(p) & in_box(p, 0.0)
    pad = 2
    nxB, nyB = 4 * inv_dx_B + 1 + 2 * pad, int(round(2.0 * inv_dx_B)) + 1 + 2 * pad
    oB = -pad * (lat // inv_dx_B)
    xB, _ = _sample(2, inv_dx_B, [0, 0], [4 * inv_dx_B, 2 * inv_dx_B], ppc1d, regB, seed, 6)
    sx0, sx1 = int(round(fx0 * inv_dx_S)), int(round(fx1 * inv_dx_S))
    sy0, sy1 = int(round(fy0 * inv_dx_S)), int(round(fy1 * inv_dx_S))
    xS, _ = _sample(2, inv_dx_S, [sx0, sy0], [sx1, sy1], ppc1d, regS, seed, 7)
    spB, spS = 1.0 / (inv_dx_B * ppc1d), 1.0 / (inv_dx_S * ppc1d)

    def dist_out(p, shrink):
        """Distance from points outside the box (shrunk by shrink) to the box."""
        ex = np.maximum.reduce([(fx0 + shrink) - p[:, 0], p[:, 0] - (fx1 - shrink), np.zeros(len(p))])
        ey = np.maximum.reduce([(fy0 + shrink) - p[:, 1], p[:, 1] - (fy1 - shrink), np.zeros(len(p))])
        return np.hypot(ex, ey)

    def dist_in(p):
        """Distance from points inside the fine box to its edge."""
        return np.minimum(np.minimum(p[:, 0] - fx0, fx1 - p[:, 0]), np.minimum(p[:, 1] - fy0, fy1 - p[:, 1]))

    matB = (xB[:, 1] > 1.0).astype(np.int32)
    matS = (xS[:, 1] > 1.0).astype(np.int32)
    flB = np.where(dist_out(xB, band) < spB, FLAG_BOUNDARY, 0)
    flS = np.where(dist_in(xS) < spS, FLAG_BOUNDARY, 0)
    flB = flB | np.where(xB[:, 1] < spB, 2, 0) | np.where((xB[:, 1] > c[1] - spB) & (matB == 1), 4, 0)
    m_ref = rho / (inv_dx_B ** 2 * ppc1d ** 2)
    B = _domain(2, h0, [oB, oB], lat // inv_dx_B, [nxB, nyB], xB, matB, [E_block, E_cyl], [nu, nu], rho,
                ppc1d, flB, [BC_FIX, BC_TRANSLATE], [0b11, 0b10], m_ref, tau_rel)
    oS = [(sx0 - pad) * (lat // inv_dx_S), (sy0 - pad) * (lat // inv_dx_S)]
    S = _domain(2, h0, oS, lat // inv_dx_S, [sx1 - sx0 + 1 + 2 * pad, sy1 - sy0 + 1 + 2 * pad], xS, matS,
                [E_block, E_cyl], [nu, nu], rho, ppc1d, flS, [], [], m_ref, tau_rel)

    def bc_params(frame):
        pB = np.zeros((2, 8))
        ds = plate_disp / ramp_frames if frame < ramp_frames else 0.0
        pB[1, 1] = -ds / dT
        return pB, np.zeros((1, 8))

    return Scene(name="hertz", B=B, S=S, dT=dT, M=M, n_frames=n_frames, bc_params=bc_params,
                 eps_tol=eps_tol_rel * float(S.mass.mean()), meta={"R": R})


def fold_scene(inv_dx_B=100, inv_dx_S=400, ppc1d=2, length=1.0, width=0.2, thick=0.02, E=5e5, nu=0.35,
               rho=1000.0, seed=0, dT=2e-3, M=4, n_frames=500, angle=math.pi, hinge_x=0.5,
               fine_box=((0.4, 0.6), (-0.02, 0.22), (-0.02, 0.04)), band=0.06, margin=0.05, tau_rel=1e-3,
               eps_tol_rel=1e-9, name="fold"):
    """3D folding slab: [0,length] x [0,width] x [0,thick], the layer of
    particles within one spacing of x = 0 clamped, the layer at x = length
    turned rigidly by `angle` about the axis through (hinge_x, ., thick/2)
    along -y (the free end lifts) at a constant rate over n_frames frames.
    The fine domain carries the material inside fine_box; the coarse domain
    the material outside fine_box shrunk by band along x.  The coarse grid covers the
    half circle the free end sweeps, the fine grid the band its free half
    sweeps; both grids extend a further `margin` along x and below the slab,
    where the soft slab's own motion (the stretch towards the lifted end, the
    sag between the clamp and the hinge) carries material past the box and
    the sweep."""
    lat = math.lcm(inv_dx_B, inv_dx_S, 100)
    h0 = 1.0 / lat
    (fx0, fx1), (fy0, fy1), (fz0, fz1) = fine_box

    def slab(p):
        return ((p[:, 0] >= 0.0) & (p[:, 0] <= length) & (p[:, 1] >= 0.0) & (p[:, 1] <= width)
                & (p[:, 2] >= 0.0) & (p[:, 2] <= thick))

    # The coarse domain's hole is the fine box shrunk by `band` along x only:
    # the box spans the slab's whole width and thickness, so its y and z
    # faces carry no interface and the overlap width is the band along x.
    # Default 0.06 (six coarse cells, like the inclusion's overlap of eight):
    # the Schwarz contraction improves with the overlap width (Sec. 2.3);
    # measured on the first frames, 26 iterations per frame at 0.02, 9 at
    # 0.04 and 6 at 0.06.
    def in_box(p, sh):
        return ((p[:, 0] >= fx0 + sh) & (p[:, 0] <= fx1 - sh) & (p[:, 1] >= fy0) & (p[:, 1] <= fy1)
                & (p[:, 2] >= fz0) & (p[:, 2] <= fz1))

    regB = lambda p: slab(p) & ~in_box(p, band)
    regS = lambda p: slab(p) & in_box(p, 0.0)
    ncx, ncy, ncz = int(round(length * inv_dx_B)), int(round(width * inv_dx_B)), max(1, int(round(thick * inv_dx_B)))
    xB, _ = _sample(3, inv_dx_B, [0, 0, 0], [ncx, ncy, ncz], ppc1d, regB, seed, 8)
    sx = [int(round(fx0 * inv_dx_S)), int(round(fx1 * inv_dx_S))]
    sy = [int(round(fy0 * inv_dx_S)), int(round(fy1 * inv_dx_S))]
    sz = [int(round(fz0 * inv_dx_S)), int(round(fz1 * inv_dx_S))]
    xS, _ = _sample(3, inv_dx_S, [max(sx[0], 0), max(sy[0], 0), max(sz[0], 0)],
                    [sx[1], sy[1], sz[1]], ppc1d, regS, seed, 9)
    spB, spS = 1.0 / (inv_dx_B * ppc1d), 1.0 / (inv_dx_S * ppc1d)

    def dist_out(p, sh):
        e = [np.maximum.reduce([(lo + (sh if a == 0 else 0.0)) - p[:, a], p[:, a] - (hi - (sh if a == 0 else 0.0)),
                                np.zeros(len(p))])
             for a, (lo, hi) in enumerate(fine_box)]
        return np.sqrt(e[0] ** 2 + e[1] ** 2 + e[2] ** 2)

    def dist_in(p):
        return np.min([np.minimum(p[:, a] - lo, hi - p[:, a]) for a, (lo, hi) in enumerate(fine_box)], axis=0)

    flB = np.where(dist_out(xB, band) < spB, FLAG_BOUNDARY, 0)
    flB = flB | np.where(xB[:, 0] < spB, 2, 0) | np.where(xB[:, 0] > length - spB, 4, 0)
    flS = np.where(dist_in(xS) < spS, FLAG_BOUNDARY, 0)
    m_ref = rho / (inv_dx_B ** 3 * ppc1d ** 3)
    pad = 3
    reach = length - hinge_x
    cB = lat // inv_dx_B
    mB, mS = int(math.ceil(margin * inv_dx_B)), int(math.ceil(margin * inv_dx_S))
    lo = [-pad - mB, -pad, -pad - mB]
    hi = [ncx + pad + mB, ncy + pad, int(math.ceil((thick / 2 + reach) * inv_dx_B)) + pad]
    B = _domain(3, h0, [l * cB for l in lo], cB, [hi[a] - lo[a] + 1 for a in range(3)], xB,
                np.zeros(len(xB), np.int32), [E], [nu], rho, ppc1d, flB, [BC_FIX, BC_ROTATE], [0b111, 0b111],
                m_ref, tau_rel)
    cS = lat // inv_dx_S
    loS = [sx[0] - pad - mS, sy[0] - pad, sz[0] - pad - mS]
    # the fine grid also covers the quarter circle that the free half of the
    # fine box sweeps about the hinge axis as the end turns up to 90 degrees
    # (and past it, down again), so fine particles stay inside their grid
    sweep_z = int(math.ceil((thick / 2 + math.hypot(fx1 - hinge_x, thick / 2)) * inv_dx_S))
    hiS = [sx[1] + pad + mS, sy[1] + pad, max(sz[1], sweep_z) + pad]
    S = _domain(3, h0, [l * cS for l in loS], cS, [hiS[a] - loS[a] + 1 for a in range(3)], xS,
                np.zeros(len(xS), np.int32), [E], [nu], rho, ppc1d, flS, [], [], m_ref, tau_rel)
    omega = angle / (n_frames * dT)

    def bc_params(frame):
        pB = np.zeros((2, 8))
        pB[1, :7] = [hinge_x, 0.0, thick / 2, 0.0, -1.0, 0.0, omega if frame < n_frames else 0.0]
        return pB, np.zeros((1, 8))

    return Scene(name=name, B=B, S=S, dT=dT, M=M, n_frames=n_frames, bc_params=bc_params,
                 eps_tol=eps_tol_rel * float(S.mass.mean()) if len(xS) else 0.0,
                 meta={"inv_dx_B": inv_dx_B, "inv_dx_S": inv_dx_S})


def hinge_scene(cells_B=2, cells_S=6, thick=0.003, length=0.09, width=0.06, hinge=0.01, transition=3e-4,
                E_stiff=1e5, E_soft=1e3, nu=0.4, rho=1000.0, n_bins=4, ppc1d=2, seed=0, dT=5e-4, M=2,
                n_frames=400, margin=0.006, band=0.0045, pad=3, tau_rel=1e-3, eps_tol_rel=1e-9, name="hinge"):
    """The three-dimensional showcase of Sec. 4.4: a thin structure
    [0,thick] x [0,length] x [0,width] (0.3 x 9 x 6 cm) made of two stiff
    panels (E_stiff = 100 kPa) joined by a compliant hinge (E_soft = 1 kPa),
    nu = 0.4, with a linear transition of the modulus over `transition`
    (0.03 cm) on either side of the hinge; particles in the transition take
    one of n_bins intermediate moduli by position.  The paper gives neither
    the hinge width, the loading nor the coarse resolution; readings: a
    hinge band of width `hinge` across the middle of the length; the end
    layer y < spacing clamped and the end layer y > length - spacing turned
    rigidly by 180 degrees over n_frames about the z-parallel axis through
    (thick/2 + hinge/pi, length/2), so that the hinge closes into a half
    circle of its own length and the panels end parallel; the fine domain
    (cells_S cells through the thickness) carries all material within
    hinge/2 + transition + margin of the hinge centre, the coarse domain
    (cells_B cells through the thickness) the rest, overlapping by `band`
    (three coarse cells by default: the Schwarz contraction improves with
    the overlap width, Sec. 2.3; measured on the first frames, 70 iterations
    per frame at one coarse cell and a 3 mm margin, 20 at three cells and
    6 mm).  Both grids sit on one lattice of pitch thick / lcm(cells_B,
    cells_S).  ppc1d: particles per cell, per axis or the same on every
    axis."""
    lat = math.lcm(cells_B, cells_S)
    h0 = thick / lat
    dqB, dqS = lat // cells_B, lat // cells_S
    dxB, dxS = dqB * h0, dqS * h0
    yc = 0.5 * length
    half_f = 0.5 * hinge + transition + margin
    Rb = hinge / math.pi
    cx = 0.5 * thick + Rb

    def solid(p):
        return ((p[:, 0] >= 0.0) & (p[:, 0] <= thick) & (p[:, 1] >= 0.0) & (p[:, 1] <= length)
                & (p[:, 2] >= 0.0) & (p[:, 2] <= width))

    regS = lambda p: solid(p) & (np.abs(p[:, 1] - yc) <= half_f)
    regB = lambda p: solid(p) & (np.abs(p[:, 1] - yc) > half_f - band)

    def materials(y):
        """Material index by distance from the hinge centre: 0 stiff, 1 soft,
        2 .. 1 + n_bins the transition from soft to stiff."""
        d = np.abs(y - yc) - 0.5 * hinge
        k = np.floor(d / transition * n_bins).astype(np.int64)
        return np.where(d <= 0.0, 1, np.where(k >= n_bins, 0, 2 + np.clip(k, 0, n_bins - 1))).astype(np.int32)

    E = [E_stiff, E_soft] + [E_soft + (E_stiff - E_soft) * (k + 0.5) / n_bins for k in range(n_bins)]
    nus = [nu] * len(E)
    ncx, ncy, ncz = (int(round(thick / dxB)), int(round(length / dxB)), int(round(width / dxB)))
    xB, cB = _sample(3, 1.0 / dxB, [0, 0, 0], [ncx, ncy, ncz], ppc1d, regB, seed, 10)
    sy0 = int(math.floor((yc - half_f) / dxS))
    sy1 = int(math.ceil((yc + half_f) / dxS))
    nsx, nsz = int(round(thick / dxS)), int(round(width / dxS))
    xS, cS = _sample(3, 1.0 / dxS, [0, sy0, 0], [nsx, sy1, nsz], ppc1d, regS, seed, 11)
    ppc = _per_axis(ppc1d, 3)
    spB, spS = dxB / ppc[1], dxS / ppc[1]
    flB = np.where(np.abs(cB[:, 1] - yc) < half_f - band + spB, FLAG_BOUNDARY, 0)
    flB = flB | np.where(cB[:, 1] < spB, 2, 0) | np.where(cB[:, 1] > length - spB, 4, 0)
    flS = np.where(np.abs(cS[:, 1] - yc) > half_f - spS, FLAG_BOUNDARY, 0)
    m_ref = rho * dxB ** 3 / math.prod(ppc)
    # coarse grid: the half disc the free end sweeps about the fold axis
    reach = math.hypot(Rb, yc)
    loB = [-pad, -pad, -pad]
    hiB = [int(math.ceil((cx + reach) / dxB)) + pad, ncy + pad, ncz + pad]
    B = _domain(3, h0, [l * dqB for l in loB], dqB, [hiB[a] - loB[a] + 1 for a in range(3)], xB,
                materials(cB[:, 1]), E, nus, rho, ppc1d, flB, [BC_FIX, BC_ROTATE], [0b111, 0b111], m_ref, tau_rel)
    # fine grid: the hinge band and the half disc its free side sweeps
    reachS = math.hypot(Rb, half_f)
    loS = [-pad, int(math.floor((yc - reachS) / dxS)) - pad, -pad]
    hiS = [int(math.ceil((cx + reachS) / dxS)) + pad, int(math.ceil((yc + reachS) / dxS)) + pad, nsz + pad]
    S = _domain(3, h0, [l * dqS for l in loS], dqS, [hiS[a] - loS[a] + 1 for a in range(3)], xS,
                materials(cS[:, 1]), E, nus, rho, ppc1d, flS, [], [], m_ref, tau_rel)
    omega = math.pi / (n_frames * dT)

    def bc_params(frame):
        pB = np.zeros((2, 8))
        pB[1, :7] = [cx, yc, 0.5 * width, 0.0, 0.0, -1.0, omega if frame < n_frames else 0.0]
        return pB, np.zeros((1, 8))

    return Scene(name=name, B=B, S=S, dT=dT, M=M, n_frames=n_frames, bc_params=bc_params,
                 eps_tol=eps_tol_rel * float(S.mass.mean()) if len(xS) else 0.0,
                 meta={"cells_B": cells_B, "cells_S": cells_S, "hinge": hinge, "fold_axis": (cx, yc)})


def translation_scene(inv_dx_B=20, inv_dx_S=50, velocity=(0.3, -0.2), ppc1d=2, seed=0, dT=1e-3, M=2,
                      E=1e4, nu=0.3):
    """The inclusion geometry with no scene BCs and a uniform initial velocity:
    a rigid translation, which the coupled method must reproduce exactly."""
    sc = inclusion_scene(inv_dx_B, inv_dx_S, ppc1d=ppc1d, E_matrix=E, E_inc=E, nu=nu, seed=seed, dT=dT,
                         M=M, loaded=False, name="translation")
    for D in (sc.B, sc.S):
        D.v[:] = np.asarray(velocity)
    return sc


# ---------------------------------------------------------------------------
# Benchmark workloads (the paper's inclusion example at the resolutions used
# for measurement)
# ---------------------------------------------------------------------------

# Misfit of the inclusion particles, F0 = (1 - delta) I (Sec. 4.3); the paper
# does not give its value.
INCLUSION_DELTA = 0.01


def workload(name: str, seed: int = 0) -> Scene:
    if name == "inclusion_tiny":
        return inclusion_scene(20, 50, seed=seed, n_frames=50, delta=INCLUSION_DELTA, name=name)
    if name == "inclusion_refined":
        return inclusion_scene(160, 400, seed=seed, n_frames=200, delta=INCLUSION_DELTA, name=name)
    if name == "hertz":
        return hertz_scene(128, 512, ppc1d=3, seed=seed, M=4, n_frames=400)
    if name == "fold":
        return fold_scene(seed=seed)
    if name == "hinge":
        return hinge_scene(seed=seed)
    if name == "hinge_paper":
        # Sec. 4.4 at its own resolution: h = 0.3 cm / 54 = 5.6e-3 cm in the
        # fine domain and 4 particles per cell (2 x 2 across the thickness and
        # along the length, one layer along the fold axis); the coarse domain
        # is 3x coarser, the ratio of the reduced hinge.
        return hinge_scene(cells_B=18, cells_S=54, ppc1d=(2, 2, 1), seed=seed, name=name)
    if name == "hinge_tiny":
        return hinge_scene(cells_B=1, cells_S=2, length=0.03, width=0.012, hinge=0.006, margin=0.002, band=0.002,
                           n_frames=40, seed=seed, name=name)
    if name == "fold_tiny":
        return fold_scene(20, 40, thick=0.1, fine_box=((0.35, 0.65), (-0.05, 0.25), (-0.05, 0.15)), band=0.05,
                          dT=2e-3, M=2, n_frames=50, seed=seed, name=name)
    raise KeyError(name)


def batch_scene(s: int, E_override: Optional[float] = None) -> Scene:
    """Scene s of the batched family: inclusion radius U(0.03, 0.08), inclusion E
    log-uniform in [2e4, 2e5], coarse dx in {1/80, 1/120, 1/160} and fine dx in
    {1/200, 1/300, 1/400}, drawn from SplitMix64 with seed s."""
    u = uniform01(stream_seed(s, 99), np.arange(4, dtype=np.uint64))
    r_inc = 0.03 + 0.05 * u[0]
    E_inc = math.exp(math.log(2e4) + (math.log(2e5) - math.log(2e4)) * u[1])
    invB = [80, 120, 160][min(int(u[2] * 3), 2)]
    invS = [200, 300, 400][min(int(u[3] * 3), 2)]
    if E_override is not None:
        E_inc = E_override
    sc = inclusion_scene(invB, invS, r_inc=r_inc, E_inc=E_inc, seed=s, n_frames=100, delta=INCLUSION_DELTA,
                         name="batch%d" % s)
    sc.meta.update({"seed": s})
    return sc


def batch_target_E(s: int) -> float:
    """Inclusion Young's modulus of the target run of batched scene s: drawn
    log-uniform in [2e4, 2e5] like the scene's own, from seed 1000 + s."""
    u = uniform01(stream_seed(1000 + s, 99), np.arange(4, dtype=np.uint64))
    return math.exp(math.log(2e4) + (math.log(2e5) - math.log(2e4)) * u[1])


def top_edge_target(sc: Scene, n_frames: int, seed: int = 0):
    """Seeded target of the top-edge displacement loss of an inclusion scene:
    the coarse particles of the driven top layer (scene group 1) and target
    positions after n_frames, x0 + (0, -drive displacement) plus a seeded
    offset of up to 1e-3 coarse cells per component.  Returns (indices into
    the coarse particle arrays, target positions [k][2])."""
    idx = np.nonzero(sc.B.flags & 4)[0]
    x0 = np.asarray(sc.B.x)[idx]
    ramp = sc.meta.get("ramp_frames", 1)
    disp = sc.meta.get("top_disp", 0.0) * min(n_frames, ramp) / ramp
    dxB = 1.0 / sc.meta.get("inv_dx_B", 1)
    jit = uniform01(stream_seed(seed, 77), np.arange(2 * len(idx), dtype=np.uint64)).reshape(-1, 2) - 0.5
    target = x0 + np.array([0.0, -disp]) + 2e-3 * dxB * jit
    return idx, target
