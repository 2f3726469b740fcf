"""Seeded synthetic inputs: curvilinear grids and initial flow states.

This module builds the numbers that both the GPU library and the CPU checker consume:
grid-point coordinates (with a 6-deep halo) and the conserved state
Q = (rho, rho u, rho v, rho w, e) on the 3-deep-halo box.  It holds none of the
discretisation: no metrics, fluxes, interpolation or time stepping.

Units follow the paper's nondimensionalisation (Sec. 2, Eq 1): rho_inf = 1, sound speed
c_inf = 1, so T = gamma p / rho has T_inf = 1 and p_inf = 1/gamma; velocities are in
units of c_inf, so a Mach number is a speed.

Layouts (C order, float64):
  coordinates  xyz[3][nk+12][nj+12][ni+12]   (x, y, z planes, halo 6)
  state        Q[5][nk+6][nj+6][ni+6]         (halo 3)
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

GAMMA = 1.4
PRANDTL = 0.71
SUTHERLAND = 110.4 / 288.15
WENO_EPS = 1e-6
HALO = 3
CHALO = 6

# face kinds, faces ordered (i-, i+, j-, j+, k-, k+)
BC_PERIODIC, BC_INTERFACE, BC_WALL, BC_FARFIELD = 0, 1, 2, 3


@dataclasses.dataclass
class Block:
    """One structured block: sizes, coordinates, initial state and face kinds."""

    ni: int
    nj: int
    nk: int
    xyz: np.ndarray
    q: np.ndarray
    bc: Tuple[int, int, int, int, int, int] = (0, 0, 0, 0, 0, 0)

    @property
    def points(self) -> int:
        return self.ni * self.nj * self.nk


@dataclasses.dataclass
class Interface:
    """A 1-to-1 face connection with identity orientation of the tangential indices."""

    block_a: int
    face_a: int
    block_b: int
    face_b: int


@dataclasses.dataclass
class Workload:
    name: str
    blocks: List[Block]
    interfaces: List[Interface]
    gamma: float = GAMMA
    mach: float = 0.5
    reynolds: float = 1000.0
    prandtl: float = PRANDTL
    suth: float = SUTHERLAND
    eps: float = WENO_EPS
    viscous: bool = True
    cfl: float = 0.5
    steps: int = 10
    t_wall: float = 1.0
    qinf: Tuple[float, float, float, float, float] = (1.0, 0.0, 0.0, 0.0, 1.0 / (GAMMA * (GAMMA - 1.0)))
    description: str = ""

    @property
    def points(self) -> int:
        return sum(b.points for b in self.blocks)


# ----------------------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------------------
def conserved(rho, u, v, w, p, gamma=GAMMA) -> np.ndarray:
    """Stack (rho, rho u, rho v, rho w, e) with e = p/(gamma-1) + rho |u|^2 / 2 (Eq 1)."""
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, e]).astype(np.float64)


def index_grid(ni, nj, nk, halo=CHALO):
    """Integer index arrays (k, j, i) over the box with the given halo, shape (nk+2h, nj+2h, ni+2h)."""
    k = np.arange(-halo, nk + halo, dtype=np.float64)
    j = np.arange(-halo, nj + halo, dtype=np.float64)
    i = np.arange(-halo, ni + halo, dtype=np.float64)
    return np.meshgrid(k, j, i, indexing="ij")


def state_coords(xyz: np.ndarray) -> np.ndarray:
    """Coordinates on the halo-3 state box, sliced from the halo-6 coordinate box."""
    d = CHALO - HALO
    return xyz[:, d:-d, d:-d, d:-d]


def wrap_halo(a: np.ndarray, axes=(0, 1, 2), halo=HALO) -> np.ndarray:
    """Fill the halo of (nvar, nk+2h, nj+2h, ni+2h) by periodic copies along the given axes."""
    out = a.copy()
    for ax in axes:
        arr_ax = ax + 1
        n = out.shape[arr_ax] - 2 * halo
        src = np.arange(-halo, n + halo) % n + halo
        out = np.take(out, src, axis=arr_ax)
    return out


# ----------------------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------------------
def wavy_grid(n: int, length: float = 1.0, amp: float = 0.1, nj: Optional[int] = None,
              nk: Optional[int] = None, kz: float = 1.0) -> np.ndarray:
    """Triply periodic wavy grid x = X + a sin(2 pi Y/L) sin(2 pi Z/L) and its cyclic images.

    X, Y, Z are the index coordinates scaled to [0, L); the halo holds the unwrapped
    periodic images (X continues linearly beyond the box).
    """
    ni = n
    nj = n if nj is None else nj
    nk = n if nk is None else nk
    K, J, I = index_grid(ni, nj, nk)
    X = I * (length / ni)
    Y = J * (length / nj)
    Z = K * (length / nk)
    w = 2.0 * math.pi / length
    x = X + amp * np.sin(w * Y) * np.sin(kz * w * Z)
    y = Y + amp * np.sin(kz * w * Z) * np.sin(w * X)
    z = Z + amp * np.sin(w * X) * np.sin(w * Y)
    return np.ascontiguousarray(np.stack([x, y, z]))


def cartesian_grid(ni: int, nj: int, nk: int, lx=1.0, ly=1.0, lz=1.0) -> np.ndarray:
    K, J, I = index_grid(ni, nj, nk)
    return np.ascontiguousarray(np.stack([I * (lx / ni), J * (ly / nj), K * (lz / nk)]))


# ----------------------------------------------------------------------------------------
# flows
# ----------------------------------------------------------------------------------------
def isentropic_vortex(x, y, x0, y0, radius, swirl, uinf, gamma=GAMMA, period=1.0):
    """Isentropic vortex in radial equilibrium, periodic images by nearest-image distance.

    Swirl speed u_theta = swirl (r/R) exp((1 - r^2/R^2)/2) (peak `swirl` at r = R) on top of
    a uniform stream uinf along x; T = 1 - (gamma-1) swirl^2 exp(1 - r^2/R^2) / 2,
    rho = T^(1/(gamma-1)), p = rho^gamma / gamma.  Returns (rho, u, v, w, p).
    """
    dx = x - x0
    dy = y - y0
    if period:
        dx = dx - period * np.round(dx / period)
        dy = dy - period * np.round(dy / period)
    r2 = (dx * dx + dy * dy) / (radius * radius)
    g = np.exp(0.5 * (1.0 - r2))
    u = uinf - swirl * (dy / radius) * g
    v = swirl * (dx / radius) * g
    T = 1.0 - 0.5 * (gamma - 1.0) * swirl * swirl * g * g
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma / gamma
    return rho, u, v, np.zeros_like(u), p


def taylor_green(x, y, z, v0, gamma=GAMMA):
    """Taylor-Green vortex on the 2 pi cube at T = 1: returns (rho, u, v, w, p)."""
    u = v0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -v0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = 1.0 / gamma + (v0 * v0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = gamma * p  # T = gamma p / rho = 1
    return rho, u, v, w, p


def uniform_state(shape, rho=1.0, u=0.0, v=0.0, w=0.0, p=1.0 / GAMMA, gamma=GAMMA):
    one = np.ones(shape)
    return conserved(rho * one, u * one, v * one, w * one, p * one, gamma)


# ----------------------------------------------------------------------------------------
# the benchmark / parity workloads
# ----------------------------------------------------------------------------------------
def periodic_workload(name, xyz, q_interior_fn, **kw) -> Workload:
    ni, nj, nk = xyz.shape[3] - 2 * CHALO, xyz.shape[2] - 2 * CHALO, xyz.shape[1] - 2 * CHALO
    q = wrap_halo(q_interior_fn(state_coords(xyz)))
    blk = Block(ni, nj, nk, xyz, np.ascontiguousarray(q))
    return Workload(name, [blk], [], **kw)


def vortex_wavy(n: int = 32, seed: Optional[int] = 1, noise: float = 1e-3, viscous: bool = True,
                mach: float = 0.5, steps: int = 10, nj=None, nk=None, amp=0.1) -> Workload:
    """Single periodic block on the unit wavy grid with an isentropic vortex.

    Mach 0.5 stream along x, vortex centre (0.5, 0.5), radius 0.08, peak swirl 0.2,
    Re = 1000; seeded U(-noise, noise) added to u, v, w on interior points.
    """
    xyz = wavy_grid(n, 1.0, amp, nj=nj, nk=nk)

    def init(c):
        x, y = c[0], c[1]
        rho, u, v, w, p = isentropic_vortex(x, y, 0.5, 0.5, 0.08, 0.2, mach)
        if seed is not None and noise > 0.0:
            rng = np.random.default_rng(seed)
            u = u + rng.uniform(-noise, noise, size=u.shape)
            v = v + rng.uniform(-noise, noise, size=u.shape)
            w = w + rng.uniform(-noise, noise, size=u.shape)
        return conserved(rho, u, v, w, p)

    return periodic_workload(f"vortex_wavy_{n}", xyz, init, mach=mach, reynolds=1000.0,
                             viscous=viscous, steps=steps,
                             description=f"{n}^3 periodic wavy grid, isentropic vortex Mach {mach}")


def taylor_green_wavy(n: int = 256, seed: Optional[int] = 2, noise: float = 1e-4, steps: int = 100,
                      amp: float = 0.05) -> Workload:
    """Single periodic block on the 2 pi cube with a sinusoidal grid perturbation.

    Taylor-Green vortex at Mach 0.1 (V0 = 0.1), Re = 1600, T = 1, with seeded N(0, noise^2)
    added to u, v, w.
    """
    xyz = wavy_grid(n, 2.0 * math.pi, amp)

    def init(c):
        rho, u, v, w, p = taylor_green(c[0], c[1], c[2], 0.1)
        if seed is not None and noise > 0.0:
            rng = np.random.default_rng(seed)
            u = u + rng.normal(0.0, noise, size=u.shape)
            v = v + rng.normal(0.0, noise, size=u.shape)
            w = w + rng.normal(0.0, noise, size=u.shape)
        return conserved(rho, u, v, w, p)

    return periodic_workload(f"taylor_green_{n}", xyz, init, mach=0.1, reynolds=1600.0, steps=steps,
                             description=f"{n}^3 Taylor-Green vortex, Mach 0.1, Re 1600, wavy 2pi cube")
