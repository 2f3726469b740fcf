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
BC_PERIODIC, BC_INTERFACE, BC_WALL, BC_FARFIELD, BC_FARFIELD_CHAR = 0, 1, 2, 3, 4


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
    """A 1-to-1 face connection.  orient maps the tangential indices of face_a onto those
    of face_b (t1 < t2 the tangential axes of a face): bit 0 swaps t1 and t2, bit 1
    reverses a's t1, bit 2 reverses a's t2; 0 is the identity of aligned blocks."""

    block_a: int
    face_a: int
    block_b: int
    face_b: int
    orient: int = 0


@dataclasses.dataclass
class Patch:
    """A rectangle of face_a of block_a joined node to node with a rectangle of face_b of
    block_b: a's rectangle starts at a_lo and spans n nodes along a's tangential axes
    t1 < t2; b's starts at b_lo along b's t1 < t2; orient as for Interface, inside the
    rectangles."""

    block_a: int
    face_a: int
    a_lo: Tuple[int, int]
    n: Tuple[int, int]
    block_b: int
    face_b: int
    b_lo: Tuple[int, int]
    orient: int = 0


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
    visc_closure: int = 0  # viscous terms at wall / far-field faces: 0 reflected ghosts, 1 one-sided
    patches: List[Patch] = dataclasses.field(default_factory=list)  # patched connections (no interfaces then)

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


def double_shock_tube(n: int = 128, across: int = 7) -> Workload:
    """Two mirror-image shock tubes on the periodic unit interval (a Cartesian n x across x
    across grid, spacing 1/n): high state (rho 1, p 1) for x in [0.25 - dx/2, 0.75 - dx/2),
    low state (rho 0.125, p 0.1) elsewhere, at rest; Euler.  The discontinuities sit
    midway between nodes and the two tubes do not interact before t ~ 0.2."""
    dx = 1.0 / n
    xyz = cartesian_grid(n, across, across, 1.0, across * dx, across * dx)

    def state(c):
        x = c[0]
        high = (x >= 0.25 - dx / 2) & (x < 0.75 - dx / 2)
        rho = np.where(high, 1.0, 0.125)
        p = np.where(high, 1.0, 0.1)
        zero = np.zeros_like(x)
        return conserved(rho, zero, zero, zero, p)

    return periodic_workload(f"double_shock_tube_{n}", xyz, state, viscous=False, cfl=0.3,
                             description=f"two shock tubes, {n} x {across} x {across}, Euler")


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


# ----------------------------------------------------------------------------------------
# multi-block workloads
# ----------------------------------------------------------------------------------------
def _block_index(a, b, c, na, nb):
    return a + na * (b + nb * c)


def structured_interfaces(na, nb, nc, periodic=(True, True, True)):
    """1-to-1 interfaces of an na x nb x nc arrangement of blocks (i+ of a block to i- of
    the next, and so on), with wrap-around seams along the periodic directions."""
    out = []
    for c in range(nc):
        for b in range(nb):
            for a in range(na):
                me = _block_index(a, b, c, na, nb)
                if a + 1 < na or (periodic[0] and na > 0):
                    out.append(Interface(me, 1, _block_index((a + 1) % na, b, c, na, nb), 0))
                if b + 1 < nb or periodic[1]:
                    out.append(Interface(me, 3, _block_index(a, (b + 1) % nb, c, na, nb), 2))
                if c + 1 < nc or periodic[2]:
                    out.append(Interface(me, 5, _block_index(a, b, (c + 1) % nc, na, nb), 4))
    return out


def _sample(arr: np.ndarray, halo: int, gi, gj, gk) -> np.ndarray:
    """arr[:, k, j, i] at global indices (arrays of equal shape) of an array stored with
    `halo` layers on every face."""
    return np.ascontiguousarray(arr[:, gk + halo, gj + halo, gi + halo])


def rotated_split(wl_single: Workload, n1: int, about: str = "i") -> Workload:
    """Cut a periodic single-block workload along i into A = [0, n1) and B = [n1, ni), and
    store B with its index axes rotated, so that the two blocks meet through oriented
    interfaces.  about="i": B's (i', j', k') is global (n1 + i', nj-1-k', j') (a quarter
    turn about i; A's i faces meet B's i faces with A's j along B's reversed k', orient 3).
    about="k": B's (i', j', k') is global (ni-1-j', i', k') (a quarter turn about k; A's
    i+ face meets B's j+ face and A's i- face B's j- face, orient 0, the normal index of B
    running against A's).  Coordinates and states are sampled from the single block, whose
    halos hold the periodic images, so both blocks carry identical data."""
    b = wl_single.blocks[0]
    ni, nj, nk = b.ni, b.nj, b.nk
    assert 0 < n1 < ni

    def local(nx, ny, nz, h):
        k, j, i = np.meshgrid(np.arange(-h, nz + h), np.arange(-h, ny + h), np.arange(-h, nx + h), indexing="ij")
        return i, j, k

    def block_a(h, arr):
        i, j, k = local(n1, nj, nk, h)
        return _sample(arr, h, i, j, k)

    if about == "i":
        dims = (ni - n1, nk, nj)
        to_global = lambda i, j, k: (n1 + i, nj - 1 - k, j)
        ifc = [Interface(0, 1, 1, 0, 3), Interface(0, 0, 1, 1, 3)]
        bc_b = (BC_INTERFACE, BC_INTERFACE, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    elif about == "k":
        dims = (nj, ni - n1, nk)
        to_global = lambda i, j, k: (ni - 1 - j, i, k)
        ifc = [Interface(0, 1, 1, 3, 0), Interface(0, 0, 1, 2, 0)]
        bc_b = (BC_PERIODIC, BC_PERIODIC, BC_INTERFACE, BC_INTERFACE, BC_PERIODIC, BC_PERIODIC)
    else:
        raise ValueError(about)

    def block_b(h, arr):
        i, j, k = local(*dims, h)
        return _sample(arr, h, *to_global(i, j, k))

    bc_a = (BC_INTERFACE, BC_INTERFACE, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    blocks = [Block(n1, nj, nk, block_a(CHALO, b.xyz), block_a(HALO, b.q), bc_a),
              Block(*dims, block_b(CHALO, b.xyz), block_b(HALO, b.q), bc_b)]
    return dataclasses.replace(wl_single, name=wl_single.name + f"_rotated_{about}", blocks=blocks, interfaces=ifc)


def rotated_to_single(about: str, ni: int, nj: int, nk: int, n1: int, arr_b: np.ndarray) -> np.ndarray:
    """Block B's interior values of rotated_split placed at their global (k, j, i) positions
    (an array of shape (nvar, nk, nj, ni - n1) for the global i range [n1, ni))."""
    nvar = arr_b.shape[0]
    out = np.empty((nvar, nk, nj, ni - n1))
    inner = arr_b[:, HALO:-HALO, HALO:-HALO, HALO:-HALO]
    kb, jb, ib = np.meshgrid(*(np.arange(n) for n in inner.shape[1:]), indexing="ij")
    if about == "i":
        gi, gj, gk = n1 + ib, nj - 1 - kb, jb
    else:
        gi, gj, gk = ni - 1 - jb, ib, kb
    out[:, gk, gj, gi - n1] = inner
    return out


def draw_block_sizes(seed: int = 4, lo=(48, 64, 32), hi=(192, 128, 96), counts=(4, 3, 2),
                     total=(36_000_000, 44_000_000), step: int = 8):
    """Per-axis block extents (multiples of `step` in [lo, hi]) redrawn until the product of
    the axis totals lies in `total`."""
    rng = np.random.default_rng(seed)
    while True:
        sizes = [list(rng.integers(lo[d] // step, hi[d] // step + 1, size=counts[d]) * step) for d in range(3)]
        pts = int(np.prod([sum(s) for s in sizes]))
        if total[0] <= pts <= total[1]:
            return [[int(v) for v in s] for s in sizes]


def split_block(wl_single: Workload, sizes, periodic=(True, True, True)) -> Workload:
    """Cut a single-block workload into a structured arrangement of blocks with the given
    per-axis extents; coordinates and states are sliced from the single block (whose
    halos already hold the periodic images), so the blocks hold identical data."""
    b = wl_single.blocks[0]
    assert sum(sizes[0]) == b.ni and sum(sizes[1]) == b.nj and sum(sizes[2]) == b.nk
    na, nb, nc = len(sizes[0]), len(sizes[1]), len(sizes[2])
    off = [np.concatenate([[0], np.cumsum(s)]) for s in sizes]
    blocks = []
    for c in range(nc):
        for bb in range(nb):
            for a in range(na):
                i0, j0, k0 = int(off[0][a]), int(off[1][bb]), int(off[2][c])
                ni, nj, nk = sizes[0][a], sizes[1][bb], sizes[2][c]
                xyz = np.ascontiguousarray(b.xyz[:, k0:k0 + nk + 12, j0:j0 + nj + 12, i0:i0 + ni + 12])
                q = np.ascontiguousarray(b.q[:, k0:k0 + nk + 6, j0:j0 + nj + 6, i0:i0 + ni + 6])
                blocks.append(Block(ni, nj, nk, xyz, q, (BC_INTERFACE,) * 6))
    out = dataclasses.replace(wl_single, name=wl_single.name + f"_{na}x{nb}x{nc}blocks", blocks=blocks,
                              interfaces=structured_interfaces(na, nb, nc, periodic))
    return out


def _tangential(axis):
    return (1, 2) if axis == 0 else (0, 2) if axis == 1 else (0, 1)


def split_boxes(wl_single: Workload, boxes, name: str) -> Workload:
    """Blocks cut from a single-block workload as index boxes (i0, i1, j0, j1, k0, k1) of
    its interior; the boxes need not fill it (what they leave out is solid).  Two boxes
    whose faces lie on one index plane, or on the two sides of a periodic seam, are joined
    by a patch over the overlap of the faces.  A box spanning a periodic direction wraps
    onto itself there.  A face covered completely is an interface; the rest of a face
    keeps the single block's kind where it lies on the domain's boundary and becomes an
    isothermal wall where it borders the solid.  Coordinates and states are sliced from the
    single block, whose halos hold the periodic images and the wall mirrors."""
    b = wl_single.blocks[0]
    N = (b.ni, b.nj, b.nk)
    per = [b.bc[2 * d] == BC_PERIODIC for d in range(3)]
    blocks, patches = [], []
    for (i0, i1, j0, j1, k0, k1) in boxes:
        assert 0 <= i0 < i1 <= N[0] and 0 <= j0 < j1 <= N[1] and 0 <= k0 < k1 <= N[2]
    lo = [(bx[0], bx[2], bx[4]) for bx in boxes]
    hi = [(bx[1], bx[3], bx[5]) for bx in boxes]
    covered = [[np.zeros(0, bool)] * 6 for _ in boxes]
    for a in range(len(boxes)):
        for d in range(3):
            t = _tangential(d)
            ext = (hi[a][t[0]] - lo[a][t[0]], hi[a][t[1]] - lo[a][t[1]])
            for side in (0, 1):
                covered[a][2 * d + side] = np.zeros(ext[::-1], bool)  # [t2][t1]
    for a in range(len(boxes)):
        for d in range(3):
            if per[d] and lo[a][d] == 0 and hi[a][d] == N[d]:
                continue  # wraps onto itself
            t = _tangential(d)
            for c in range(len(boxes)):
                # a's high face against c's low face, directly or across the periodic seam
                if not (hi[a][d] == lo[c][d] or (per[d] and hi[a][d] == N[d] and lo[c][d] == 0)):
                    continue
                if per[d] and lo[c][d] == 0 and hi[c][d] == N[d]:
                    continue
                ov = [(max(lo[a][x], lo[c][x]), min(hi[a][x], hi[c][x])) for x in t]
                if ov[0][0] >= ov[0][1] or ov[1][0] >= ov[1][1]:
                    continue
                n = (ov[0][1] - ov[0][0], ov[1][1] - ov[1][0])
                a_lo = (ov[0][0] - lo[a][t[0]], ov[1][0] - lo[a][t[1]])
                c_lo = (ov[0][0] - lo[c][t[0]], ov[1][0] - lo[c][t[1]])
                patches.append(Patch(a, 2 * d + 1, a_lo, n, c, 2 * d, c_lo))
                covered[a][2 * d + 1][a_lo[1]:a_lo[1] + n[1], a_lo[0]:a_lo[0] + n[0]] = True
                covered[c][2 * d][c_lo[1]:c_lo[1] + n[1], c_lo[0]:c_lo[0] + n[0]] = True
    for a, (i0, i1, j0, j1, k0, k1) in enumerate(boxes):
        bc = []
        for d in range(3):
            if per[d] and lo[a][d] == 0 and hi[a][d] == N[d]:
                bc += [BC_PERIODIC, BC_PERIODIC]
                continue
            for side in (0, 1):
                f = 2 * d + side
                if covered[a][f].all():
                    bc.append(BC_INTERFACE)
                elif (side == 0 and lo[a][d] == 0 or side == 1 and hi[a][d] == N[d]) and not per[d]:
                    bc.append(b.bc[f])
                else:
                    bc.append(BC_WALL)
        xyz = np.ascontiguousarray(b.xyz[:, k0:k1 + 12, j0:j1 + 12, i0:i1 + 12])
        q = np.ascontiguousarray(b.q[:, k0:k1 + 6, j0:j1 + 6, i0:i1 + 6])
        blocks.append(Block(i1 - i0, j1 - j0, k1 - k0, xyz, q, tuple(bc)))
    return dataclasses.replace(wl_single, name=name, blocks=blocks, interfaces=[], patches=patches)


def patched_vortex(n: int = 32, cut_i: int = 13, cut_j: int = 11, cut_k: int = 9, viscous: bool = True,
                   steps: int = 5) -> Workload:
    """The periodic wavy vortex box in four blocks whose faces meet several blocks each:
    A = [0, cut_i) x all x all; B = [cut_i, n) x [0, cut_j) x all; C1, C2 = [cut_i, n) x
    [cut_j, n) x ([0, cut_k), [cut_k, n)).  A's i faces meet B, C1 and C2 (directly and across
    the periodic seam), B's j faces meet C1 and C2."""
    wl = vortex_wavy(n, viscous=viscous, steps=steps)
    boxes = [(0, cut_i, 0, n, 0, n), (cut_i, n, 0, cut_j, 0, n), (cut_i, n, cut_j, n, 0, cut_k),
             (cut_i, n, cut_j, n, cut_k, n)]
    return split_boxes(wl, boxes, f"vortex_wavy_{n}_patched_4blocks")


def periodic_step(ni: int = 48, nj: int = 32, nk: int = 16, step_i: int = 20, step_j: int = 10, seed: int = 5,
                  mach: float = 0.3, reynolds: float = 1000.0, steps: int = 5) -> Workload:
    """A periodic row of backward-facing steps cut from the channel: the channel's
    [0, step_i) x [0, step_j) corner is solid.  Block A = [0, step_i) x [step_j, nj) sits
    above the step, block B = [step_i, ni) x [0, nj) behind it.  B's i faces are walls (the
    step's face and, across the periodic seam, its back) below step_j and patches to A
    above it; A's lower face is the step's top wall."""
    wl = channel(ni, nj, nk, seed=seed, mach=mach, reynolds=reynolds, steps=steps)
    boxes = [(0, step_i, step_j, nj, 0, nk), (step_i, ni, 0, nj, 0, nk)]
    out = split_boxes(wl, boxes, f"periodic_step_{ni}x{nj}x{nk}")
    out.description = f"{ni}x{nj}x{nk} channel with a {step_i}x{step_j} solid step, Mach {mach}, Re {reynolds}"
    return out


def o_grid_vortices(seed: int = 4, sizes=None, n_vortices: int = 8, mach: float = 0.2,
                    reynolds: float = 1000.0, steps: int = 50) -> Workload:
    """24 uneven blocks (4 around x 3 radial x 2 spanwise) of an O-grid around a cylinder of
    diameter 1: theta = -2 pi I/NI + 0.05 sin(2 pi z/Lz), r_j = 0.5 + sum_{m<j} 2e-3 * 1.05^min(m,64)
    (wall spacing 2e-3, stretching ratio 1.05), z = 2 K/NK (Lz = 2), x = r cos theta,
    y = r sin theta.  No-slip isothermal wall at the cylinder (j = 0), far field at the
    outer radius, periodic in theta and z.  Uniform Mach 0.2 stream along x plus seeded
    isentropic vortices (centres 1.5 <= r <= 6, radius 0.3, peak swirl 0.05, random sign)."""
    if sizes is None:
        sizes = draw_block_sizes(seed)
    NI, NJ, NK = (sum(s) for s in sizes)
    Lz = 2.0
    m = np.arange(NJ + 8)
    dr = 2e-3 * 1.05 ** np.minimum(m, 64)
    r_nodes = 0.5 + np.concatenate([[0.0], np.cumsum(dr)])[:NJ]

    def radius(gj):
        gj = np.asarray(gj).astype(np.int64)
        inside = np.clip(gj, 0, NJ - 1)
        r = r_nodes[inside]
        below = gj < 0
        r = np.where(below, 2 * r_nodes[0] - r_nodes[np.clip(-gj, 0, NJ - 1)], r)   # mirrored at the wall
        above = gj > NJ - 1
        r = np.where(above, r_nodes[NJ - 1] + (gj - (NJ - 1)) * (r_nodes[NJ - 1] - r_nodes[NJ - 2]), r)
        return r

    rng = np.random.default_rng(seed + 100)
    vr = rng.uniform(1.5, 6.0, n_vortices)
    vt = rng.uniform(0.0, 2 * np.pi, n_vortices)
    vs = rng.choice([-1.0, 1.0], n_vortices) * 0.05
    centres = np.stack([vr * np.cos(vt), vr * np.sin(vt)], axis=1)

    def coords(gi, gj, gk):
        z = Lz * gk / NK
        th = -2 * np.pi * np.mod(gi, NI) / NI + 0.05 * np.sin(2 * np.pi * z / Lz)
        r = radius(gj)
        return r * np.cos(th), r * np.sin(th), z

    def state(x, y, z):
        u = np.full_like(x, mach)
        v = np.zeros_like(x)
        T = np.ones_like(x)
        for (cx, cy), sw in zip(centres, vs):
            dx, dy = x - cx, y - cy
            r2 = (dx * dx + dy * dy) / 0.09
            g = np.exp(0.5 * (1.0 - r2))
            u = u - sw * (dy / 0.3) * g
            v = v + sw * (dx / 0.3) * g
            T = T - 0.5 * (GAMMA - 1.0) * sw * sw * g * g
        rho = T ** (1.0 / (GAMMA - 1.0))
        p = rho ** GAMMA / GAMMA
        return conserved(rho, u, v, np.zeros_like(u), p)

    off = [np.concatenate([[0], np.cumsum(s)]) for s in sizes]
    blocks = []
    na, nb, nc = (len(s) for s in sizes)
    for c in range(nc):
        for b in range(nb):
            for a in range(na):
                ni, nj, nk = sizes[0][a], sizes[1][b], sizes[2][c]
                K, J, I = index_grid(ni, nj, nk, CHALO)
                x, y, z = coords(I + off[0][a], J + off[1][b], K + off[2][c])
                xyz = np.ascontiguousarray(np.stack([x, y, z]))
                d = CHALO - HALO
                q = np.ascontiguousarray(state(x[d:-d, d:-d, d:-d], y[d:-d, d:-d, d:-d], z[d:-d, d:-d, d:-d]))
                bc = [BC_INTERFACE] * 6
                if b == 0:
                    bc[2] = BC_WALL
                if b == nb - 1:
                    bc[3] = BC_FARFIELD
                blocks.append(Block(ni, nj, nk, xyz, q, tuple(bc)))
    qinf = tuple(float(v) for v in conserved(np.array(1.0), np.array(mach), np.array(0.0), np.array(0.0),
                                             np.array(1.0 / GAMMA)).ravel())
    return Workload(f"o_grid_{len(blocks)}blocks", blocks, structured_interfaces(na, nb, nc, (True, False, True)),
                    mach=mach, reynolds=reynolds, steps=steps, qinf=qinf,
                    description=f"O-grid, {len(blocks)} uneven blocks, {NI}x{NJ}x{NK} = {NI*NJ*NK} points")


def channel(ni: int = 512, nj: int = 512, nk: int = 384, seed: int = 5, mach: float = 0.3,
            reynolds: float = 16200.0, beta: float = 2.5, bump: float = 0.02, steps: int = 20) -> Workload:
    """Channel block: x = 2 pi I/ni (periodic), y = tanh(beta eta)/tanh(beta) with
    eta = -1 + 2 J/(nj-1) (no-slip isothermal walls at J = 0 and nj-1), z = pi K/nk
    (periodic), plus the bump y += 0.02 (1 - y^2) sin x cos 2z.  Laminar profile
    u = Ma (1 - y^2), T = 1, p = 1/gamma, plus seeded N(0, (0.05 Ma)^2) (1 - y^2) on u, v, w."""
    K, J, I = index_grid(ni, nj, nk, CHALO)
    x = 2 * np.pi * I / ni
    z = np.pi * K / nk

    def ymap(jj):
        eta = -1.0 + 2.0 * jj / (nj - 1)
        return np.tanh(beta * eta) / np.tanh(beta)

    # walls at J = 0 and nj-1; ghost points are odd mirrors of the interior ones
    jj = np.where(J < 0, -J, np.where(J > nj - 1, 2 * (nj - 1) - J, J))
    y0 = ymap(jj)
    y0 = np.where(J < 0, 2 * ymap(0) - y0, np.where(J > nj - 1, 2 * ymap(nj - 1) - y0, y0))
    yb = y0 + bump * (1 - np.minimum(y0 * y0, 1.0)) * np.sin(x) * np.cos(2 * z)
    xyz = np.ascontiguousarray(np.stack([x, yb, z]))
    d = CHALO - HALO
    xs, ys = x[d:-d, d:-d, d:-d], yb[d:-d, d:-d, d:-d]
    prof = np.maximum(1.0 - ys * ys, 0.0)
    rng = np.random.default_rng(seed)
    sig = 0.05 * mach
    u = mach * prof + rng.normal(0.0, sig, size=xs.shape) * prof
    v = rng.normal(0.0, sig, size=xs.shape) * prof
    w = rng.normal(0.0, sig, size=xs.shape) * prof
    one = np.ones_like(xs)
    q = conserved(one, u, v, w, one / GAMMA)
    q = wrap_halo(q, axes=(0, 2))
    bc = (BC_PERIODIC, BC_PERIODIC, BC_WALL, BC_WALL, BC_PERIODIC, BC_PERIODIC)
    blk = Block(ni, nj, nk, xyz, np.ascontiguousarray(q), bc)
    return Workload(f"channel_{ni}x{nj}x{nk}", [blk], [], mach=mach, reynolds=reynolds, steps=steps,
                    description=f"{ni}x{nj}x{nk} channel, tanh stretching {beta}, bump {bump}, Mach {mach}")
