"""Seeded synthetic workloads shared by the HIP path, its tests and the oracle's tests.

This module holds only input generation: node positions, resolution fields and
initial flow fields. It contains none of the LABFM arithmetic (no basis
functions, no moment matrices, no operators), so that the oracle and the GPU
path can both be fed the identical arrays without sharing any of the method.

Node sets follow the uniform-resolution recipe of the paper's section on node
generation (a Cartesian lattice, each node shifted by a random vector), with a
per-coordinate uniform jitter of +/-0.3 s and no iterative shifting. Nodes are
returned in Morton (Z-curve) order of their lattice cell so that nodes close in
space are close in memory.

Random numbers come from numpy's PCG64 generator seeded through SeedSequence.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Stencil scale h/s per LABFM order m for the periodic Taylor-Green workloads.
# Chosen so that the mean stencil population on a +/-0.3 s jittered lattice is
# ~30 (m=4), ~60 (m=6), ~90 (m=8) and ~130 (m=10) neighbours.
H_OVER_S = {2: 1.2, 4: 1.55, 6: 2.2, 8: 2.68, 10: 3.2}


@dataclass(frozen=True)
class Box:
    """Rectangular domain [0, Lx) x [0, Ly), each axis periodic or not."""

    Lx: float
    Ly: float
    periodic_x: bool = True
    periodic_y: bool = True


@dataclass
class NodeSet:
    """Structure-of-arrays node description (all float64 except m)."""

    x: np.ndarray
    y: np.ndarray
    s: np.ndarray  # local distribution length scale s_i
    h: np.ndarray  # stencil length scale h_i (stencil radius is 2 h_i)
    m: np.ndarray  # int8 LABFM order per node
    box: Box
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def morton_key_2d(ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    """Z-order key of non-negative integer cell coordinates (< 2**21)."""

    def part1by1(a: np.ndarray) -> np.ndarray:
        a = a.astype(np.uint64) & np.uint64(0xFFFFFFFF)
        a = (a | (a << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
        a = (a | (a << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
        a = (a | (a << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
        a = (a | (a << np.uint64(2))) & np.uint64(0x3333333333333333)
        a = (a | (a << np.uint64(1))) & np.uint64(0x5555555555555555)
        return a

    return part1by1(ix) | (part1by1(iy) << np.uint64(1))


def morton_order(x: np.ndarray, y: np.ndarray, box: Box, cell: float) -> np.ndarray:
    """Stable permutation sorting points by the Morton key of their cell."""
    nx = max(1, int(math.ceil(box.Lx / cell)))
    ny = max(1, int(math.ceil(box.Ly / cell)))
    ix = np.minimum(np.floor(x / cell).astype(np.int64), nx - 1).clip(0)
    iy = np.minimum(np.floor(y / cell).astype(np.int64), ny - 1).clip(0)
    key = morton_key_2d(ix, iy)
    return np.argsort(key, kind="stable")


def jittered_lattice(n_side: int, L: float = 2.0 * math.pi, jitter: float = 0.3,
                     seed: int = 1, m: int = 4, h_over_s: float | None = None,
                     periodic: bool = True, morton: bool = True) -> NodeSet:
    """n_side x n_side lattice on [0, L)^2 with each coordinate shifted by
    U(-jitter*s, +jitter*s), wrapped into the box when periodic.

    Non-periodic boxes keep the jittered points inside [0, L) by clipping the
    shift at the walls (only used for exactness tests on global polynomials).
    """
    s = L / n_side
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    iy, ix = np.meshgrid(np.arange(n_side), np.arange(n_side), indexing="ij")
    ix = ix.ravel()
    iy = iy.ravel()
    ex = rng.uniform(-jitter, jitter, ix.size) * s
    ey = rng.uniform(-jitter, jitter, ix.size) * s
    x = (ix + 0.5) * s + ex
    y = (iy + 0.5) * s + ey
    if periodic:
        x = np.mod(x, L)
        y = np.mod(y, L)
        # np.mod can return L itself for tiny negative inputs; fold that to 0
        x[x >= L] -= L
        y[y >= L] -= L
    if morton:
        order = np.argsort(morton_key_2d(ix, iy), kind="stable")
        x, y = x[order], y[order]
    hs = H_OVER_S[m] if h_over_s is None else h_over_s
    n = x.size
    return NodeSet(
        x=np.ascontiguousarray(x, dtype=np.float64),
        y=np.ascontiguousarray(y, dtype=np.float64),
        s=np.full(n, s, dtype=np.float64),
        h=np.full(n, hs * s, dtype=np.float64),
        m=np.full(n, m, dtype=np.int8),
        box=Box(L, L, periodic, periodic),
        meta={"n_side": n_side, "L": L, "jitter": jitter, "seed": seed,
              "m": m, "h_over_s": hs, "spacing": s},
    )


def random_cloud(n: int, L: float = 1.0, seed: int = 0, periodic: bool = True) -> tuple:
    """Uniform random points (for neighbour-search tests with clustered or
    duplicate-prone layouts)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    x = rng.uniform(0.0, L, n)
    y = rng.uniform(0.0, L, n)
    return np.ascontiguousarray(x), np.ascontiguousarray(y), Box(L, L, periodic, periodic)


# --------------------------------------------------------------------------
# Initial flow fields
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class FlowParams:
    """Isothermal flow constants: sound speed squared, viscosity, body force."""

    c2: float
    mu: float
    gx: float = 0.0
    gy: float = 0.0


def taylor_green_params(Re: float = 100.0, Ma: float = 0.1, L: float = 2.0 * math.pi,
                        U0: float = 1.0, rho0: float = 1.0) -> FlowParams:
    """Reynolds number on the unit velocity and the domain half-width L/2;
    Mach number U0/c."""
    c = U0 / Ma
    mu = rho0 * U0 * (0.5 * L) / Re
    return FlowParams(c2=c * c, mu=mu)


def taylor_green_state(x: np.ndarray, y: np.ndarray, L: float = 2.0 * math.pi) -> tuple:
    """u = sin(kx) cos(ky), v = -cos(kx) sin(ky), rho = 1 with k = 2 pi / L.

    Returns (rho, u, v)."""
    k = 2.0 * math.pi / L
    u = np.sin(k * x) * np.cos(k * y)
    v = -np.cos(k * x) * np.sin(k * y)
    rho = np.ones_like(x)
    return rho, u, v


def fourier_perturbation(x: np.ndarray, y: np.ndarray, seed: int, amp: float = 0.01,
                         kmax: int = 4, L: float = 2.0 * math.pi) -> tuple:
    """Three smooth periodic perturbations: amp * sum over integer wave vectors
    with 1 <= max(|kx|,|ky|) <= kmax of Gaussian-weighted sin and cos modes."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    base = 2.0 * math.pi / L
    out = []
    for _ in range(3):
        f = np.zeros_like(x)
        for kx in range(-kmax, kmax + 1):
            for ky in range(0, kmax + 1):
                if max(abs(kx), abs(ky)) == 0 or (ky == 0 and kx < 0):
                    continue
                a, b = rng.standard_normal(2)
                ph = base * (kx * x + ky * y)
                f += a * np.sin(ph) + b * np.cos(ph)
        out.append(amp * f / math.sqrt(2 * (2 * kmax + 1) * (kmax + 1)))
    return tuple(out)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    n_side: int
    m: int
    seed: int
    steps: int
    L: float = 2.0 * math.pi
    # viscous coefficient of eq. dt (the paper's 0.4). Where the viscous term
    # sets dt with m = 8 (the 2048 x 2048 case), 0.4 puts the fastest decaying
    # mode of the discrete viscous operator outside the Runge-Kutta scheme's
    # real-axis stability interval (about [-2.785, 0]) and the run diverges;
    # 0.25 keeps it inside.
    visc_coef: float = 0.4

    def nodes(self) -> NodeSet:
        return jittered_lattice(self.n_side, L=self.L, seed=self.seed, m=self.m)


# Small periodic Taylor-Green case (4,096 nodes, m=4, 20 RK steps).
TG64_M4 = Workload("tg64_m4", 64, 4, seed=1, steps=20)
# Main periodic Taylor-Green case (262,144 nodes, m=8, 1000 RK steps).
TG512_M8 = Workload("tg512_m8", 512, 8, seed=2, steps=1000)
# Large mixed-precision case (4,194,304 nodes, m=8, 500 RK steps).
TG2048_M8 = Workload("tg2048_m8", 2048, 8, seed=4, steps=500, visc_coef=0.25)
# Adjoint case (65,536 nodes, m=6, 200 RK steps).
TG256_M6 = Workload("tg256_m6", 256, 6, seed=5, steps=200)

WORKLOADS = {w.name: w for w in (TG64_M4, TG512_M8, TG2048_M8, TG256_M6)}


# --------------------------------------------------------------------------
# Graded node sets around circular obstacles (variable resolution)
# --------------------------------------------------------------------------

_nodegen = None


def _place_nodes(L: float, smin: float, sgrid: np.ndarray, max_nodes: int) -> tuple:
    """The paper's sweep placement, run by the host helper libnodegen.so."""
    import ctypes
    import os

    global _nodegen
    if _nodegen is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnodegen.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run __graft_entry__.build()")
        _nodegen = ctypes.CDLL(path)
        _nodegen.place_nodes.restype = ctypes.c_int64
        _nodegen.place_nodes.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64]
    sg = np.ascontiguousarray(sgrid, dtype=np.float64)
    x = np.empty(max_nodes)
    y = np.empty(max_nodes)
    n = _nodegen.place_nodes(L, smin, sg.ctypes.data, sg.shape[0], x.ctypes.data, y.ctypes.data,
                             max_nodes)
    if n < 0:
        raise RuntimeError("node placement failed (cell overflow)")
    return x[:n].copy(), y[:n].copy()


def variable_resolution(s0: float, m: int = 6, L: float = 1.0, grid: int = 1024) -> NodeSet:
    """Periodic square of side L whose spacing varies smoothly with x, from
    s0 at x = 0, L/2, L to s0/2 at x = L/4, 3L/4:
        s(x) = s0 (3 + cos(4 pi x / L)) / 4,
    nodes placed by the paper's sweep for that spacing (no iterative
    shifting: the shifting iteration as read clusters nodes), h = (h/s)_m s
    with s scaled to the sweep's packing like graded_holes, Morton ordered."""
    g = (np.arange(grid) + 0.5) * (L / grid)
    sgrid = np.tile(s0 * (3.0 + np.cos(4.0 * np.pi * g / L)) / 4.0, (grid, 1))
    x, y = _place_nodes(L, 0.5 * s0, sgrid, int(8 * L * L / (0.25 * s0 * s0)))
    s = s0 * (3.0 + np.cos(4.0 * np.pi * x / L)) / 4.0 * SWEEP_SPACING_FACTOR
    h = H_OVER_S[m] * s
    box = Box(L, L, True, True)
    order = morton_order(x, y, box, 0.5 * s0)
    return NodeSet(
        x=np.ascontiguousarray(x[order]), y=np.ascontiguousarray(y[order]),
        s=np.ascontiguousarray(s[order]), h=np.ascontiguousarray(h[order]),
        m=np.full(x.size, m, dtype=np.int8), box=box, meta={"s0": s0},
    )


@dataclass(frozen=True)
class HoleField:
    centres: np.ndarray  # (k, 2)
    radii: np.ndarray    # (k,)
    L: float

    def distance(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        """Signed distance to the nearest obstacle surface (negative inside),
        nearest periodic images."""
        d = np.full(x.shape, np.inf)
        for (cx, cy), r in zip(self.centres, self.radii):
            dx = np.abs(x - cx)
            dy = np.abs(y - cy)
            dx = np.minimum(dx, self.L - dx)
            dy = np.minimum(dy, self.L - dy)
            d = np.minimum(d, np.hypot(dx, dy) - r)
        return d


RAMP_WALL_SPACINGS = 60.0
# The sweep (minimum distance s/sqrt2 between nodes) places 1.77 nodes per s^2
# (measured on uniform s); the node spacing s_i of the method, the spacing of
# the square lattice of the same density, is therefore s / sqrt(1.77).
SWEEP_SPACING_FACTOR = 1.0 / math.sqrt(1.77)


def graded_spacing(d: np.ndarray, s0: float) -> np.ndarray:
    """s = 0.5 s0 within 3 wall spacings of an obstacle, a cosine ramp to
    2 s0 over the next 60 wall spacings, 2 s0 beyond; 0 inside obstacles.
    The ramp is long enough that a stencil (radius 2h = 6.4 s for m = 10)
    sees a spacing within about a factor 1.5 of its own."""
    sw, sb = 0.5 * s0, 2.0 * s0
    t = np.clip((d - 3.0 * sw) / (RAMP_WALL_SPACINGS * sw), 0.0, 1.0)
    s = sw + (sb - sw) * 0.5 * (1.0 - np.cos(np.pi * t))
    return np.where(d < 0.0, 0.0, s)


def graded_holes(n_target: int = 1_000_000, seed: int = 3, n_holes: int = 24,
                 r_range: tuple = (0.05, 0.15), L: float = 1.0, jitter: float = 0.3,
                 grid: int = 2048) -> NodeSet:
    """Periodic unit box with n_holes circular obstacles (centres uniform,
    radii uniform in r_range times L, overlaps allowed), nodes placed by the
    paper's sweep (no iterative shifting) for the graded spacing of
    graded_spacing(), then jittered by
    U(-jitter s, jitter s) per coordinate (a jittered node that would land in
    an obstacle keeps its swept position), Morton ordered. The spacing scale
    s0 is calibrated so that the node count is within 2% of n_target. Orders:
    m = 4 within 1.5 wall spacings of an obstacle, 6 within 3, else 10."""
    ss = np.random.SeedSequence(seed).spawn(2)
    rng = np.random.Generator(np.random.PCG64(ss[0]))
    centres = rng.uniform(0.0, L, (n_holes, 2))
    radii = rng.uniform(r_range[0], r_range[1], n_holes) * L
    holes = HoleField(centres, radii, L)
    g = (np.arange(grid) + 0.5) * (L / grid)
    gx, gy = np.meshgrid(g, g, indexing="xy")  # row index = y
    dgrid = holes.distance(gx, gy)
    fluid = np.mean(dgrid >= 0.0)
    # first guess: nodes ~ area / s^2 with the bulk spacing dominating
    s0 = math.sqrt(fluid * L * L / n_target) / 1.6
    for _ in range(6):
        sgrid = graded_spacing(dgrid, s0)
        x, y = _place_nodes(L, 0.5 * s0, sgrid, int(4 * n_target))
        n = x.size
        if abs(n - n_target) <= 0.02 * n_target:
            break
        s0 *= math.sqrt(n / n_target)
    d = holes.distance(x, y)
    s = graded_spacing(d, s0)
    rng2 = np.random.Generator(np.random.PCG64(ss[1]))
    jx = x + rng2.uniform(-jitter, jitter, n) * s
    jy = y + rng2.uniform(-jitter, jitter, n) * s
    jx = np.mod(jx, L)
    jy = np.mod(jy, L)
    jx[jx >= L] -= L
    jy[jy >= L] -= L
    dj = holes.distance(jx, jy)
    ok = dj >= 0.0
    x = np.where(ok, jx, x)
    y = np.where(ok, jy, y)
    d = holes.distance(x, y)
    # the sweep looks the spacing up on a grid; drop the few swept points
    # that lie (by a fraction of a grid cell) inside an obstacle
    keep = d >= 0.0
    x, y, d = x[keep], y[keep], d[keep]
    n = x.size
    s = graded_spacing(d, s0) * SWEEP_SPACING_FACTOR
    sw = 0.5 * s0
    m = np.where(d < 1.5 * sw, 4, np.where(d < 3.0 * sw, 6, 10)).astype(np.int8)
    hs = np.array([H_OVER_S[k] for k in (4, 6, 10)])
    h = np.where(m == 4, hs[0], np.where(m == 6, hs[1], hs[2])) * s
    order = morton_order(x, y, Box(L, L), 0.5 * s0)
    return NodeSet(
        x=np.ascontiguousarray(x[order]), y=np.ascontiguousarray(y[order]),
        s=np.ascontiguousarray(s[order]), h=np.ascontiguousarray(h[order]),
        m=np.ascontiguousarray(m[order]), box=Box(L, L, True, True),
        meta={"n_target": n_target, "seed": seed, "s0": s0, "n_holes": n_holes,
              "fluid_fraction": float(fluid), "holes": holes},
    )


# --------------------------------------------------------------------------
# Channel between two flat no-slip walls (Poiseuille start-up)
# --------------------------------------------------------------------------

# Levels of the 5-node orthogonal strip along a wall (section "Boundary
# discretisation"): 0 is the wall node i0, 1..4 the nodes i1..i4 at q s along
# the inward normal; -1 marks the bulk.
STRIP_DEPTH = 5
# Order of LABFM at strip levels 0..2 (the paper reduces it to 4 there).
WALL_ORDER = 4
# Stencil scale of a wall node: its one-sided finite-difference column reaches
# i4 at 4 s, which must lie inside the stencil radius 2 h.
WALL_H_OVER_S = 2.1
# Stencil scale at strip levels 1 and 2. Their stencils are cut by the wall;
# with the bulk's m = 4 value (1.55 s) the order-4 Laplacian there has weights
# large enough that the viscous term makes the explicit step unstable (growth
# ~1e9 per step at s = H/20); at 2.0 s the filtered step has spectral radius 1.
NEAR_WALL_H_OVER_S = 2.0


@dataclass(frozen=True)
class Strips:
    """Strip columns of a node set: for each wall node, the node indices of
    i0..i4 (column[k, q] is level q) and the unit normal into the fluid."""

    column: np.ndarray   # int32 (count, 5)
    normal: np.ndarray   # float64 (count, 2)
    level: np.ndarray    # int8 (n,), -1 off the strips

    @property
    def count(self) -> int:
        return int(self.column.shape[0])


def channel(n_x: int, H: float = 1.0, m: int = 6, jitter: float = 0.3, seed: int = 7,
            morton: bool = True) -> tuple:
    """Square channel [0, H) x [0, H], periodic in x, flat walls at y = 0 and
    y = H, uniform spacing s = H / n_x (requires n_x >= 10).

    Each wall carries the 5-node orthogonal strip: rows at y = q s (bottom) and
    y = H - q s (top) for q = 0..4, n_x nodes per row at x = (k + 1/2) s, so
    that every wall node has i1..i4 on its normal. Rows q = 5..n_x-5 form the
    bulk, a lattice with each coordinate shifted by U(-jitter s, +jitter s)
    (x wrapped). Orders: 4 on strip levels 0..2, m elsewhere; h = 2.1 s on the
    walls, 2.0 s on levels 1 and 2, (h/s)_m s elsewhere.

    Returns (NodeSet, Strips), nodes in Morton order of their lattice cell."""
    if n_x < 2 * STRIP_DEPTH:
        raise ValueError("channel needs n_x >= 10")
    s = H / n_x
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    n_rows = n_x + 1
    iy, ix = np.meshgrid(np.arange(n_rows), np.arange(n_x), indexing="ij")
    ix, iy = ix.ravel(), iy.ravel()
    lvl = np.minimum(iy, n_x - iy)
    level = np.where(lvl < STRIP_DEPTH, lvl, -1).astype(np.int8)
    bulk = level < 0
    ex = np.where(bulk, rng.uniform(-jitter, jitter, ix.size), 0.0) * s
    ey = np.where(bulk, rng.uniform(-jitter, jitter, ix.size), 0.0) * s
    x = (ix + 0.5) * s + ex
    y = iy * s + ey
    y[iy == n_x] = H  # the top wall lies exactly on y = H
    x = np.mod(x, H)
    x[x >= H] -= H
    order = (np.argsort(morton_key_2d(ix, iy), kind="stable") if morton
             else np.arange(ix.size))
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    x, y, level = x[order], y[order], level[order]
    # node index of lattice point (k, r)
    idx = rank.reshape(n_rows, n_x)
    q = np.arange(STRIP_DEPTH)
    bottom = idx[q[None, :], np.arange(n_x)[:, None]]           # (n_x, 5)
    top = idx[(n_x - q)[None, :], np.arange(n_x)[:, None]]      # (n_x, 5)
    column = np.ascontiguousarray(np.concatenate([bottom, top]), dtype=np.int32)
    normal = np.concatenate([np.tile([0.0, 1.0], (n_x, 1)), np.tile([0.0, -1.0], (n_x, 1))])
    n = x.size
    mm = np.where((level >= 0) & (level <= 2), WALL_ORDER, m).astype(np.int8)
    hs = np.where(level == 0, WALL_H_OVER_S,
                  np.where(mm == WALL_ORDER, NEAR_WALL_H_OVER_S, H_OVER_S[m]))
    nodes = NodeSet(
        x=np.ascontiguousarray(x), y=np.ascontiguousarray(y),
        s=np.full(n, s), h=np.ascontiguousarray(hs * s), m=np.ascontiguousarray(mm),
        box=Box(H, H, True, False),
        meta={"n_x": n_x, "H": H, "m": m, "jitter": jitter, "seed": seed, "spacing": s},
    )
    return nodes, Strips(column=column, normal=np.ascontiguousarray(normal), level=level)


@dataclass(frozen=True)
class Poiseuille:
    """Start-up of body-force driven flow between walls y = 0 and y = H, from
    rest: Re = rho0 U0 H / mu, Ma = U0 / c with U0 = rho0 g H^2 / (8 mu) the
    steady centre-line velocity."""

    Re: float = 10.0
    Ma: float = 0.05
    H: float = 1.0
    U0: float = 1.0
    rho0: float = 1.0

    @property
    def mu(self) -> float:
        return self.rho0 * self.U0 * self.H / self.Re

    @property
    def gx(self) -> float:
        return 8.0 * self.mu * self.U0 / (self.rho0 * self.H * self.H)

    def flow(self) -> FlowParams:
        c = self.U0 / self.Ma
        return FlowParams(c2=c * c, mu=self.mu, gx=self.gx, gy=0.0)

    def time(self, t_star: float) -> float:
        """Dimensional time of t* = t U0 / H."""
        return t_star * self.H / self.U0


POISEUILLE = Poiseuille()


def poiseuille_startup(y: np.ndarray, t: float, H: float, nu: float, g: float,
                       n_terms: int = 400) -> np.ndarray:
    """Analytic u(y, t) of flow between walls y = 0, H started from rest by a
    body force g (the incompressible start-up, which the isothermal equations
    also admit with uniform density): the solution of u_t = nu u_yy + g,
    u(0) = u(H) = 0, u(y, 0) = 0,
        u = g y (H - y) / (2 nu)
            - sum_{k odd} 4 g H^2 / (nu pi^3 k^3) sin(k pi y / H) e^{-k^2 pi^2 nu t / H^2}
    (the sine series of the steady parabola, each mode decaying at its own
    rate); n_terms odd modes are summed."""
    y = np.asarray(y, dtype=np.float64)
    u = g * y * (H - y) / (2.0 * nu)
    for j in range(n_terms):
        k = 2 * j + 1
        amp = 4.0 * g * H * H / (nu * math.pi ** 3 * k ** 3)
        u = u - amp * np.sin(k * math.pi * y / H) * math.exp(-(k * math.pi) ** 2 * nu * t / (H * H))
    return u


# Initial stencil scale of the stencil optimisation (section "Stencil
# optimisation"): h0 = 2.8 s.
STENCIL_H0_OVER_S = 2.8


def cylinder(n_theta: int, R: float = 0.2, L: float = 1.0, m: int = 6, jitter: float = 0.3,
             seed: int = 9) -> tuple:
    """A no-slip circular wall of radius R centred in the periodic box
    [0, L)^2 (the geometry of the paper's cylinder flows): n_theta wall nodes
    at angles 2 pi k / n_theta, each with its strip column i1..i4 at radius
    R + q s along the outward (into the fluid) normal, s = 2 pi R / n_theta;
    the fluid beyond R + 4.5 s is a jittered lattice of spacing s. Orders and
    stencil scales as in channel(). Returns (NodeSet, Strips) in Morton order
    of a cell grid of side s."""
    s = 2.0 * math.pi * R / n_theta
    cx = cy = 0.5 * L
    phi = 2.0 * math.pi * np.arange(n_theta) / n_theta
    q = np.arange(STRIP_DEPTH)
    rr = R + q[None, :] * s                                   # (1, 5)
    sx = cx + rr * np.cos(phi)[:, None]                       # (n_theta, 5)
    sy = cy + rr * np.sin(phi)[:, None]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    nl = int(round(L / s))
    sl = L / nl
    iy, ix = np.meshgrid(np.arange(nl), np.arange(nl), indexing="ij")
    bx = (ix.ravel() + 0.5) * sl + rng.uniform(-jitter, jitter, nl * nl) * sl
    by = (iy.ravel() + 0.5) * sl + rng.uniform(-jitter, jitter, nl * nl) * sl
    keep = np.hypot(bx - cx, by - cy) > R + 4.5 * s
    bx, by = np.mod(bx[keep], L), np.mod(by[keep], L)
    x = np.concatenate([sx.ravel(), bx])
    y = np.concatenate([sy.ravel(), by])
    level = np.concatenate([np.tile(q, n_theta), np.full(bx.size, -1)]).astype(np.int8)
    box = Box(L, L, True, True)
    order = morton_order(x, y, box, s)
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    x, y, level = x[order], y[order], level[order]
    column = np.ascontiguousarray(rank[: n_theta * STRIP_DEPTH].reshape(n_theta, STRIP_DEPTH),
                                  dtype=np.int32)
    normal = np.ascontiguousarray(np.stack([np.cos(phi), np.sin(phi)], axis=1))
    n = x.size
    mm = np.where((level >= 0) & (level <= 2), WALL_ORDER, m).astype(np.int8)
    hs = np.where(level == 0, WALL_H_OVER_S,
                  np.where(mm == WALL_ORDER, NEAR_WALL_H_OVER_S, H_OVER_S[m]))
    nodes = NodeSet(
        x=np.ascontiguousarray(x), y=np.ascontiguousarray(y), s=np.full(n, s),
        h=np.ascontiguousarray(hs * s), m=np.ascontiguousarray(mm), box=box,
        meta={"n_theta": n_theta, "R": R, "L": L, "m": m, "spacing": s},
    )
    return nodes, Strips(column=column, normal=normal, level=level)
