"""Seeded synthetic workloads: particles, material, boundary conditions.

This module only lays out inputs (particle positions on Gauss points, volumes,
identity deformation state, Dirichlet masks and prescribed values, seeded
material draws).  It holds none of the method's arithmetic, and both the HIP
path and the CPU oracle consume what it produces.

Geometry and material follow the paper's problem statement (Sec. 2.1:
displacement-controlled Dirichlet boundaries, traction boundaries, gravity)
with the five synthetic configurations:

* ``c1``: plane-strain confined column under gravity (32x32 grid, h = 1/32,
  0.5 x 0.5 m block, Hencky, E = 1 MPa, nu = 0.3), one load step.
* ``c2``: plane-strain rigid footing on Drucker-Prager soil (256x128 grid,
  h = 1/256, 1.0 x 0.5 m), geostatic step then 1 mm footing steps.
* ``c3``: the 3-D footing (128^3 grid, soil in the lower half, friction angle
  uniform in [25, 35] deg per particle).
* ``c4``: u-p consolidation under a 10 kPa surface load with top drainage
  (512x512 grid, dt = 1 s).
* ``c5``: a batch of c2-like footings with seeded particle counts, stiffness
  and friction.

All grids carry one ghost node per side: nodes -1..n+1 per axis.  Grid
vectors are node-interleaved over the full padded grid, x fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

GAUSS_1D = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))

MODEL_HENCKY, MODEL_DP, MODEL_UP = 0, 1, 2


@dataclass
class Problem:
    """Grid, material and time-step data of one simulation."""
    dim: int
    n: tuple                      # cells per axis (3 entries, unused ones 0)
    h: float
    x0: tuple = (0.0, 0.0, 0.0)
    up: int = 0                   # 1: u-p poromechanics
    dp: int = 0                   # 1: Drucker-Prager plasticity
    dp_match: int = 0             # 0 outer cone, 1 plane strain, 2 inner cone
    E: float = 1e6
    nu: float = 0.3
    phi: float = 0.0              # radians
    c: float = 0.0
    psi: float = 0.0
    rho0: float = 2000.0
    g: tuple = (0.0, -9.81, 0.0)
    perm: float = 0.0             # intrinsic permeability k [m^2]
    mu_f: float = 1e-3            # fluid viscosity [Pa s]
    biot: float = 1.0
    rho_f: float = 1000.0
    dt: float = 1.0
    apex_reg: float = 1e-6          # tangent scale of apex returns (values are exact)
    shape: int = 0                # 0 quadratic B-splines, 1 cpGIMP
    elastic: int = 0              # 0 Hencky, 1 compressible Neo-Hookean (elastic only)
    lp0: tuple = (0.0, 0.0, 0.0)  # cpGIMP: initial half-width of the particle domain per axis
    name: str = ""

    @property
    def ndof(self) -> int:
        return self.dim + (1 if self.up else 0)

    @property
    def nodes_per_axis(self):
        return [int(self.n[k]) + 3 for k in range(self.dim)]

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.nodes_per_axis))

    def node_coords(self, axis: int) -> np.ndarray:
        """Coordinates of the node lattice along one axis (nodes -1..n+1)."""
        return self.x0[axis] + np.arange(-1, self.n[axis] + 2) * self.h

    def node_grid_index(self):
        """Per-axis integer node index (-1..n+1) of every full-grid node."""
        axes = [np.arange(-1, self.n[k] + 2) for k in range(self.dim)]
        mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
        return [m.reshape(-1) for m in mesh]


@dataclass
class Particles:
    """SoA particle state (component-major arrays)."""
    x: np.ndarray                 # [dim][np]
    vol0: np.ndarray              # [np]
    F: np.ndarray                 # [dim*dim][np]
    be: np.ndarray                # 2D [4][np] (xx,yy,xy,zz); 3D [6][np] (xx,yy,zz,yz,xz,xy)
    fp: np.ndarray | None = None  # [dim][np] applied particle force (traction x area)
    E: np.ndarray | None = None   # [np]
    phi: np.ndarray | None = None  # [np]

    @property
    def np(self) -> int:
        return int(self.vol0.shape[0])

    def copy(self):
        cp = lambda a: None if a is None else a.copy()
        return Particles(cp(self.x), cp(self.vol0), cp(self.F), cp(self.be), cp(self.fp), cp(self.E), cp(self.phi))


@dataclass
class Dirichlet:
    """Constrained unknowns over the full padded grid: mask [n_nodes][ndof]
    and the prescribed value of the unknown (the displacement increment of
    the step; the total pore pressure for u-p)."""
    mask: np.ndarray
    value: np.ndarray


@dataclass
class Workload:
    prob: Problem
    particles: Particles
    n_steps: int                        # counted load steps
    geostatic: bool = False             # extra uncounted gravity step 0
    walls: list = field(default_factory=list)       # (axis, side, node_index, dofs)
    footing: tuple | None = None        # (ranges per axis, normal axis, dofs fixed, push)
    p_drained: tuple | None = None      # (axis, node_index_min) with p = 0
    tol: float = 1e-10

    # ------------------------------------------------------------------
    def _base_mask(self):
        P = self.prob
        nd = P.ndof
        mask = np.zeros((P.n_nodes, nd), dtype=np.uint8)
        value = np.zeros((P.n_nodes, nd))
        idx = P.node_grid_index()
        for axis, side, node, dofs in self.walls:
            sel = idx[axis] <= node if side == "lo" else idx[axis] >= node
            for d in dofs:
                mask[sel, d] = 1
        if self.p_drained is not None:
            axis, node = self.p_drained
            mask[idx[axis] >= node, P.dim] = 1
        return mask, value, idx

    def footing_nodes(self) -> np.ndarray:
        """Full-grid ids of the footing nodes (empty if no footing)."""
        if self.footing is None:
            return np.zeros(0, dtype=np.int64)
        _, _, idx = self._base_mask()
        ranges = self.footing[0]
        sel = np.ones(self.prob.n_nodes, dtype=bool)
        for axis, (lo, hi) in enumerate(ranges):
            sel &= (idx[axis] >= lo) & (idx[axis] <= hi)
        return np.nonzero(sel)[0].astype(np.int64)

    def bc(self, step: int) -> Dirichlet:
        """Dirichlet data of load step ``step`` (0 is the geostatic step when
        ``geostatic`` is set; footing steps then run 1..n_steps)."""
        mask, value, _ = self._base_mask()
        push_active = self.footing is not None and (step >= 1 or not self.geostatic)
        if push_active:
            fn = self.footing_nodes()
            _, normal, fixed, push = self.footing
            for d in fixed:
                mask[fn, d] = 1
                value[fn, d] = 0.0
            mask[fn, normal] = 1
            value[fn, normal] = push
        return Dirichlet(mask, value)

    def gravity_scale(self, step: int) -> float:
        return 1.0

    def steps(self):
        """Load-step numbers in run order."""
        first = 0 if self.geostatic else 1
        return list(range(first, self.n_steps + 1))


# ---------------------------------------------------------------- builders --
def gauss_particles(dim: int, h: float, x0, cell_lo, cell_hi, points=GAUSS_1D):
    """2 points per axis in every cell of the box [cell_lo, cell_hi), at the
    given cell fractions (default: the 2-point Gauss rule).  Order: cells x
    fastest, then points x fastest."""
    cells = [np.arange(cell_lo[k], cell_hi[k]) for k in range(dim)]
    cmesh = [m.reshape(-1) for m in np.meshgrid(*cells[::-1], indexing="ij")[::-1]]
    gp = [np.array(points)] * dim
    gmesh = [m.reshape(-1) for m in np.meshgrid(*gp[::-1], indexing="ij")[::-1]]
    nc, ng = cmesh[0].shape[0], gmesh[0].shape[0]
    x = np.empty((dim, nc * ng))
    for k in range(dim):
        x[k] = x0[k] + (cmesh[k][:, None] + gmesh[k][None, :]).reshape(-1) * h
    return x


def identity_state(dim: int, x: np.ndarray, h: float, ppc: int) -> Particles:
    n = x.shape[1]
    F = np.zeros((dim * dim, n))
    for k in range(dim):
        F[k * dim + k] = 1.0
    if dim == 2:
        be = np.zeros((4, n)); be[0] = be[1] = be[3] = 1.0
    else:
        be = np.zeros((6, n)); be[0] = be[1] = be[2] = 1.0
    vol0 = np.full(n, h ** dim / ppc)
    return Particles(np.ascontiguousarray(x), vol0, F, be)


def make_c1() -> Workload:
    """Plane-strain confined column under gravity (closed form: uniaxial
    Hencky compression, lambda(Y) = W0(s)/s)."""
    h = 1.0 / 32
    P = Problem(dim=2, n=(32, 32, 0), h=h, E=1e6, nu=0.3, rho0=2000.0, g=(0.0, -9.81, 0.0), name="c1")
    x = gauss_particles(2, h, (0.0, 0.0), (0, 0), (16, 16))
    parts = identity_state(2, x, h, 4)
    walls = [(0, "lo", 0, (0,)), (0, "hi", 16, (0,)), (1, "lo", 0, (0, 1))]
    return Workload(P, parts, n_steps=1, walls=walls)


def footing_2d(n_y: int, E: float, phi_deg: float, n_steps: int, name: str, nu=0.3) -> Workload:
    n_x = 2 * n_y
    h = 0.5 / n_y
    P = Problem(dim=2, n=(n_x, n_y, 0), h=h, dp=1, E=E, nu=nu, phi=math.radians(phi_deg), c=0.0, psi=0.0,
                rho0=2000.0, g=(0.0, -9.81, 0.0), name=name)
    x = gauss_particles(2, h, (0.0, 0.0), (0, 0), (n_x, n_y))
    parts = identity_state(2, x, h, 4)
    walls = [(0, "lo", 0, (0,)), (0, "hi", n_x, (0,)), (1, "lo", 0, (0, 1))]
    # footing 0.1 m wide centred at x = 0.5: nodes with x_i in [0.45, 0.55]
    i_lo = (9 * n_y + 9) // 10
    i_hi = (11 * n_y) // 10
    footing = (((i_lo, i_hi), (n_y, n_y + 1)), 1, (0,), -1e-3)
    return Workload(P, parts, n_steps=n_steps, geostatic=True, walls=walls, footing=footing)


def make_c2(n_steps: int = 50) -> Workload:
    return footing_2d(128, 1e7, 30.0, n_steps, "c2")


def make_c3(n: int = 128, n_steps: int = 20, seed: int = 1003) -> Workload:
    """3-D footing on a cube: n^3 grid, soil in the lower half, 8 particles
    per cell, friction angle uniform in [25, 35] deg per particle."""
    h = 1.0 / n
    P = Problem(dim=3, n=(n, n, n), h=h, dp=1, E=5e7, nu=0.25, phi=math.radians(30.0), c=0.0, psi=0.0,
                rho0=2000.0, g=(0.0, 0.0, -9.81), name="c3")
    x = gauss_particles(3, h, (0.0, 0.0, 0.0), (0, 0, 0), (n, n, n // 2))
    parts = identity_state(3, x, h, 8)
    rng = np.random.default_rng(seed)
    parts.phi = np.radians(rng.uniform(25.0, 35.0, size=parts.np))
    walls = [(0, "lo", 0, (0,)), (0, "hi", n, (0,)), (1, "lo", 0, (1,)), (1, "hi", n, (1,)),
             (2, "lo", 0, (0, 1, 2))]
    lo = (9 * n + 19) // 20          # ceil(0.45 n)
    hi = (11 * n) // 20              # floor(0.55 n)
    footing = (((lo, hi), (lo, hi), (n // 2, n // 2 + 1)), 2, (0, 1), -1e-3)
    return Workload(P, parts, n_steps=n_steps, geostatic=True, walls=walls, footing=footing)


def make_c4(n: int = 512, n_steps: int = 100, load: float = 1e4, H: float = 1.0, width_cells: int | None = None,
            E=1e7, nu=0.3, perm=1e-12, mu_f=1e-3, dt=1.0) -> Workload:
    """u-p consolidation: soil fills the grid, rollers on the sides, fixed
    base, surface load on the top particle row, p = 0 on the top nodes."""
    ny = n
    nx = n if width_cells is None else width_cells
    h = H / ny
    P = Problem(dim=2, n=(nx, ny, 0), h=h, up=1, E=E, nu=nu, perm=perm, mu_f=mu_f, biot=1.0, rho_f=1000.0,
                rho0=2000.0, g=(0.0, 0.0, 0.0), dt=dt, name="c4")
    x = gauss_particles(2, h, (0.0, 0.0), (0, 0), (nx, ny))
    parts = identity_state(2, x, h, 4)
    top = x[1] > (ny - 0.5) * h
    top &= x[1] >= x[1].max() - 1e-12 * h
    fp = np.zeros((2, parts.np))
    fp[1, top] = -load * h / 2.0          # traction x tributary width (2 particles per cell width)
    parts.fp = fp
    walls = [(0, "lo", 0, (0,)), (0, "hi", nx, (0,)), (1, "lo", 0, (0, 1))]
    return Workload(P, parts, n_steps=n_steps, walls=walls, p_drained=(1, ny))


def c5_draws(seed: int, nsim: int = 64):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsim):
        ns = int(rng.integers(10000, 200001))
        logE = float(rng.uniform(6.0, 8.0))
        phi = float(rng.uniform(20.0, 40.0))
        out.append((ns, 10.0 ** logE, phi))
    return out


def footing_push(E: float, phi: float, c: float, n_steps: int, B: float = 0.1, nu: float = 0.3,
                 rho0: float = 2000.0, g: float = 9.81, frac: float = 0.5) -> float:
    """Per-step footing displacement (negative = down) whose total over
    n_steps is frac times the elastic settlement of a strip of width B at
    its bearing capacity q = c Nc + gamma B N_gamma / 2 (surface footing,
    Vesic factors), s = q B (1 - nu^2) / E: the path stays below the limit
    load, where perfect plasticity has no unique solution."""
    t = math.tan(phi)
    nq = math.exp(math.pi * t) * math.tan(math.pi / 4 + phi / 2) ** 2
    nc = (nq - 1.0) / t
    ng = 2.0 * (nq + 1.0) * t
    q = c * nc + 0.5 * rho0 * g * B * ng
    return -frac * q * B * (1.0 - nu * nu) / E / n_steps


def make_c5(nsim: int = 64, n_steps: int = 30, seed: int = 1005, target_seed: int = 2005, gradient: bool = True):
    """Batch of 2-D footings; returns (list of Workload, target (E, phi) list).
    gradient=True applies gradient_reading to every sim, with a push per sim
    sized (footing_push) for the softer-capacity of its drawn and its target
    (E, friction), so both runs stay below the limit load."""
    sims, targets = [], []
    draws = c5_draws(seed, nsim)
    tdraws = c5_draws(target_seed, nsim)
    for s, ((ns, E, phi), (_, Et, phit)) in enumerate(zip(draws, tdraws)):
        n_y = max(2, int(round(math.sqrt(ns / 8.0))))
        w = footing_2d(n_y, E, phi, n_steps, f"c5_{s}")
        if gradient:
            c = 1e3
            push = max(footing_push(E, math.radians(phi), c, n_steps), footing_push(Et, math.radians(phit), c, n_steps))
            gradient_reading(w, cohesion=c, push=push)
        w.particles.E = np.full(w.particles.np, E)
        w.particles.phi = np.full(w.particles.np, math.radians(phi))
        sims.append(w)
        targets.append((Et, math.radians(phit)))
    return sims, targets


def gradient_reading(w: Workload, cohesion: float = 1e3, push: float = -1e-4) -> Workload:
    """The footing reading used for gradients (a path Newton follows): a
    small cohesion, associated flow and 0.1 mm footing pushes.  With zero
    cohesion and zero dilation the footing path loses ellipticity."""
    w.prob.c = cohesion
    w.prob.dp_match = 4          # outer cone, associated flow
    w.footing = (w.footing[0], w.footing[1], w.footing[2], push)
    return w


def small_footing(n_y: int = 8, n_steps: int = 3, E=1e7, phi_deg=30.0) -> Workload:
    """A c2-shaped footing on a coarse grid (for tests)."""
    return footing_2d(n_y, E, phi_deg, n_steps, f"footing{n_y}")


def bar_column(n_cells: int = 64, l0: float = 50.0, rho0: float = 80.0, E: float = 1e4, nu: float = 0.0,
               n_steps: int = 40, j2_yield: float | None = None, cpgimp: bool = False) -> Workload:
    """Bar compaction under self-weight (paper Sec. 4.2 geometry): a one-cell
    wide plane-strain column of height l0 with 2x2 particles per cell,
    rollers on both sides, fixed base; gravity is ramped over n_steps.
    j2_yield: the elastoplastic case, J2 plasticity with sqrt(2 J2) <= j2_yield
    (5 kPa in the paper); cpgimp: the paper's shape functions (particle domain
    half-width h/4 per axis, 2 particles per cell and axis)."""
    h = l0 / n_cells
    P = Problem(dim=2, n=(1, n_cells, 0), h=h, E=E, nu=nu, rho0=rho0, g=(0.0, -9.81, 0.0), name="bar")
    if j2_yield is not None:
        P.dp, P.dp_match, P.c = 1, 3, float(j2_yield)
    if cpgimp:
        # particle domains of half-width h/4 around the cell quarter points tile the bar
        P.shape, P.lp0 = 1, (h / 4.0, h / 4.0, 0.0)
        x = gauss_particles(2, h, (0.0, 0.0), (0, 0), (1, n_cells), points=(0.25, 0.75))
    else:
        x = gauss_particles(2, h, (0.0, 0.0), (0, 0), (1, n_cells))
    parts = identity_state(2, x, h, 4)
    walls = [(0, "lo", 2, (0,)), (1, "lo", 0, (0, 1))]   # every x-node is a roller
    return Workload(P, parts, n_steps=n_steps, walls=walls)


def with_gravity(prob: Problem, scale: float) -> Problem:
    return replace(prob, g=tuple(scale * v for v in prob.g))


CONFIGS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4}
