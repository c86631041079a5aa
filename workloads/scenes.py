"""Seeded synthetic scenes for the WCSPH step.

This module only lays out particles and grids.  It holds none of the
method's arithmetic (no kernel, no equation of state used by the solver, no
neighbor predicate, no integrator): it produces the canonical encoded state
that both the GPU library and the CPU oracle consume.

Canonical encoded state (one entry per particle, all little-endian):

* ``cell``  int32   linear cell index  cx + nx*(cy + ny*cz) (+ scene cell base)
* ``pos``   float32 [N,4]  xyz = offset from the cell centre [m], w = mass [kg]
* ``vel``   float32 [N,4]  xyz = velocity [m/s], w = density [kg/m^3]
* ``info``  uint32  type << 30 | id   (type 0 = fluid, 1 = dynamic boundary)

The physical position is origin + (c + 1/2) * cell_size + offset, evaluated
in float64 with cell_size taken as its float32 value.

Geometry follows the paper's use cases: a uniform lattice of spacing dp with
particle centres at (k + 1/2) dp, fluid columns at rest under gravity with a
hydrostatic density profile, and three layers of fixed ("dynamic") boundary
particles outside the tank walls and floor (paper, sections "The SPH in
GPUSPH" and "Test case setup").  Particle mass is rho0 * dp^3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLUID = 0
BOUNDARY = 1
TYPE_SHIFT = 30
ID_MASK = (1 << TYPE_SHIFT) - 1


@dataclass
class Grid:
    origin: np.ndarray          # float64 [3]
    cell_size: np.ndarray       # float32 [3]
    ncell: np.ndarray           # int32 [3]
    periodic: int = 0           # bit d set: axis d is periodic
    cell_base: int = 0

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.ncell.astype(np.int64)))


@dataclass
class Params:
    dp: float
    h: float
    r_search: float
    rho0: float = 1000.0
    gamma: float = 7.0
    c0: float = 20.0
    alpha: float = 0.01
    eps_visc: float = 0.01
    nu: float = 0.0
    g: tuple = (0.0, 0.0, -9.81)
    cfl: float = 0.3
    visc_model: int = 0         # laminar term: 0 none (artificial only), 1 Morris, 2 Monaghan K form
    delta: float = 0.0          # density diffusion coefficient (0 = off)
    kernel: int = 0             # 0 Wendland, 1 cubic spline, 2 quadratic, 3 Gaussian
    formulation: int = 0        # 0 golden rule, 1 Landrini-Morris


@dataclass
class Scene:
    name: str
    grid: Grid
    params: Params
    cell: np.ndarray
    pos: np.ndarray
    vel: np.ndarray
    info: np.ndarray
    n_fluid: int
    n_boundary: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])

    def copy(self) -> "Scene":
        return Scene(self.name, self.grid, self.params, self.cell.copy(), self.pos.copy(),
                     self.vel.copy(), self.info.copy(), self.n_fluid, self.n_boundary,
                     dict(self.meta))


def make_grid(lo, hi, r_search: float, periodic: int = 0, cell_base: int = 0) -> Grid:
    """Uniform grid over [lo, hi] whose cell side is at least r_search.

    Cell side per axis is L / floor(L / r_s) (so a periodic axis is divided
    exactly), stored as float32 and never below the float32 search radius.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    rs32 = np.float32(r_search)
    cs = np.zeros(3, dtype=np.float32)
    nc = np.zeros(3, dtype=np.int32)
    for d in range(3):
        L = float(hi[d] - lo[d])
        n = max(1, int(math.floor(L / float(rs32))))
        while n > 1 and np.float32(L / n) < rs32:
            n -= 1
        cs[d] = np.float32(L / n)
        nc[d] = n
        if (periodic >> d) & 1:
            if n < 3:
                raise ValueError("a periodic axis needs at least 3 cells")
    return Grid(origin=lo.copy(), cell_size=cs, ncell=nc, periodic=int(periodic), cell_base=int(cell_base))


def encode_positions(grid: Grid, x: np.ndarray):
    """float64 positions [N,3] -> (linear cell int32, float32 offsets [N,3])."""
    cs = grid.cell_size.astype(np.float64)
    rel = x - grid.origin[None, :]
    c = np.floor(rel / cs[None, :]).astype(np.int64)
    for d in range(3):
        if (grid.periodic >> d) & 1:
            c[:, d] %= int(grid.ncell[d])
        if c[:, d].min() < 0 or c[:, d].max() >= grid.ncell[d]:
            raise ValueError("particle outside the grid on axis %d" % d)
    centre = grid.origin[None, :] + (c + 0.5) * cs[None, :]
    off = (x - centre).astype(np.float32)
    nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
    lin = c[:, 0] + nx * (c[:, 1] + ny * c[:, 2]) + grid.cell_base
    return lin.astype(np.int32), off


def decode_positions(grid: Grid, cell: np.ndarray, off: np.ndarray) -> np.ndarray:
    """Inverse of encode_positions, in float64 (exact lift of the float32 offsets)."""
    nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
    lc = cell.astype(np.int64) - grid.cell_base
    cx = lc % nx
    cy = (lc // nx) % ny
    cz = lc // (nx * ny)
    c = np.stack([cx, cy, cz], axis=1).astype(np.float64)
    cs = grid.cell_size.astype(np.float64)
    return grid.origin[None, :] + (c + 0.5) * cs[None, :] + off.astype(np.float64)


def lattice(nx: int, ny: int, nz: int, dp: float, lo=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Points (i + 1/2) dp offset by lo, x fastest."""
    i = (np.arange(nx) + 0.5) * dp
    j = (np.arange(ny) + 0.5) * dp
    k = (np.arange(nz) + 0.5) * dp
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return pts + np.asarray(lo, dtype=np.float64)[None, :]


def tank_walls(nx: int, ny: int, nz: int, dp: float, layers: int = 3,
               walls_x: bool = True, walls_y: bool = True) -> np.ndarray:
    """Boundary lattice outside an open-top tank whose inside is
    [0, nx dp] x [0, ny dp] x [0, nz dp]: `layers` layers under the floor and
    around the side walls (up to the tank height)."""
    lx0 = -layers if walls_x else 0
    lx1 = nx + layers if walls_x else nx
    ly0 = -layers if walls_y else 0
    ly1 = ny + layers if walls_y else ny
    ii = np.arange(lx0, lx1)
    jj = np.arange(ly0, ly1)
    pts = []
    # floor
    kk = np.arange(-layers, 0)
    Z, Y, X = np.meshgrid(kk, jj, ii, indexing="ij")
    pts.append(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    # side ring
    kk = np.arange(0, nz)
    Z, Y, X = np.meshgrid(kk, jj, ii, indexing="ij")
    ring = np.ones(X.shape, dtype=bool)
    inside = np.ones(X.shape, dtype=bool)
    if walls_x:
        inside &= (X >= 0) & (X < nx)
    if walls_y:
        inside &= (Y >= 0) & (Y < ny)
    ring &= ~inside
    pts.append(np.stack([X[ring], Y[ring], Z[ring]], axis=1))
    idx = np.concatenate(pts, axis=0).astype(np.float64)
    return (idx + 0.5) * dp


def hydrostatic_density(z: np.ndarray, H: float, p: Params) -> np.ndarray:
    """Density of a fluid at rest under gravity: the pressure rho0*g*(H-z)
    mapped back through Cole's equation of state (initial condition only)."""
    gmag = abs(p.g[2])
    B = p.rho0 * p.c0 ** 2 / p.gamma
    depth = np.maximum(H - z, 0.0)
    return p.rho0 * (1.0 + p.rho0 * gmag * depth / B) ** (1.0 / p.gamma)


def _assemble(name, grid, params, xf, xb, H, vel_f=None, meta=None, rho_scale=None) -> Scene:
    x = np.concatenate([xf, xb], axis=0)
    nf, nb = xf.shape[0], xb.shape[0]
    cell, off = encode_positions(grid, x)
    n = nf + nb
    pos = np.zeros((n, 4), dtype=np.float32)
    pos[:, :3] = off
    pos[:, 3] = np.float32(params.rho0 * params.dp ** 3)
    vel = np.zeros((n, 4), dtype=np.float32)
    if vel_f is not None:
        vel[:nf, :3] = vel_f.astype(np.float32)
    rho = hydrostatic_density(x[:, 2], H, params)
    if rho_scale is not None:
        rho = rho * rho_scale
    vel[:, 3] = rho.astype(np.float32)
    ids = np.arange(n, dtype=np.uint32)
    types = np.concatenate([np.full(nf, FLUID, np.uint32), np.full(nb, BOUNDARY, np.uint32)])
    info = (types << np.uint32(TYPE_SHIFT)) | ids
    return Scene(name, grid, params, cell, pos, vel, info, nf, nb, meta or {})


def sph_params(dp: float, **kw) -> Params:
    """Wendland C2 with h = 1.3 dp (support 2h) and a search radius 10% above
    the support, Cole EOS rho0 = 1000, gamma = 7, c0 = 20 m/s."""
    h = 1.3 * dp
    skin = kw.pop("skin", 0.1)
    return Params(dp=dp, h=h, r_search=2.0 * h * (1.0 + skin), **kw)


def still_water(dp: float = 0.02, side: float = 0.4, **kw) -> Scene:
    """Tank side^3 full of water at rest, 3 boundary layers on floor and walls."""
    p = sph_params(dp, **kw)
    n = int(round(side / dp))
    xf = lattice(n, n, n, dp)
    xb = tank_walls(n, n, n, dp)
    L = n * dp
    lo = (-3 * dp, -3 * dp, -3 * dp)
    hi = (L + 3 * dp, L + 3 * dp, L + 0.5 * L)
    grid = make_grid(lo, hi, p.r_search)
    return _assemble("still_water", grid, p, xf, xb, H=L, meta={"H": L})


def dam_break(dp: float = 0.0043, box=(1.6, 0.67, 0.6), column=(0.4, 0.67, 0.3),
              u0_sigma: float = 0.0, seed: int = 1, **kw) -> Scene:
    """Water column in the corner x = 0 of an open-top box, 3 wall layers."""
    p = sph_params(dp, **kw)
    Nx, Ny, Nz = (int(math.floor(b / dp + 1e-9)) for b in box)
    cx, cz = int(math.floor(column[0] / dp + 1e-9)), int(math.floor(column[2] / dp + 1e-9))
    xf = lattice(cx, Ny, cz, dp)
    xb = tank_walls(Nx, Ny, Nz, dp)
    lo = (-3 * dp, -3 * dp, -3 * dp)
    hi = (Nx * dp + 3 * dp, Ny * dp + 3 * dp, max(Nz * dp, 1.5 * cz * dp) + 0.3 * Nz * dp)
    grid = make_grid(lo, hi, p.r_search)
    vel_f = None
    if u0_sigma > 0:
        rng = np.random.default_rng(seed)
        vel_f = rng.normal(0.0, u0_sigma, size=xf.shape)
    return _assemble("dam_break", grid, p, xf, xb, H=cz * dp, vel_f=vel_f,
                     meta={"H": cz * dp, "box": (Nx, Ny, Nz), "column": (cx, Ny, cz)})


def channel(dp: float = 0.005, length=4.0, width=1.0, depth=0.5, seed: int = 5,
            perturb: float = 1e-3, **kw) -> Scene:
    """Channel periodic in y: floor and x-end walls (3 layers), density
    hydrostatic times (1 + U[-perturb, perturb])."""
    p = sph_params(dp, **kw)
    Nx = int(round(length / dp))
    Ny = int(round(width / dp))
    Nz = int(round(depth / dp))
    xf = lattice(Nx, Ny, Nz, dp)
    xb = tank_walls(Nx, Ny, Nz, dp, walls_y=False)
    lo = (-3 * dp, 0.0, -3 * dp)
    hi = (Nx * dp + 3 * dp, Ny * dp, Nz * dp * 1.6)
    grid = make_grid(lo, hi, p.r_search, periodic=0b010)
    rng = np.random.default_rng(seed)
    scale = np.ones(xf.shape[0] + xb.shape[0])
    scale[: xf.shape[0]] += rng.uniform(-perturb, perturb, size=xf.shape[0])
    return _assemble("channel", grid, p, xf, xb, H=Nz * dp, rho_scale=scale,
                     meta={"H": Nz * dp})


def periodic_box(n: int = 8, dp: float = 0.02, jitter: float = 0.0, u_sigma: float = 0.0,
                 rho_sigma: float = 0.0, seed: int = 0, boundary_frac: float = 0.0, **kw) -> Scene:
    """Fully periodic cube of n^3 lattice particles with optional jitter of
    positions, random velocities and density noise; a fraction of the
    particles may be typed as boundary (zero velocity).  Test input only."""
    kw.setdefault("g", (0.0, 0.0, 0.0))
    p = sph_params(dp, **kw)
    rng = np.random.default_rng(seed)
    x = lattice(n, n, n, dp)
    if jitter > 0:
        x = x + rng.uniform(-jitter, jitter, size=x.shape) * dp
    L = n * dp
    x %= L
    grid = make_grid((0.0, 0.0, 0.0), (L, L, L), p.r_search, periodic=0b111)
    nb = int(round(boundary_frac * x.shape[0]))
    order = rng.permutation(x.shape[0])
    xb = x[order[:nb]]
    xf = x[order[nb:]]
    vel_f = rng.normal(0.0, u_sigma, size=xf.shape) if u_sigma > 0 else None
    sc = _assemble("periodic_box", grid, p, xf, xb, H=0.0, vel_f=vel_f)
    if rho_sigma > 0:
        sc.vel[:, 3] = (p.rho0 * (1.0 + rng.normal(0.0, rho_sigma, size=sc.n))).astype(np.float32)
    return sc


def random_cloud(n: int = 500, box=(0.2, 0.2, 0.2), dp: float = 0.02, u_sigma: float = 0.05,
                 rho_sigma: float = 0.005, boundary_frac: float = 0.2, periodic: int = 0,
                 seed: int = 0, **kw) -> Scene:
    """Uniformly random particles in a box (clustered or sparse regions and
    empty cells appear naturally).  Test input only."""
    kw.setdefault("g", (0.0, 0.0, -9.81))
    p = sph_params(dp, **kw)
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    x = rng.uniform(0.0, 1.0, size=(n, 3)) * box[None, :]
    grid = make_grid((0.0, 0.0, 0.0), tuple(box), p.r_search, periodic=periodic)
    nb = int(round(boundary_frac * n))
    xb, xf = x[:nb], x[nb:]
    vel_f = rng.normal(0.0, u_sigma, size=xf.shape) if u_sigma > 0 else None
    sc = _assemble("random_cloud", grid, p, xf, xb, H=0.0, vel_f=vel_f)
    sc.vel[:, 3] = (p.rho0 * (1.0 + rng.normal(0.0, rho_sigma, size=sc.n))).astype(np.float32)
    return sc


def adversarial_pairs(n_pairs: int = 60, dp: float = 0.02, seed: int = 11, box: float = 0.6,
                      periodic: int = 0) -> Scene:
    """Pairs of particles placed at r_s (1 + k 2^-23), k in -3..3, along
    random oblique directions (double positions, then the float32
    encoding): separations within a few float32 roundings of the search
    radius, where the predicate's rounding order decides.  Test input only."""
    rng = np.random.default_rng(seed)
    p = sph_params(dp, g=(0.0, 0.0, 0.0))
    grid = make_grid((0.0, 0.0, 0.0), (box, box, box), p.r_search, periodic=periodic)
    rs = float(np.float32(p.r_search))
    xs = []
    for k in range(n_pairs):
        c = rng.uniform(0.25 * box, 0.75 * box, size=3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rs * (1.0 + (k % 7 - 3) * 2.0 ** -23)
        xs.append(c)
        xs.append(c + r * d)
    x = np.array(xs)
    cell, off = encode_positions(grid, x)
    n = x.shape[0]
    pos = np.zeros((n, 4), np.float32)
    pos[:, :3] = off
    pos[:, 3] = np.float32(p.rho0 * dp ** 3)
    vel = np.zeros((n, 4), np.float32)
    vel[:, 3] = np.float32(p.rho0)
    info = np.arange(n, dtype=np.uint32)
    return Scene("adversarial_pairs", grid, p, cell, pos, vel, info, n, 0)


def shuffled(scene: Scene, seed: int = 0) -> Scene:
    """Same particles in a random storage order (ids keep their values)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(scene.n)
    s = scene.copy()
    s.cell, s.pos, s.vel, s.info = scene.cell[perm], scene.pos[perm], scene.vel[perm], scene.info[perm]
    return s


def dam_break_1m(**kw) -> Scene:
    """Dam break with ~1M fluid particles (dp = 4.3 mm)."""
    return dam_break(dp=0.0043, **kw)


def dam_break_64k(seed: int = 2, **kw) -> Scene:
    """Differentiable dam break, ~64k fluid particles, u0 ~ N(0, 0.01 m/s)."""
    return dam_break(dp=0.0107, u0_sigma=0.01, seed=seed, **kw)


def channel_16m(**kw) -> Scene:
    """Channel periodic in y with ~16M fluid particles (dp = 5 mm)."""
    return channel(dp=0.005, **kw)


def batched_tanks(n_scenes: int = 128, seed: int = 4, dp: float = 0.01,
                  n_min: int = 2000, n_max: int = 60000):
    """Independent tanks: fluid count log-uniform in [n_min, n_max], column
    aspect (height/length) uniform in [0.3, 2], alpha uniform in [0.005, 0.05].
    Column L x L x aL, tank 3L x L x 1.5 max(aL, L)."""
    rng = np.random.default_rng(seed)
    scenes = []
    cell_base = 0
    for s in range(n_scenes):
        nf_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        a = rng.uniform(0.3, 2.0)
        alpha = rng.uniform(0.005, 0.05)
        L = dp * (nf_target / a) ** (1.0 / 3.0)
        nl = max(2, int(round(L / dp)))
        nh = max(2, int(round(a * L / dp)))
        Nx, Ny, Nz = 3 * nl, nl, int(math.ceil(1.5 * max(nh, nl)))
        p = sph_params(dp, alpha=alpha)
        xf = lattice(nl, nl, nh, dp)
        xb = tank_walls(Nx, Ny, Nz, dp)
        lo = (-3 * dp, -3 * dp, -3 * dp)
        hi = (Nx * dp + 3 * dp, Ny * dp + 3 * dp, Nz * dp + 0.5 * Nz * dp)
        grid = make_grid(lo, hi, p.r_search, cell_base=cell_base)
        sc = _assemble("tank%03d" % s, grid, p, xf, xb, H=nh * dp, meta={"H": nh * dp, "aspect": a})
        cell_base += grid.n_cells
        scenes.append(sc)
    return scenes


CONFIGS = {
    "still_water_8k": lambda: still_water(0.02),
    "dam_break_1m": dam_break_1m,
    "dam_break_64k": dam_break_64k,
    "channel_16m": channel_16m,
}


BRICK_CELLS = 3


def stack_scenes(scenes, gap_cells: int = 2):
    """Lay independent scenes out in one grid, stacked along z, so that one
    neighbour search and one set of launches covers all of them.

    Every scene must use the same particle spacing (hence the same search
    radius).  The common cell side is the float32 search radius on all axes;
    each scene keeps its particles' positions relative to its own lower
    corner, placed at an integer number of cells, so its cell-relative
    encoding is identical to the one it has alone on its own sub-grid
    (returned as `sub_grids`).  `gap_cells` empty cell layers separate
    consecutive scenes (more where needed to start each scene at a multiple
    of BRICK_CELLS cells), so no pair of particles of different scenes is ever
    listed.  Returns (combined Scene, per-cell alpha float32[n_cells],
    sub_grids, per-scene (first particle, count) in the combined input)."""
    rs = float(np.float32(scenes[0].params.r_search))
    for s in scenes:
        if float(np.float32(s.params.r_search)) != rs:
            raise ValueError("stacked scenes need a common search radius")
    cs = np.float32(rs)
    csd = float(cs)
    # each scene's extent in cells (its own grid rounded up to whole cells)
    ext = []
    for s in scenes:
        L = s.grid.ncell.astype(np.float64) * s.grid.cell_size.astype(np.float64)
        ext.append(np.ceil(L / csd - 1e-9).astype(np.int64))
    nx = int(max(e[0] for e in ext))
    ny = int(max(e[1] for e in ext))
    # scene origins at multiples of the 3-cell brick of the LDS kernels, so a
    # scene's cells take the same place in their bricks stacked or alone
    z0 = []
    z = 0
    for e in ext:
        z0.append(z)
        z += int(e[2]) + gap_cells
        z = -(-z // BRICK_CELLS) * BRICK_CELLS
    nz = z0[-1] + int(ext[-1][2])
    grid = Grid(origin=np.zeros(3), cell_size=np.full(3, cs, np.float32),
                ncell=np.array([nx, ny, nz], np.int32), periodic=0, cell_base=0)
    xs, types, rho, vel, mass = [], [], [], [], []
    sub_grids, ranges = [], []
    first = 0
    alpha = np.zeros(grid.n_cells, np.float32)
    for s, e, zz in zip(scenes, ext, z0):
        x = decode_positions(s.grid, s.cell, s.pos[:, :3]) - s.grid.origin[None, :]
        x[:, 2] += zz * csd
        xs.append(x)
        types.append((s.info >> np.uint32(TYPE_SHIFT)).astype(np.uint32))
        vel.append(s.vel)
        mass.append(s.pos[:, 3])
        sub = Grid(origin=np.array([0.0, 0.0, zz * csd]), cell_size=grid.cell_size.copy(),
                   ncell=np.array([nx, ny, int(e[2])], np.int32), periodic=0, cell_base=0)
        sub_grids.append(sub)
        ranges.append((first, s.n))
        first += s.n
        a = np.float32(s.params.alpha)
        alpha[zz * nx * ny:(zz + int(e[2])) * nx * ny] = a
    x = np.concatenate(xs)
    cell, off = encode_positions(grid, x)
    n = x.shape[0]
    pos = np.zeros((n, 4), np.float32)
    pos[:, :3] = off
    pos[:, 3] = np.concatenate(mass)
    info = (np.concatenate(types) << np.uint32(TYPE_SHIFT)) | np.arange(n, dtype=np.uint32)
    p0 = scenes[0].params
    params = Params(**{k: getattr(p0, k) for k in p0.__dataclass_fields__})
    sc = Scene("stacked", grid, params, cell, pos, np.concatenate(vel).astype(np.float32), info,
               sum(s.n_fluid for s in scenes), sum(s.n_boundary for s in scenes),
               {"scenes": len(scenes), "z0": z0})
    return sc, alpha, sub_grids, ranges


def scene_cells(stacked: Scene) -> np.ndarray:
    """Scene index of every cell of a grid made by stack_scenes: scene k
    owns the cell layers from its first one up to the next scene's (its gap
    layers included), the last scene up to the top."""
    z0 = list(stacked.meta["z0"])
    nx, ny, nz = (int(v) for v in stacked.grid.ncell)
    layer = np.zeros(nz, np.int32)
    for k, z in enumerate(z0):
        layer[z:] = k
    return np.repeat(layer, nx * ny).astype(np.int32)


def scene_on_subgrid(stacked: Scene, sub_grid: Grid, rng):
    """The particles [first, first + count) of a stacked scene re-encoded on
    their own sub-grid (same offsets, local cells), with their own ids."""
    first, count = rng
    x = decode_positions(stacked.grid, stacked.cell[first:first + count], stacked.pos[first:first + count, :3])
    cell, off = encode_positions(sub_grid, x)
    pos = stacked.pos[first:first + count].copy()
    pos[:, :3] = off
    info = stacked.info[first:first + count].copy()
    return Scene("sub", sub_grid, stacked.params, cell, pos, stacked.vel[first:first + count].copy(), info,
                 int(((info >> np.uint32(TYPE_SHIFT)) == FLUID).sum()),
                 int(((info >> np.uint32(TYPE_SHIFT)) == BOUNDARY).sum()))
