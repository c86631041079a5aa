"""Pins of the oracle's time step and of its double-precision rebuild.

orc_dt: the adaptive step of section "The GPU in GPUSPH" (a device
reduction of the largest sound speed and acceleration), read as
dt = CFL min(h / max c, sqrt(h / max |a + g|), 0.125 h^2 / nu) over fluid
particles.  Each test makes one of the three limits bind on a hand-built
state and compares with that limit written out, with the sound speed taken
from Cole's law c = c0 (rho/rho0)^((gamma - 1)/2) (section "A lightning
introduction to the method").

orc_rebin_f64 and the double predicate of orc_neighbors feed every double
rollout of the oracle (rollout, rollout_adjoint): the re-binning is checked
against its definition in exact rational arithmetic (the offset moves by
whole cells into [-cs/2, cs/2), the physical position is unchanged, periodic
axes wrap, particles leaving a closed axis are dropped), against the float32
re-binning where both are exact, and the double lists against the O(N^2)
brute force on the geometry before the re-binning (section "Optimizing the
neighbors search").
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute as B
from oracle import oracle as O
from workloads import scenes as S

TYPE_SHIFT = 30


# ------------------------------------------------------------------ dt
def _dt_state(rho, acc, types, cells):
    n = len(rho)
    info = (np.asarray(types, np.uint32) << np.uint32(TYPE_SHIFT)) | np.arange(n, dtype=np.uint32)
    st = O.State(np.asarray(cells, np.int32), np.zeros((n, 3)), np.ones(n), np.zeros((n, 3)),
                 np.asarray(rho, np.float64), info)
    return st, np.ascontiguousarray(acc, dtype=np.float64)


def _params(**kw):
    base = dict(dp=0.02, h=0.026, r_search=0.0572, g=(0.0, 0.0, -9.81), cfl=0.3, c0=20.0, nu=0.0)
    base.update(kw)
    return S.Params(**base)


def _f(x):
    return float(np.float32(x))


def _cole_c(p, rho):
    return _f(p.c0) * (rho / _f(p.rho0)) ** ((_f(p.gamma) - 1.0) / 2.0)


# four fluid particles, one boundary particle, one fluid particle dropped by
# the last build (cell -1)
TYPES = [0, 0, 0, 0, 1, 0]
CELLS = [0, 1, 2, 3, 4, -1]


def test_dt_sound_speed_limit():
    """rho = rho0 (1 + delta) on one particle: the sound speed limit with
    c = c0 (1 + delta)^3 (gamma = 7) binds."""
    p = _params()
    rho0 = _f(p.rho0)
    rho = [rho0, rho0 * 1.02, rho0, rho0 * 0.99, rho0, rho0]
    acc = np.zeros((6, 3))
    st, acc = _dt_state(rho, acc, TYPES, CELLS)
    got = O.dt(p, st, acc)
    cmax = _cole_c(p, rho0 * 1.02)
    assert abs(cmax - _f(p.c0) * 1.02 ** 3) < 1e-12 * cmax
    want = _f(p.cfl) * _f(p.h) / cmax
    # the acceleration limit sqrt(h / g) is far above it
    assert math.sqrt(_f(p.h) / 9.81) > 10 * want
    assert abs(got - want) <= 1e-13 * want


def test_dt_acceleration_limit_includes_gravity():
    """With a slow sound speed, the acceleration limit binds; gravity is
    added to the SPH acceleration before taking the magnitude: a = (3, 4,
    9.81) and g = (0, 0, -9.81) give |a + g| = 5, not |a| = 11.0."""
    p = _params(c0=0.01)
    rho0 = _f(p.rho0)
    rho = [rho0] * 6
    acc = np.zeros((6, 3))
    acc[:, 2] = -_f(-9.81)              # the others: a + g = 0
    acc[1] = (3.0, 4.0, -_f(-9.81))     # |a + g| = 5
    st, acc = _dt_state(rho, acc, TYPES, CELLS)
    got = O.dt(p, st, acc)
    want = _f(p.cfl) * math.sqrt(_f(p.h) / 5.0)
    assert _f(p.h) / _cole_c(p, rho0) > 10 * want
    assert abs(got - want) <= 1e-13 * want


def test_dt_viscous_limit():
    """nu > 0 adds 0.125 h^2 / nu, which binds for a large viscosity."""
    p = _params(nu=1.0)
    rho0 = _f(p.rho0)
    st, acc = _dt_state([rho0] * 6, np.zeros((6, 3)), TYPES, CELLS)
    got = O.dt(p, st, acc)
    h = _f(p.h)
    want = _f(p.cfl) * 0.125 * h * h / _f(p.nu)
    assert h / _f(p.c0) > 10 * want
    assert abs(got - want) <= 1e-13 * want


def test_dt_ignores_boundary_and_dropped_particles():
    """A boundary particle and a dropped fluid particle with huge
    accelerations and densities do not change the step."""
    p = _params()
    rho0 = _f(p.rho0)
    rho = [rho0] * 6
    acc = np.zeros((6, 3))
    st, acc0 = _dt_state(rho, acc, TYPES, CELLS)
    base = O.dt(p, st, acc0)
    rho2 = list(rho)
    rho2[4] = 2 * rho0
    rho2[5] = 2 * rho0
    acc2 = acc.copy()
    acc2[4] = (1e7, 0.0, 0.0)
    acc2[5] = (0.0, -1e7, 0.0)
    st2, acc2 = _dt_state(rho2, acc2, TYPES, CELLS)
    assert O.dt(p, st2, acc2) == base
    assert abs(base - _f(p.cfl) * _f(p.h) / _f(p.c0)) <= 1e-13 * base


def test_dt_scales_with_cfl():
    """dt is proportional to the safety factor on every branch."""
    for kw in ({}, {"c0": 0.01}, {"nu": 1.0}):
        a = _params(cfl=0.25, **kw)
        b = _params(cfl=0.5, **kw)
        rho0 = _f(a.rho0)
        acc = np.zeros((6, 3))
        acc[1] = (3.0, 4.0, 0.0)
        st, acc = _dt_state([rho0] * 6, acc, TYPES, CELLS)
        assert O.dt(b, st, acc) == 2.0 * O.dt(a, st, acc)


# ------------------------------------------------------------------ re-binning in double
def _coords(grid, cell):
    nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
    lc = cell.astype(np.int64) - int(grid.cell_base)
    return np.stack([lc % nx, (lc // nx) % ny, lc // (nx * ny)], axis=1)


def _rebin_exact(grid, cell, off):
    """The re-binning rule in exact rational arithmetic: per axis the offset
    moves by the whole number m of cells that brings it into [-cs/2, cs/2),
    |m| <= 4; a periodic axis wraps the cell, a closed one drops a particle
    that leaves it.  Returns (cell, offsets as Fractions, dropped mask)."""
    c = _coords(grid, cell)
    n = cell.shape[0]
    cell_out = np.full(n, -1, np.int64)
    off_out = [[None] * 3 for _ in range(n)]
    drop = np.zeros(n, bool)
    for i in range(n):
        cc = [0, 0, 0]
        for d in range(3):
            cs = Fraction(float(np.float32(grid.cell_size[d])))
            o = Fraction(float(off[i, d]))
            m = math.floor((o + cs / 2) / cs)
            if abs(m) > 4:
                drop[i] = True
            o2 = o - m * cs
            off_out[i][d] = o2
            cd = int(c[i, d]) + m
            if (grid.periodic >> d) & 1:
                cd %= int(grid.ncell[d])
            elif cd < 0 or cd >= int(grid.ncell[d]):
                drop[i] = True
            cc[d] = cd
        if not drop[i]:
            nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
            cell_out[i] = cc[0] + nx * (cc[1] + ny * cc[2]) + int(grid.cell_base)
    return cell_out, off_out, drop


@pytest.mark.parametrize("periodic", [0, 0b111, 0b010])
def test_rebin_f64_is_the_exact_rule(periodic):
    """Double offsets spread over +-4.6 cells: every kept particle's offset
    is the exact o - m cs (so the position is unchanged bit for bit) inside
    [-cs/2, cs/2), its cell moved by m (wrapped on periodic axes), and
    exactly the escapees are dropped."""
    rng = np.random.default_rng(20 + periodic)
    grid = S.make_grid((0.0, 0.0, 0.0), (0.48, 0.42, 0.36), 0.05, periodic=periodic, cell_base=7)
    n = 600
    c = np.stack([rng.integers(0, int(grid.ncell[d]), n) for d in range(3)], axis=1)
    nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
    cell = (c[:, 0] + nx * (c[:, 1] + ny * c[:, 2]) + grid.cell_base).astype(np.int32)
    cs = grid.cell_size.astype(np.float64)
    off = rng.uniform(-4.6, 4.6, size=(n, 3)) * cs[None, :]
    # offsets on the boundaries of the rule: exactly +-cs/2 and +-4.5 cs
    off[:6, 0] = [0.5 * cs[0], -0.5 * cs[0], 4.5 * cs[0], -4.5 * cs[0], 1.5 * cs[0], -1.5 * cs[0]]
    st = O.State(cell, off, np.ones(n), np.zeros((n, 3)), np.full(n, 1000.0), np.arange(n, dtype=np.uint32))
    cell_x, off_x, drop_x = _rebin_exact(grid, cell, off)
    # the oracle's double re-binning (through its rebuild: re-bin, sort, lists)
    p = S.Params(dp=0.02, h=0.02, r_search=0.05)
    st2, _, perm, dropped = O.rebuild_f64(grid, p, st)
    assert dropped == int(drop_x.sum()) and dropped > 0
    for k in range(n):
        i = int(perm[k])
        if drop_x[i]:
            assert st2.cell[k] == -1
            continue
        assert st2.cell[k] == cell_x[i]
        for d in range(3):
            o = Fraction(float(st2.off[k, d]))
            assert o == off_x[i][d], (i, d)
            assert -Fraction(float(np.float32(cs[d]))) / 2 <= o < Fraction(float(np.float32(cs[d]))) / 2


def test_rebin_f64_equals_f32_rebin_on_float32_exact_offsets():
    """Where every subtraction is exact in float32 (cs = 1/4, offsets on a
    2^-10 grid), the double and float32 re-binnings agree bit for bit."""
    rng = np.random.default_rng(5)
    grid = S.make_grid((0.0, 0.0, 0.0), (2.0, 1.5, 2.0), 0.25, periodic=0b010)
    assert np.all(grid.cell_size == np.float32(0.25))
    n = 500
    c = np.stack([rng.integers(0, int(grid.ncell[d]), n) for d in range(3)], axis=1)
    nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
    cell = (c[:, 0] + nx * (c[:, 1] + ny * c[:, 2])).astype(np.int32)
    off = rng.integers(-4 * 256 - 100, 4 * 256 + 100, size=(n, 3)) / 1024.0
    pos = np.zeros((n, 4), np.float32)
    pos[:, :3] = off.astype(np.float32)
    assert np.array_equal(pos[:, :3].astype(np.float64), off)
    c32, p32, d32 = O.rebin_f32(grid, cell, pos)
    st = O.State(cell, off, np.ones(n), np.zeros((n, 3)), np.ones(n), np.arange(n, dtype=np.uint32))
    st2, _, perm, d64 = O.rebuild_f64(grid, S.Params(dp=0.1, h=0.1, r_search=0.25), st)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    assert d32 == d64 > 0
    assert np.array_equal(st2.cell[inv], c32)
    ok = c32 >= 0
    assert np.array_equal(st2.off[inv][ok], p32[ok, :3].astype(np.float64))


# ------------------------------------------------------------------ double lists
def _ids(info):
    return (np.asarray(info, np.uint32) & np.uint32((1 << TYPE_SHIFT) - 1)).astype(np.int64)


@pytest.mark.parametrize("periodic,seed", [(0, 1), (0b111, 2), (0b101, 3)])
def test_double_lists_match_brute_force_before_rebinning(periodic, seed):
    """A random cloud whose offsets drifted by up to +-1 cell in double (|o| up to 1.5 cells):
    the oracle's double rebuild (re-bin, sort, double predicate) lists the
    same neighbours, by particle id and type, as the O(N^2) double brute
    force on the drifted state before re-binning.  With at least 8 cells on
    a periodic axis and |o| <= 1.5 cells, a pair within r_s has a cell
    difference of at most 3, so the brute force's nearest image by cell is
    the true one."""
    sc = S.random_cloud(n=2400, box=(0.48, 0.48, 0.48), dp=0.02, periodic=periodic, seed=seed, boundary_frac=0.2)
    assert np.all(sc.grid.ncell >= 8)
    rng = np.random.default_rng(100 + seed)
    st0 = O.State.lift(sc.cell, sc.pos, sc.vel, sc.info)
    cs = sc.grid.cell_size.astype(np.float64)
    drift = rng.uniform(-1.0, 1.0, size=(sc.n, 3)) * cs[None, :] * (rng.uniform(size=(sc.n, 1)) < 0.5)
    st0.off = st0.off + drift
    # keep the cloud inside the closed axes (no drops in this test)
    x = O.positions(sc.grid, st0)
    L = sc.grid.ncell * sc.grid.cell_size.astype(np.float64)
    for d in range(3):
        if not (periodic >> d) & 1:
            out = (x[:, d] < 0) | (x[:, d] >= L[d])
            st0.off[out, d] -= drift[out, d]
    st, lists, perm, dropped = O.rebuild_f64(sc.grid, sc.params, st0)
    assert dropped == 0
    moved = np.any(st.cell != st0.cell[perm])
    assert moved
    # brute force on the state before re-binning (cells and drifted offsets)
    pos64 = np.zeros((sc.n, 4))
    pos64[:, :3] = st0.off
    sets = B.neighbor_sets(sc.grid, sc.params.r_search, st0.cell, pos64, st0.info, fp64=True)
    ids0 = _ids(st0.info)
    ids = _ids(st.info)
    by_id = {int(ids0[i]): (set(ids0[f].tolist()), set(ids0[b].tolist())) for i, (f, b) in enumerate(sets)}
    total = 0
    for k in range(sc.n):
        want_f, want_b = by_id[int(ids[k])]
        got_f = set(ids[lists.fluid(k)].tolist())
        got_b = set(ids[lists.boundary(k)].tolist())
        assert got_f == want_f and got_b == want_b, k
        total += len(got_f) + len(got_b)
    assert total > 10 * sc.n


def test_double_and_float_predicates_differ_only_near_the_radius():
    """On the same float32 encoding, the double predicate and the float32
    one disagree only for pairs within 2^-20 r_s^2 of the search radius."""
    sc = S.random_cloud(n=1200, box=(0.3, 0.3, 0.3), dp=0.02, seed=8)
    b = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info)
    l64 = O.neighbors(sc.grid, sc.params, b["cell"], b["info"], b["start"], b["end"],
                      off=b["pos"][:, :3].astype(np.float64))
    r2 = B.pair_r2(sc.grid, b["cell"], b["pos"], fp64=True)
    rs = float(np.float32(sc.params.r_search))
    for i in range(sc.n):
        a = set(b["lists"].fluid(i).tolist()) | set(b["lists"].boundary(i).tolist())
        c = set(l64.fluid(i).tolist()) | set(l64.boundary(i).tolist())
        for j in a ^ c:
            assert abs(r2[i, j] - rs * rs) < 2.0 ** -20 * rs * rs


# ------------------------------------------------------------------ missed pairs
M_CLOUD = 256   # list slots for the random clouds, which cluster (no overflow)

def _moved(sc, amp, seed):
    """The oracle's sorted build of a scene and, in its order, the float32
    offsets after a seeded displacement of up to amp dp per axis (fluid
    particles only; boundary particles are fixed)."""
    b = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, max_neibs=M_CLOUD)
    assert b["lists"].overflow == 0
    rng = np.random.default_rng(seed)
    fluid = (b["info"] >> TYPE_SHIFT) == 0
    d = rng.uniform(-amp, amp, size=(sc.n, 3)) * sc.params.dp * fluid[:, None]
    # no particle leaves a closed axis (none is dropped by the rebuild)
    x = S.decode_positions(sc.grid, b["cell"], b["pos"][:, :3].astype(np.float64) + d)
    L = sc.grid.ncell * sc.grid.cell_size.astype(np.float64)
    for a in range(3):
        if not (sc.grid.periodic >> a) & 1:
            d[(x[:, a] < 0.0) | (x[:, a] >= L[a]), a] = 0.0
    pos = b["pos"].copy()
    pos[:, :3] = (pos[:, :3].astype(np.float64) + d).astype(np.float32)
    return b, pos


@pytest.mark.parametrize("amp,periodic", [(0.05, 0), (0.4, 0), (0.9, 0b011)])
def test_missed_pairs_are_the_pairs_within_2h_absent_from_the_old_lists(amp, periodic):
    """The oracle's missed-pair count equals the brute-force count of pairs
    (i, j) with float32 r < 2h at the rebuild (after re-binning, boundary-
    boundary pairs excluded) whose j is not in i's previous list; its two
    parts are the brute-force counts of those pairs and of the old lists'
    pairs within 2h."""
    sc = S.random_cloud(n=1500, box=(0.3, 0.26, 0.24), dp=0.02, periodic=periodic, seed=31, boundary_frac=0.25)
    old, pos = _moved(sc, amp, seed=40)
    i_old, i_new, missed = O.missed_pairs(sc.grid, sc.params, old, pos, max_neibs=M_CLOUD)
    # brute force at the rebuild on the re-binned encoding
    cell, pos2, dropped = O.rebin_f32(sc.grid, old["cell"], pos)
    assert dropped == 0
    r2 = B.pair_r2(sc.grid, cell, pos2)
    two_h = np.float32(2.0 * np.float32(sc.params.h))
    within = r2 < np.float32(two_h * two_h)
    np.fill_diagonal(within, False)
    typ = old["info"] >> TYPE_SHIFT
    within &= ~((typ[:, None] == 1) & (typ[None, :] == 1))
    in_old = np.zeros_like(within)
    L = old["lists"]
    for i in range(sc.n):
        in_old[i, L.fluid(i)] = True
        in_old[i, L.boundary(i)] = True
    assert i_new == int(within.sum())
    assert missed == int((within & ~in_old).sum())
    assert i_old == int((within & in_old).sum())
    if amp <= 0.05:
        assert missed == 0      # well inside the skin (0.1 x 2h = 0.26 dp)
    else:
        assert missed > 0


def test_nonfinite_count_of_the_build():
    sc = S.random_cloud(n=300, box=(0.2, 0.2, 0.2), dp=0.02, seed=3)
    pos, vel = sc.pos.copy(), sc.vel.copy()
    vel[5, 3] = np.nan       # density
    vel[9, 0] = np.inf       # velocity
    pos[11, 3] = -np.inf     # mass
    pos[17, 1] = np.nan      # offset (also dropped by the re-binning)
    vel[17, 2] = np.nan      # the same particle counts once
    b = O.build_f32(sc.grid, sc.params, sc.cell, pos, vel, sc.info)
    assert b["nonfinite"] == 4 and b["dropped"] == 1
