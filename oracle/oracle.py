"""Python front end of the FP64 CPU oracle (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product package.

The oracle consumes the canonical float32 encoded state and lifts it exactly
to float64.  Scalar parameters are lifted the same way (their float32 value,
which is what the GPU library receives), so both sides solve exactly the same
problem.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

TYPE_SHIFT = 30
BOUNDARY = 1


class OrcGrid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("cs", C.c_float * 3), ("n", C.c_int32 * 3),
                ("periodic", C.c_uint32), ("cell_base", C.c_int32)]


class OrcParams(C.Structure):
    _fields_ = [("h", C.c_double), ("r_search", C.c_double), ("rho0", C.c_double),
                ("gamma", C.c_double), ("c0", C.c_double), ("alpha", C.c_double),
                ("eps_visc", C.c_double), ("nu", C.c_double), ("g", C.c_double * 3),
                ("cfl", C.c_double), ("visc_model", C.c_int32), ("delta", C.c_double),
                ("kernel", C.c_int32), ("formulation", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32 = C.c_int
        L.orc_rebin.argtypes = [P, i32, P, P]
        L.orc_rebin.restype = i32
        L.orc_rebin_f64.argtypes = [P, i32, P, P]
        L.orc_rebin_f64.restype = i32
        L.orc_sort_perm.argtypes = [i32, P, P, P]
        L.orc_sort_perm.restype = None
        L.orc_cell_ranges.argtypes = [P, i32, P, P, P]
        L.orc_cell_ranges.restype = None
        L.orc_neighbors.argtypes = [P, C.c_float, i32, P, P, P, P, P, P, i32, P, P, P, P]
        L.orc_neighbors.restype = i32
        L.orc_forces.argtypes = [P, P, i32, P, P, P, P, P, P, P, P, P, P, i32, P, P, P, P, P]
        L.orc_forces.restype = None
        L.orc_count_interactions_f32.argtypes = [P, C.c_float, i32, P, P, P, P, P, P, i32]
        L.orc_count_interactions_f32.restype = C.c_int64
        L.orc_integrate.argtypes = [P, i32, C.c_double, i32, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_integrate.restype = None
        L.orc_dt.argtypes = [P, i32, P, P, P, P]
        L.orc_dt.restype = C.c_double
        for nm in ("orc_kernel_W", "orc_kernel_F", "orc_kernel_dF"):
            getattr(L, nm).argtypes = [i32, C.c_double, C.c_double]
            getattr(L, nm).restype = C.c_double
        L.orc_wendland_W.argtypes = [C.c_double, C.c_double]
        L.orc_wendland_W.restype = C.c_double
        L.orc_wendland_F.argtypes = [C.c_double, C.c_double]
        L.orc_wendland_F.restype = C.c_double
        L.orc_pressure.argtypes = [P, C.c_double]
        L.orc_pressure.restype = C.c_double
        L.orc_sound_speed.argtypes = [P, C.c_double]
        L.orc_sound_speed.restype = C.c_double
        L.orc_threads.argtypes = []
        L.orc_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return a.ctypes.data_as(C.c_void_p)


def f32(x) -> float:
    """The float32 value of a parameter, as a Python float."""
    return float(np.float32(x))


def grid_struct(grid) -> OrcGrid:
    g = OrcGrid()
    for d in range(3):
        g.origin[d] = float(grid.origin[d])
        g.cs[d] = float(grid.cell_size[d])
        g.n[d] = int(grid.ncell[d])
    g.periodic = int(grid.periodic)
    g.cell_base = int(grid.cell_base)
    return g


def params_struct(p, alpha=None) -> OrcParams:
    """Parameters as the GPU receives them (float32 values lifted to double),
    unless p.exact_values is set (finite-difference checks of the oracle)."""
    rnd = float if getattr(p, "exact_values", False) else f32
    q = OrcParams()
    q.h = rnd(p.h)
    q.r_search = rnd(p.r_search)
    q.rho0 = rnd(p.rho0)
    q.gamma = rnd(p.gamma)
    q.c0 = rnd(p.c0)
    q.alpha = rnd(p.alpha if alpha is None else alpha)
    q.eps_visc = rnd(p.eps_visc)
    q.nu = rnd(p.nu)
    for d in range(3):
        q.g[d] = rnd(p.g[d])
    q.cfl = rnd(p.cfl)
    q.visc_model = int(p.visc_model)
    q.delta = rnd(getattr(p, "delta", 0.0))
    q.kernel = int(getattr(p, "kernel", 0))
    q.formulation = int(getattr(p, "formulation", 0))
    return q


def set_threads(t: int):
    lib().orc_set_threads(int(t))


def threads() -> int:
    return int(lib().orc_threads())


# ---------------------------------------------------------------- kernel / EOS
def wendland_W(r: float, h: float) -> float:
    return lib().orc_wendland_W(float(r), float(h))


def wendland_F(r: float, h: float) -> float:
    return lib().orc_wendland_F(float(r), float(h))


# smoothing kernels of listing l:ktemplate (support 2h)
WENDLAND, CUBIC_SPLINE, QUADRATIC, GAUSSIAN = 0, 1, 2, 3
KERNELS = {"wendland": WENDLAND, "cubic_spline": CUBIC_SPLINE, "quadratic": QUADRATIC, "gaussian": GAUSSIAN}


def kernel_W(kind: int, r: float, h: float) -> float:
    return lib().orc_kernel_W(int(kind), float(r), float(h))


def kernel_F(kind: int, r: float, h: float) -> float:
    """F = (1/r) dW/dr."""
    return lib().orc_kernel_F(int(kind), float(r), float(h))


def kernel_dF(kind: int, r: float, h: float) -> float:
    """dF/dr."""
    return lib().orc_kernel_dF(int(kind), float(r), float(h))


def pressure(params, rho: float) -> float:
    ps = params_struct(params)
    return lib().orc_pressure(C.byref(ps), float(rho))


def sound_speed(params, rho: float) -> float:
    ps = params_struct(params)
    return lib().orc_sound_speed(C.byref(ps), float(rho))


# ---------------------------------------------------------------- state
class State:
    """Double-precision particle state (cell-relative offsets)."""

    def __init__(self, cell, off, mass, vel, rho, info):
        self.cell = np.ascontiguousarray(cell, dtype=np.int32)
        self.off = np.ascontiguousarray(off, dtype=np.float64)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        self.vel = np.ascontiguousarray(vel, dtype=np.float64)
        self.rho = np.ascontiguousarray(rho, dtype=np.float64)
        self.info = np.ascontiguousarray(info, dtype=np.uint32)

    @property
    def n(self):
        return self.cell.shape[0]

    def copy(self):
        return State(self.cell.copy(), self.off.copy(), self.mass.copy(), self.vel.copy(),
                     self.rho.copy(), self.info.copy())

    def take(self, perm):
        return State(self.cell[perm], self.off[perm], self.mass[perm], self.vel[perm],
                     self.rho[perm], self.info[perm])

    @property
    def is_fluid(self):
        return (self.info >> TYPE_SHIFT) != BOUNDARY

    @staticmethod
    def lift(cell, pos, vel, info) -> "State":
        """Exact float32 -> float64 lift of the canonical encoding."""
        pos = np.asarray(pos, dtype=np.float32)
        vel = np.asarray(vel, dtype=np.float32)
        return State(cell, pos[:, :3].astype(np.float64), pos[:, 3].astype(np.float64),
                     vel[:, :3].astype(np.float64), vel[:, 3].astype(np.float64), info)


# ---------------------------------------------------------------- neighbour search
class Lists:
    def __init__(self, nf, nb, fl, bl, max_neibs, overflow):
        self.nf, self.nb, self.fl, self.bl = nf, nb, fl, bl
        self.max_neibs = max_neibs
        self.overflow = overflow

    def fluid(self, i):
        return self.fl[i, : self.nf[i]]

    def boundary(self, i):
        return self.bl[i, : self.nb[i]]


def rebin_f32(grid, cell, pos):
    """Float32 re-binning (in copies).  Returns (cell, pos, dropped)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32).copy()
    pos = np.ascontiguousarray(pos, dtype=np.float32).copy()
    g = grid_struct(grid)
    dropped = lib().orc_rebin(C.byref(g), cell.shape[0], _p(cell), _p(pos))
    return cell, pos, int(dropped)


def sort_perm(cell, info) -> np.ndarray:
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    info = np.ascontiguousarray(info, dtype=np.uint32)
    perm = np.zeros(cell.shape[0], dtype=np.int32)
    lib().orc_sort_perm(cell.shape[0], _p(cell), _p(info), _p(perm))
    return perm


def cell_ranges(grid, cell_sorted):
    cell_sorted = np.ascontiguousarray(cell_sorted, dtype=np.int32)
    nc = grid.n_cells
    start = np.zeros(nc, dtype=np.int32)
    end = np.zeros(nc, dtype=np.int32)
    g = grid_struct(grid)
    lib().orc_cell_ranges(C.byref(g), cell_sorted.shape[0], _p(cell_sorted), _p(start), _p(end))
    return start, end


def neighbors(grid, params, cell, info, start, end, max_neibs=128, pos=None, off=None) -> Lists:
    """Split neighbour lists from the float32 predicate (pos given) or the
    double predicate (off given)."""
    n = cell.shape[0]
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    info = np.ascontiguousarray(info, dtype=np.uint32)
    nf = np.zeros(n, dtype=np.int32)
    nb = np.zeros(n, dtype=np.int32)
    fl = np.zeros((n, max_neibs), dtype=np.int32)
    bl = np.zeros((n, max_neibs), dtype=np.int32)
    g = grid_struct(grid)
    if pos is not None:
        pos = np.ascontiguousarray(pos, dtype=np.float32)
        pp, op = _p(pos), None
    else:
        off = np.ascontiguousarray(off, dtype=np.float64)
        pp, op = None, _p(off)
    ov = lib().orc_neighbors(C.byref(g), C.c_float(f32(params.r_search)), n, _p(cell), pp, op,
                             _p(info), _p(start), _p(end), max_neibs, _p(nf), _p(nb), _p(fl), _p(bl))
    return Lists(nf, nb, fl, bl, max_neibs, int(ov))


def build_f32(grid, params, cell, pos, vel, info, max_neibs=128):
    """Re-bin, sort, cell ranges and float32-predicate lists of a float32
    encoded state.  Returns a dict with the sorted float32 arrays."""
    cell, pos, dropped = rebin_f32(grid, cell, pos)
    perm = sort_perm(cell, info)
    cell, pos, vel, info = cell[perm], pos[perm], np.asarray(vel)[perm], np.asarray(info)[perm]
    n_active = int((cell >= 0).sum())
    start, end = cell_ranges(grid, cell)
    lists = neighbors(grid, params, cell, info, start, end, max_neibs, pos=pos)
    return dict(cell=np.ascontiguousarray(cell), pos=np.ascontiguousarray(pos),
                vel=np.ascontiguousarray(vel), info=np.ascontiguousarray(info), perm=perm,
                start=start, end=end, lists=lists, n_active=n_active, dropped=dropped,
                nonfinite=nonfinite_count(pos, vel))


def nonfinite_count(pos, vel) -> int:
    """Particles with a non-finite offset, mass, velocity or density."""
    pos = np.asarray(pos, dtype=np.float32)
    vel = np.asarray(vel, dtype=np.float32)
    return int((~np.isfinite(pos).all(axis=1) | ~np.isfinite(vel).all(axis=1)).sum())


def missed_pairs(grid, params, old, pos_now, max_neibs=128):
    """Pairs within 2h that the lists of a previous build missed (section
    "Optimizing the neighbors search": lists built with an enlarged radius
    are reused for several steps).  old: a build_f32 result; pos_now: the
    float32 state [n, 4] at the next rebuild, in old's sorted order, offsets
    relative to old's cells.  Returns (interactions of old's lists at
    pos_now, interactions of the fresh lists, their difference): the fresh
    lists hold every pair within the search radius, so the difference counts
    the pairs within 2h missing from the old lists."""
    i_old = count_interactions_f32(grid, params, old["cell"], pos_now, old["lists"])
    new = build_f32(grid, params, old["cell"], pos_now, old["vel"], old["info"], max_neibs)
    i_new = count_interactions_f32(grid, params, new["cell"], new["pos"], new["lists"])
    return i_old, i_new, i_new - i_old


def rebuild_f64(grid, params, st: State, max_neibs=128):
    """Double-precision rebuild of a double state: re-bin, sort, lists."""
    st = st.copy()
    g = grid_struct(grid)
    dropped = lib().orc_rebin_f64(C.byref(g), st.n, _p(st.cell), _p(st.off))
    perm = sort_perm(st.cell, st.info)
    st = st.take(perm)
    start, end = cell_ranges(grid, st.cell)
    lists = neighbors(grid, params, st.cell, st.info, start, end, max_neibs, off=st.off)
    return st, lists, perm, int(dropped)


# ---------------------------------------------------------------- derivatives / integration
def forces(grid, params, st: State, lists: Lists, alpha=None):
    """Returns (acc [n,3], drho [n], s_acc [n,3], s_drho [n], n_interactions)."""
    n = st.n
    acc = np.zeros((n, 3))
    drho = np.zeros(n)
    s_acc = np.zeros((n, 3))
    s_drho = np.zeros(n)
    ninter = C.c_int64(0)
    g = grid_struct(grid)
    ps = params_struct(params, alpha)
    lib().orc_forces(C.byref(ps), C.byref(g), n, _p(st.cell), _p(st.off), _p(st.mass), _p(st.vel),
                     _p(st.rho), _p(st.info), _p(lists.nf), _p(lists.nb), _p(lists.fl), _p(lists.bl),
                     lists.max_neibs, _p(acc), _p(drho), _p(s_acc), _p(s_drho), C.byref(ninter))
    return acc, drho, s_acc, s_drho, int(ninter.value)


def count_interactions_f32(grid, params, cell, pos, lists: Lists) -> int:
    g = grid_struct(grid)
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    return int(lib().orc_count_interactions_f32(C.byref(g), C.c_float(f32(params.h)), cell.shape[0],
                                                _p(cell), _p(pos), _p(lists.nf), _p(lists.nb),
                                                _p(lists.fl), _p(lists.bl), lists.max_neibs))


def integrate(params, stage, dt, st_n: State, acc, drho, vel_star=None) -> State:
    out = st_n.copy()
    ps = params_struct(params)
    vs = st_n.vel if vel_star is None else np.ascontiguousarray(vel_star, dtype=np.float64)
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    drho = np.ascontiguousarray(drho, dtype=np.float64)
    lib().orc_integrate(C.byref(ps), int(stage), float(dt), st_n.n, _p(st_n.cell), _p(st_n.info),
                        _p(st_n.off), _p(st_n.vel), _p(st_n.rho), _p(vs), _p(acc), _p(drho),
                        _p(out.off), _p(out.vel), _p(out.rho))
    return out


def dt(params, st: State, acc) -> float:
    ps = params_struct(params)
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    return float(lib().orc_dt(C.byref(ps), st.n, _p(st.cell), _p(st.info), _p(st.rho), _p(acc)))


def step(grid, params, st: State, lists: Lists, dt_fixed=None, alpha=None):
    """One predictor/corrector step on fixed lists.  Returns (state, dt)."""
    acc, drho, _, _, _ = forces(grid, params, st, lists, alpha)
    h = dt(params, st, acc) if dt_fixed is None else float(dt_fixed)
    star = integrate(params, 0, h, st, acc, drho)
    acc2, drho2, _, _, _ = forces(grid, params, star, lists, alpha)
    new = integrate(params, 1, h, st, acc2, drho2, vel_star=star.vel)
    return new, h


def rollout(grid, params, st: State, steps: int, rebuild_every: int = 10, max_neibs: int = 128,
            dt_fixed=None, callback=None):
    """Double-precision rollout with periodic rebuilds.  Returns (state, time)."""
    t = 0.0
    lists = None
    for s in range(steps):
        if s % rebuild_every == 0 or lists is None:
            st, lists, _, _ = rebuild_f64(grid, params, st, max_neibs)
        st, h = step(grid, params, st, lists, dt_fixed)
        t += h
        if callback is not None:
            callback(s, st, t)
    return st, t


def positions(grid, st: State) -> np.ndarray:
    """Physical positions (double) of a double state."""
    nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
    lc = st.cell.astype(np.int64) - int(grid.cell_base)
    c = np.stack([lc % nx, (lc // nx) % ny, lc // (nx * ny)], axis=1).astype(np.float64)
    cs = np.asarray(grid.cell_size, dtype=np.float32).astype(np.float64)
    return np.asarray(grid.origin, dtype=np.float64)[None, :] + (c + 0.5) * cs[None, :] + st.off


# ---------------------------------------------------------------- reverse mode
def _setup_reverse():
    L = lib()
    if getattr(L, "_rev_ready", False):
        return L
    P = C.c_void_p
    i32 = C.c_int
    L.orc_forces_reverse.argtypes = [P, P, i32, P, P, P, P, P, P, P, P, P, P, i32, P, P, P, P, P, P]
    L.orc_forces_reverse.restype = None
    L.orc_forces_reverse_scales.argtypes = [P, P, i32, P, P, P, P, P, P, P, P, P, P, i32, P, P, P, P, P, P]
    L.orc_forces_reverse_scales.restype = None
    L.orc_integrate_reverse.argtypes = [i32, C.c_double, i32, P, P, P, P, P, P, P, P, P, P, P]
    L.orc_integrate_reverse.restype = None
    L._rev_ready = True
    return L


class Adj:
    """Adjoint of a double state: offsets, velocities, densities."""

    def __init__(self, go, gu, grho):
        self.go = np.ascontiguousarray(go, dtype=np.float64)
        self.gu = np.ascontiguousarray(gu, dtype=np.float64)
        self.grho = np.ascontiguousarray(grho, dtype=np.float64)

    @staticmethod
    def zeros(n):
        return Adj(np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n))

    def copy(self):
        return Adj(self.go.copy(), self.gu.copy(), self.grho.copy())

    def __add__(self, o):
        return Adj(self.go + o.go, self.gu + o.gu, self.grho + o.grho)


def forces_reverse(grid, params, st: State, lists: Lists, abar, dbar, into: Adj | None = None, alpha=None):
    """Adds the reverse of forces() for upstream (abar, dbar) to `into` (or a
    new zero adjoint).  Returns (adjoint, gparams[alpha, c0, nu])."""
    L = _setup_reverse()
    adj = Adj.zeros(st.n) if into is None else into
    gp = np.zeros(3)
    g = grid_struct(grid)
    ps = params_struct(params, alpha)
    abar = np.ascontiguousarray(abar, dtype=np.float64)
    dbar = np.ascontiguousarray(dbar, dtype=np.float64)
    L.orc_forces_reverse(C.byref(ps), C.byref(g), st.n, _p(st.cell), _p(st.off), _p(st.mass), _p(st.vel),
                         _p(st.rho), _p(st.info), _p(lists.nf), _p(lists.nb), _p(lists.fl), _p(lists.bl),
                         lists.max_neibs, _p(abar), _p(dbar), _p(adj.go), _p(adj.gu), _p(adj.grho), _p(gp))
    return adj, gp


def forces_reverse_scales(grid, params, st: State, lists: Lists, abar, dbar, alpha=None):
    """Magnitude scales of forces_reverse (the reverse with every factor
    taken in absolute value): (Adj of scales, scales of gparams[3]).  The
    error gate of a float evaluation of the reverse is a multiple of these."""
    L = _setup_reverse()
    sc = Adj.zeros(st.n)
    sp = np.zeros(3)
    g = grid_struct(grid)
    ps = params_struct(params, alpha)
    abar = np.ascontiguousarray(abar, dtype=np.float64)
    dbar = np.ascontiguousarray(dbar, dtype=np.float64)
    L.orc_forces_reverse_scales(C.byref(ps), C.byref(g), st.n, _p(st.cell), _p(st.off), _p(st.mass), _p(st.vel),
                                _p(st.rho), _p(st.info), _p(lists.nf), _p(lists.nb), _p(lists.fl), _p(lists.bl),
                                lists.max_neibs, _p(abar), _p(dbar), _p(sc.go), _p(sc.gu), _p(sc.grho), _p(sp))
    return sc, sp


def integrate_reverse(stage, dt, st_n: State, adj_out: Adj):
    """Returns (adjoint of stage inputs without the derivative terms,
    gu_star (stage 1 only, else None), abar, dbar)."""
    L = _setup_reverse()
    n = st_n.n
    out = Adj.zeros(n)
    gu_star = np.zeros((n, 3)) if stage == 1 else None
    abar = np.zeros((n, 3))
    dbar = np.zeros(n)
    L.orc_integrate_reverse(int(stage), float(dt), n, _p(st_n.cell), _p(st_n.info), _p(adj_out.go),
                            _p(adj_out.gu), _p(adj_out.grho), _p(out.go), _p(out.gu), _p(out.grho),
                            _p(gu_star) if gu_star is not None else None, _p(abar), _p(dbar))
    return out, gu_star, abar, dbar


def step_reverse(grid, params, st_n: State, star: State, lists: Lists, dt, adj_next: Adj, alpha=None):
    """Reverse of step() with fixed dt: adjoint of state n and gparams."""
    gp = np.zeros(3)
    base1, gu_star, abar1, dbar1 = integrate_reverse(1, dt, st_n, adj_next)
    adj_star = Adj(np.zeros((st_n.n, 3)), gu_star, np.zeros(st_n.n))
    adj_star, g1 = forces_reverse(grid, params, star, lists, abar1, dbar1, into=adj_star, alpha=alpha)
    base0, _, abar0, dbar0 = integrate_reverse(0, dt, st_n, adj_star)
    adj_n = base1 + base0
    adj_n, g0 = forces_reverse(grid, params, st_n, lists, abar0, dbar0, into=adj_n, alpha=alpha)
    return adj_n, g0 + g1


def rollout_adjoint(grid, params, st0: State, steps: int, dt: float, loss_and_grad, rebuild_every: int = 10,
                    max_neibs: int = 128):
    """Double-precision rollout with a fixed time step and its reverse.

    loss_and_grad(final_state) -> (L, Adj of the final state).  Returns
    (L, Adj of st0 in st0's particle order, gparams[alpha, c0, nu], final state).
    Every state is kept (test sizes only)."""
    tape = []
    st = st0
    lists = None
    for s in range(steps):
        if s % rebuild_every == 0 or lists is None:
            st, lists, perm, _ = rebuild_f64(grid, params, st, max_neibs)
            tape.append(("perm", perm))
        acc, drho, _, _, _ = forces(grid, params, st, lists)
        star = integrate(params, 0, dt, st, acc, drho)
        acc2, drho2, _, _, _ = forces(grid, params, star, lists)
        new = integrate(params, 1, dt, st, acc2, drho2, vel_star=star.vel)
        tape.append(("step", st, star, lists))
        st = new
    Lval, adj = loss_and_grad(st)
    gp = np.zeros(3)
    for rec in reversed(tape):
        if rec[0] == "step":
            _, st_n, star, lists = rec
            adj, g = step_reverse(grid, params, st_n, star, lists, dt, adj)
            gp += g
        else:
            perm = rec[1]
            back = Adj.zeros(adj.go.shape[0])
            back.go[perm] = adj.go
            back.gu[perm] = adj.gu
            back.grho[perm] = adj.grho
            adj = back
    return Lval, adj, gp, st


def front_loss(grid, front_ids):
    """L = mean x of the particles whose ids are front_ids; returns a
    loss_and_grad callable for rollout_adjoint."""
    ids = np.asarray(front_ids, dtype=np.int64)

    def f(st: State):
        x = positions(grid, st)
        pid = (st.info & np.uint32((1 << TYPE_SHIFT) - 1)).astype(np.int64)
        sel = np.isin(pid, ids)
        L = x[sel, 0].mean()
        adj = Adj.zeros(st.n)
        adj.go[sel, 0] = 1.0 / sel.sum()
        return L, adj
    return f


# ---------------------------------------------------------------- very large inputs
def _setup_rows():
    L = lib()
    if getattr(L, "_rows_ready", False):
        return L
    P = C.c_void_p
    i32 = C.c_int
    L.orc_neighbors_rows.argtypes = [P, C.c_float, P, P, P, P, P, i32, P, i32, P, P, P, P]
    L.orc_neighbors_rows.restype = i32
    L.orc_forces_rows.argtypes = [P, P, P, P, P, P, P, P, P, i32, P, P, P, P, i32, P, P, P, P]
    L.orc_forces_rows.restype = None
    L.orc_count_interactions_rows.argtypes = [P, C.c_float, P, P, P, i32, P, P, P, P, i32]
    L.orc_count_interactions_rows.restype = C.c_int64
    L._rows_ready = True
    return L


def sorted_f32(grid, cell, pos, vel, info):
    """Re-bin, sort and cell ranges of a float32 encoded state (no lists)."""
    cell, pos, dropped = rebin_f32(grid, cell, pos)
    perm = sort_perm(cell, info)
    cell, pos, vel, info = cell[perm], pos[perm], np.asarray(vel)[perm], np.asarray(info)[perm]
    start, end = cell_ranges(grid, cell)
    return dict(cell=np.ascontiguousarray(cell), pos=np.ascontiguousarray(pos), vel=np.ascontiguousarray(vel),
                info=np.ascontiguousarray(info), perm=perm, start=start, end=end,
                n_active=int((cell >= 0).sum()), dropped=dropped)


def neighbors_rows(grid, params, sorted_state, rows, max_neibs=128) -> Lists:
    """Float32-predicate lists of the sorted particles `rows` (row-indexed)."""
    L = _setup_rows()
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    m = rows.shape[0]
    nf = np.zeros(m, np.int32)
    nb = np.zeros(m, np.int32)
    fl = np.zeros((m, max_neibs), np.int32)
    bl = np.zeros((m, max_neibs), np.int32)
    g = grid_struct(grid)
    ss = sorted_state
    ov = L.orc_neighbors_rows(C.byref(g), C.c_float(f32(params.r_search)), _p(ss["cell"]), _p(ss["pos"]),
                              _p(ss["info"]), _p(ss["start"]), _p(ss["end"]), max_neibs, _p(rows), m,
                              _p(nf), _p(nb), _p(fl), _p(bl))
    return Lists(nf, nb, fl, bl, max_neibs, int(ov))


def forces_rows(grid, params, st: State, rows, lists: Lists):
    """Derivatives of the particles `rows` of a double state, from
    row-indexed lists.  Returns (acc, drho, s_acc, s_drho), row-indexed."""
    L = _setup_rows()
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    m = rows.shape[0]
    acc = np.zeros((m, 3))
    drho = np.zeros(m)
    s_acc = np.zeros((m, 3))
    s_drho = np.zeros(m)
    g = grid_struct(grid)
    ps = params_struct(params)
    L.orc_forces_rows(C.byref(ps), C.byref(g), _p(st.cell), _p(st.off), _p(st.mass), _p(st.vel), _p(st.rho),
                      _p(st.info), _p(rows), m, _p(lists.nf), _p(lists.nb), _p(lists.fl), _p(lists.bl), lists.max_neibs,
                      _p(acc), _p(drho), _p(s_acc), _p(s_drho))
    return acc, drho, s_acc, s_drho


def count_interactions_rows(grid, params, sorted_state, rows, lists: Lists) -> int:
    L = _setup_rows()
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    g = grid_struct(grid)
    ss = sorted_state
    return int(L.orc_count_interactions_rows(C.byref(g), C.c_float(f32(params.h)), _p(ss["cell"]), _p(ss["pos"]),
                                             _p(rows), rows.shape[0], _p(lists.nf), _p(lists.nb), _p(lists.fl),
                                             _p(lists.bl), lists.max_neibs))
