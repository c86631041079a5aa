"""The corrector half of the step in one kernel (sph_forces_corrector)
against the separate calls it replaces, sph_forces(state *) followed by
sph_integrate(stage 1): the entry point promises the same state n+1, clock
and derivatives bit for bit, so every comparison here is exact.  The
separate calls are themselves checked against the FP64 oracle in
test_gpu_parity.py (stage by stage and over a 10-step rollout)."""
import dataclasses

import numpy as np
import pytest

from workloads import scenes as S

from parity import log, make_sim, torch_sync

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _moving_cloud(seed, **kw):
    return S.shuffled(S.random_cloud(n=1800, box=(0.3, 0.2, 0.25), dp=0.02, seed=seed, boundary_frac=0.35,
                                     u_sigma=0.3, rho_sigma=0.01, alpha=0.2, **kw), seed=seed + 1)


def _dropped_cloud():
    # particles pushed out of the (non-periodic) grid are dropped by the
    # build (cell < 0): the corrector leaves them as they are
    sc = _moving_cloud(41)
    rng = np.random.default_rng(42)
    k = rng.choice(sc.n, size=40, replace=False)
    sc.pos[k[:30], 0] += np.float32(0.4)
    sc.pos[k[30:], 2] -= np.float32(0.35)
    return sc


def _isolated_dam_break():
    # a small dam break with a few fluid particles alone in the empty part of
    # the tank: no neighbour, so the corrector reaches them in the pass over
    # the particles with an empty list
    sc = S.dam_break(dp=0.02, box=(0.8, 0.3, 0.4), column=(0.2, 0.3, 0.2))
    x = S.decode_positions(sc.grid, sc.cell, sc.pos[:, :3])
    k = np.arange(5)
    x[k] = np.array([[0.5 + 0.06 * j, 0.15, 0.25] for j in range(5)])
    cell, off = S.encode_positions(sc.grid, x)
    sc.cell[:] = cell
    sc.pos[:, :3] = off
    sc.vel[k, 0] = np.float32(0.3)
    return sc


def _variant(sc, kernel, visc, form, delta):
    return dataclasses.replace(sc, params=dataclasses.replace(sc.params, kernel=kernel, visc_model=visc, nu=2e-3,
                                                              formulation=form, delta=delta))


SCENES = {
    "still_water": (lambda: S.still_water(), 128),
    "cloud_boundary": (lambda: _moving_cloud(31), 192),
    "cloud_periodic_xyz": (lambda: _moving_cloud(33, periodic=0b111), 192),
    "cloud_dropped": (_dropped_cloud, 192),
    "cloud_cubic_morris_landrini_diffusion": (lambda: _variant(_moving_cloud(35), 1, 1, 1, 0.1), 192),
    "cloud_gaussian_monaghan_k": (lambda: _variant(_moving_cloud(37), 3, 2, 0, 0.0), 192),
    "dam_break_64k": (lambda: S.dam_break_64k(), 128),
    "isolated_fluid": (_isolated_dam_break, 128),
}


def _state(sim):
    return (sim.pos.clone(), sim.vel.clone(), sim.d_time.clone())


def _restore(sim, st):
    sim.pos.copy_(st[0])
    sim.vel.copy_(st[1])
    sim.d_time.copy_(st[2])


@pytest.mark.parametrize("bricks", [True, False], ids=["bricks", "gather"])
@pytest.mark.parametrize("name", list(SCENES))
def test_corrector_equals_separate_calls(name, bricks):
    """One step's corrector on the same predicted state both ways: state
    n+1, the clock and the derivatives agree bit for bit (capacity above n,
    so the rows past n must stay untouched too)."""
    make, M = SCENES[name]
    sc = make()
    log("case %s bricks=%s n=%d" % (name, bricks, sc.n))
    sim = make_sim(sc, max_neibs=M, capacity=sc.n + 61, use_bricks=bricks)
    sim.build()
    st = sim.status_host()
    assert st["overflow"] == 0
    if name == "cloud_dropped":
        assert st["dropped"] > 0
    if name == "isolated_fluid":
        cnt = sim.neib_count[: sc.n].cpu().numpy()
        info = sim.info[: sc.n].cpu().numpy().view(np.uint32)
        assert ((cnt == 0) & ((info >> 30) == 0)).sum() >= 5, "fluid particles with an empty list"
    sim.forces(False)
    sim.step_dt()
    sim.integrate(0)
    sim.d_time.fill_(0.125)
    before = _state(sim)
    # separate calls
    sim.forces(True)
    sim.integrate(1)
    torch_sync()
    sep = _state(sim)
    f_sep = sim.forces_star.clone()
    # one kernel, with the derivatives also written out
    _restore(sim, before)
    f_out = torch.full_like(sim.forces_star, float("nan"))
    sim.corrector(forces=f_out)
    torch_sync()
    fused = _state(sim)
    n = sc.n
    assert torch.equal(fused[0], sep[0]), "positions"
    assert torch.equal(fused[1], sep[1]), "velocities and densities"
    assert torch.equal(fused[2], sep[2]), "clock"
    assert torch.equal(f_out[:n], f_sep[:n]), "derivatives"
    assert torch.isnan(f_out[n:]).all(), "rows past n written"
    # the step moved the state (not a no-op that matches trivially)
    assert not torch.equal(fused[1][:n], before[1][:n])
    if name == "cloud_dropped":
        gone = sim.cell[:n] < 0
        assert int(gone.sum()) > 0
        assert torch.equal(fused[0][:n][gone], before[0][:n][gone])
        assert torch.equal(fused[1][:n][gone], before[1][:n][gone])
    # without the derivatives written out: the same state
    _restore(sim, before)
    sim.corrector()
    torch_sync()
    again = _state(sim)
    assert all(torch.equal(a, b) for a, b in zip(again, sep))


@pytest.mark.parametrize("bricks", [True, False], ids=["bricks", "gather"])
def test_rollout_fused_equals_separate(bricks):
    """25 steps of the 64k dam break (three rebuilds, adaptive dt): the step
    with the fused corrector and the step with the separate calls stay
    identical bit for bit, eagerly and as HIP graph replays."""
    sc = S.dam_break_64k()
    a = make_sim(sc, use_bricks=bricks)
    b = make_sim(sc, use_bricks=bricks)
    assert a.fuse_corrector
    b.fuse_corrector = False
    a.run(25)
    b.run(25)
    torch_sync()
    assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel) and torch.equal(a.cell, b.cell)
    assert a.time == b.time > 0.0
    # graph replays of the fused unit against the eager separate steps
    c = make_sim(sc, use_bricks=bricks)
    c.capture_unit()
    d = make_sim(sc, use_bricks=bricks)
    d.fuse_corrector = False
    for rep in range(3):
        c.replay_units(1)
        d.run(10)
        torch_sync()
        log("replay %d: t = %.9e" % (rep, c.time))
        assert torch.equal(c.pos, d.pos) and torch.equal(c.vel, d.vel), rep
        assert c.time == d.time


def test_empty_scene_advances_the_clock():
    """n = 0: nothing to update, but the clock advances by dt, as the
    separate corrector stage's does."""
    sc = S.still_water()
    sim = make_sim(sc)
    sim.n = 0
    sim.parts.n = 0
    sim.parts_star.n = 0
    sim.build()
    sim.d_dt.fill_(2.5e-4)
    sim.d_time.fill_(1.0)
    sim.corrector()
    torch_sync()
    assert float(sim.d_time.item()) == 1.0 + 2.5e-4


def test_corrector_rejects_shared_state():
    """state n and state * may not share storage (the kernel reads staged
    neighbours of state * while it rewrites state n): an error, no launch."""
    from paper_2207_11328_amd import abi
    sc = S.still_water()
    sim = make_sim(sc)
    sim.build()
    with pytest.raises(abi.SphError):
        abi.sph_forces_corrector(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, sim.d_dt,
                                 sim.parts, sim.ws_forces, cell_start=sim.cell_start, cell_end=sim.cell_end,
                                 neibs_brick=sim.neibs_brick)


def _stacked(cut_scene=None):
    from paper_2207_11328_amd.sim import Simulation
    tanks = S.batched_tanks(n_scenes=5, seed=21, n_min=400, n_max=3000)
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    table = S.scene_cells(stacked)
    if cut_scene is not None:
        table = table.copy()
        table[table == cut_scene] = -1  # that tank's cells: no scene

    def make():
        return Simulation(stacked.grid, stacked.params, stacked.cell, stacked.pos, stacked.vel, stacked.info,
                          cell_alpha=alpha, cell_scene=table)
    return stacked, make


@pytest.mark.parametrize("cut", [None, 2], ids=["all_scenes", "a_tank_of_no_scene"])
def test_corrector_scenes_equals_separate_calls(cut):
    """Batched tanks, each with its own step: one corrector both ways
    (sph_forces_corrector_scenes against sph_forces + sph_integrate_scenes),
    bit for bit, clocks included; a tank whose cells belong to no scene keeps
    its state."""
    stacked, make = _stacked(cut)
    sim = make()
    sim.build()
    sim.forces(False)
    sim.step_dt()
    sim.integrate(0)
    torch_sync()
    dts = sim.d_dt.cpu().numpy()
    log("per-scene steps %s" % np.array2string(dts, precision=6))
    sim.d_time.copy_(torch.arange(sim.n_scenes, dtype=torch.float64, device=sim.d_time.device) * 0.5)
    before = _state(sim)
    sim.forces(True)
    sim.integrate(1)
    torch_sync()
    sep = _state(sim)
    _restore(sim, before)
    sim.corrector()
    torch_sync()
    fused = _state(sim)
    assert all(torch.equal(a, b) for a, b in zip(fused, sep))
    n = stacked.n
    assert not torch.equal(fused[1][:n], before[1][:n])
    if cut is not None:
        sc = sim.cell_scene[(sim.cell[:n] - sim.g.cell_base).clamp(min=0).long()]
        alone = (sc < 0) & (sim.cell[:n] >= 0)
        assert int(alone.sum()) > 0
        assert torch.equal(fused[0][:n][alone], before[0][:n][alone])
        assert torch.equal(fused[1][:n][alone], before[1][:n][alone])


def test_batched_rollout_fused_equals_separate():
    """20 steps of batched tanks with per-scene adaptive steps, fused and
    separate corrector, eagerly and as graph replays: identical bits and
    clocks."""
    stacked, make = _stacked()
    a, b = make(), make()
    b.fuse_corrector = False
    a.run(20)
    b.run(20)
    torch_sync()
    assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel)
    assert np.array_equal(a.time, b.time)
    c = make()
    c.capture_unit()
    for rep in range(2):
        c.replay_units(1)
        torch_sync()
    assert torch.equal(c.pos, b.pos) and torch.equal(c.vel, b.vel)
    assert np.array_equal(c.time, b.time)
