"""Batched scenes: independent tanks stacked in one grid and advanced by the
same launches (one neighbour search, one derivative launch, ... per step),
and the HIP-graph capture of a rebuild unit.

* parity: each scene's batched derivatives against the FP64 oracle run on
  that scene alone, with its own alpha (1e-5 of the pair-term scale);
* batched == single: 20 fixed-dt steps of the batch equal, bit for bit, the
  same 20 steps of each scene run alone on its own grid, and so do 30 steps
  with each scene's own adaptive dt (per-scene time steps and clocks);
* per-scene dt against the oracle's dt of each scene alone;
* independence: perturbing one scene leaves every other scene bit-identical,
  with fixed and with adaptive dt;
* graph: replays of a captured 10-step unit equal the eager steps bit for bit,
  with eager work and synchronisations between replays."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import scenes as S

from parity import check_forces, log, make_sim, torch_sync

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _tanks(n=6, seed=9):
    return S.batched_tanks(n_scenes=n, seed=seed, n_min=400, n_max=3000)


def _batch_sim(stacked, alpha, dt=None, scenes=True):
    from paper_2207_11328_amd.sim import Simulation
    return Simulation(stacked.grid, stacked.params, stacked.cell, stacked.pos, stacked.vel, stacked.info,
                      cell_alpha=alpha, dt_fixed=dt, cell_scene=S.scene_cells(stacked) if scenes else None)


def _by_id(sim):
    st = sim.state_host()
    ids = (st["info"] & np.uint32((1 << 30) - 1)).astype(np.int64)
    o = np.argsort(ids)
    return ids[o], st["pos"][o], st["vel"][o]


def test_batched_forces_parity_per_scene():
    tanks = _tanks()
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    log("batch: %d scenes, %d particles, grid %s" % (len(tanks), stacked.n, list(stacked.grid.ncell)))
    sim = _batch_sim(stacked, alpha)
    sim.build()
    sim.forces()
    torch_sync()
    st = sim.state_host()
    f = sim.forces_n[: stacked.n].cpu().numpy()
    ids = (st["info"] & np.uint32((1 << 30) - 1)).astype(np.int64)
    for k, (t, sub, rng) in enumerate(zip(tanks, subs, ranges)):
        one = S.scene_on_subgrid(stacked, sub, rng)
        one.params = t.params  # its own alpha
        ob = O.build_f32(one.grid, one.params, one.cell, one.pos, one.vel, one.info)
        sto = O.State.lift(ob["cell"], ob["pos"], ob["vel"], ob["info"])
        acc, drho, sa, sd, _ = O.forces(one.grid, one.params, sto, ob["lists"])
        oid = (ob["info"] & np.uint32((1 << 30) - 1)).astype(np.int64)
        where = {v: i for i, v in enumerate(ids)}
        rows = np.array([where[v] for v in oid])
        check_forces(f[rows], acc, drho, sa, sd, label="scene %d (alpha %.4f)" % (k, t.params.alpha))


def test_batched_equals_single_bitwise_and_independent():
    tanks = _tanks()
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    dt = 2e-4
    sim = _batch_sim(stacked, alpha, dt)
    sim.run(20)
    torch_sync()
    ids_b, pos_b, vel_b = _by_id(sim)
    from paper_2207_11328_amd.sim import Simulation
    for k, (t, sub, rng) in enumerate(zip(tanks, subs, ranges)):
        one = S.scene_on_subgrid(stacked, sub, rng)
        s1 = Simulation(one.grid, t.params, one.cell, one.pos, one.vel, one.info, dt_fixed=dt)
        s1.run(20)
        torch_sync()
        ids_1, pos_1, vel_1 = _by_id(s1)
        first, count = rng
        sel = slice(first, first + count)
        assert np.array_equal(ids_b[sel], ids_1)
        # offsets are relative to cells that differ only by the scene's z base
        assert np.array_equal(pos_b[sel].view(np.uint32), pos_1.view(np.uint32)), k
        assert np.array_equal(vel_b[sel].view(np.uint32), vel_1.view(np.uint32)), k
    # independence: perturb scene 2 only
    pert = stacked.copy()
    first, count = ranges[2]
    pert.vel[first:first + count, :3] += np.float32(0.05)
    sim2 = _batch_sim(pert, alpha, dt)
    sim2.run(20)
    torch_sync()
    ids_p, pos_p, vel_p = _by_id(sim2)
    for k, (first, count) in enumerate(ranges):
        sel = slice(first, first + count)
        same = np.array_equal(pos_p[sel].view(np.uint32), pos_b[sel].view(np.uint32)) and \
            np.array_equal(vel_p[sel].view(np.uint32), vel_b[sel].view(np.uint32))
        assert same == (k != 2), k


def test_graph_replay_equals_eager():
    tanks = _tanks(n=4, seed=11)
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    eager = _batch_sim(stacked, alpha)
    graph = _batch_sim(stacked, alpha)
    graph.capture_unit()
    torch_sync()
    # capturing ran nothing
    assert graph.steps_done == 0 and bool(torch.all(graph.d_time == 0.0))
    for unit in range(3):
        eager.run(10)
        graph.replay_units(1)
        junk = torch.randn(1000, device=graph.device).sum()  # eager work between replays
        torch_sync()
        assert torch.equal(eager.pos, graph.pos) and torch.equal(eager.vel, graph.vel), unit
        assert torch.equal(eager.d_time, graph.d_time)
        assert torch.equal(eager.neibs, graph.neibs)
        del junk
    log("graph replay == eager over 3 units, t = %s s" % np.array2string(graph.time, precision=6))


def test_per_scene_dt_matches_oracle():
    """sph_step_dt_scenes: each tank's step from its own particles, against
    the oracle's dt of that tank alone (1e-5), and equal to the single-scene
    step of the tank on its own grid bit for bit."""
    from paper_2207_11328_amd.sim import Simulation
    tanks = _tanks()
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    sim = _batch_sim(stacked, alpha)
    sim.build()
    sim.forces()
    sim.step_dt()
    torch_sync()
    dts = sim.d_dt.cpu().numpy()
    assert dts.shape == (len(tanks),)
    for k, (t, sub, rng) in enumerate(zip(tanks, subs, ranges)):
        one = S.scene_on_subgrid(stacked, sub, rng)
        ob = O.build_f32(one.grid, t.params, one.cell, one.pos, one.vel, one.info)
        sto = O.State.lift(ob["cell"], ob["pos"], ob["vel"], ob["info"])
        acc, _, _, _, _ = O.forces(one.grid, t.params, sto, ob["lists"])
        dt_o = O.dt(t.params, sto, acc)
        s1 = Simulation(one.grid, t.params, one.cell, one.pos, one.vel, one.info)
        s1.build()
        s1.forces()
        s1.step_dt()
        torch_sync()
        dt_1 = float(s1.d_dt.item())
        log("scene %d: dt batched %.9e alone %.9e oracle %.9e" % (k, dts[k], dt_1, dt_o))
        assert abs(dts[k] - dt_o) <= 1e-5 * dt_o
        assert dts[k] == dt_1
    # the tanks' steps differ: one shared step would couple them
    assert len(set(dts.tolist())) > 1


def test_adaptive_dt_batched_equals_single_and_independent():
    """30 steps with each tank's own adaptive dt (per-scene steps and clocks):
    every tank equals, bit for bit, the same tank run alone with its own
    adaptive dt, and perturbing one tank leaves the others' bits and clocks
    unchanged."""
    from paper_2207_11328_amd.sim import Simulation
    tanks = _tanks()
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    steps = 30
    sim = _batch_sim(stacked, alpha)
    sim.run(steps)
    torch_sync()
    clocks = sim.time
    ids_b, pos_b, vel_b = _by_id(sim)
    for k, (t, sub, rng) in enumerate(zip(tanks, subs, ranges)):
        one = S.scene_on_subgrid(stacked, sub, rng)
        s1 = Simulation(one.grid, t.params, one.cell, one.pos, one.vel, one.info)
        s1.run(steps)
        torch_sync()
        ids_1, pos_1, vel_1 = _by_id(s1)
        first, count = rng
        sel = slice(first, first + count)
        assert np.array_equal(ids_b[sel], ids_1)
        assert np.array_equal(pos_b[sel].view(np.uint32), pos_1.view(np.uint32)), k
        assert np.array_equal(vel_b[sel].view(np.uint32), vel_1.view(np.uint32)), k
        assert clocks[k] == s1.time, k
    log("per-scene clocks after %d steps: %s" % (steps, np.array2string(clocks, precision=6)))
    pert = stacked.copy()
    first, count = ranges[2]
    pert.vel[first:first + count, :3] += np.float32(0.05)
    sim2 = _batch_sim(pert, alpha)
    sim2.run(steps)
    torch_sync()
    clocks2 = sim2.time
    ids_p, pos_p, vel_p = _by_id(sim2)
    for k, (first, count) in enumerate(ranges):
        sel = slice(first, first + count)
        same = np.array_equal(pos_p[sel].view(np.uint32), pos_b[sel].view(np.uint32)) and \
            np.array_equal(vel_p[sel].view(np.uint32), vel_b[sel].view(np.uint32)) and clocks2[k] == clocks[k]
        assert same == (k != 2), k


def test_cells_of_no_scene_are_left_alone():
    """A cell whose scene entry is outside [0, n_scenes) belongs to no scene:
    its particles keep their state through sph_integrate_scenes and count in
    no scene's step (the other tanks step exactly as with the full table)."""
    from paper_2207_11328_amd.sim import Simulation
    tanks = _tanks(n=4, seed=13)
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    table = S.scene_cells(stacked)
    cut = table.copy()
    cut[cut == 1] = -1  # tank 1's cells: no scene
    full = Simulation(stacked.grid, stacked.params, stacked.cell, stacked.pos, stacked.vel, stacked.info,
                      cell_alpha=alpha, cell_scene=table)
    part = Simulation(stacked.grid, stacked.params, stacked.cell, stacked.pos, stacked.vel, stacked.info,
                      cell_alpha=alpha, cell_scene=cut)
    assert part.n_scenes == len(tanks)
    for s in (full, part):
        s.build()
        s.forces()
        s.step_dt()
    torch_sync()
    dt_full = full.d_dt.cpu().numpy()
    dt_part = part.d_dt.cpu().numpy()
    assert np.array_equal(dt_part[[0, 2, 3]], dt_full[[0, 2, 3]])
    # scene 1 now holds no particle: only the laminar limit, if any, bounds it
    p = stacked.params
    h, nu, cfl = float(np.float32(p.h)), float(np.float32(p.nu)), float(np.float32(p.cfl))
    assert dt_part[1] == (cfl * (0.125 * h * h / nu) if nu > 0 else np.inf)
    before = part.state_host()
    part.d_dt[1] = 1e-4  # any step: the tank's particles must still stay put
    part.integrate(0)
    part.integrate(1)
    torch_sync()
    after = part.state_host()
    first, count = ranges[1]
    ids = (before["info"] & np.uint32((1 << 30) - 1)).astype(np.int64)
    sel = (ids >= first) & (ids < first + count)
    assert sel.sum() == count
    assert np.array_equal(after["pos"][sel].view(np.uint32), before["pos"][sel].view(np.uint32))
    assert np.array_equal(after["vel"][sel].view(np.uint32), before["vel"][sel].view(np.uint32))
    assert not np.array_equal(after["pos"][~sel].view(np.uint32), before["pos"][~sel].view(np.uint32))
