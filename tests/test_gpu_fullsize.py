"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the 1.62M-particle dam break (the benchmark workload) and
the 16.6M-particle channel periodic in y (the largest workload; sizes near the
capacity limits of the list).  The sorted state, cell ranges, status and
interaction count are compared in full, bit for bit; neighbour sets (with
their cell codes) and derivatives on a seeded sample of particles, which the
oracle computes one by one."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import scenes as S

from parity import (SENT, check_forces, expected_codes_rows, gpu_lists_rows, log, make_sim, support_edge_rows,
                    torch_sync)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _full_size_case(sc, n_rows, seed):
    log("full size %s: n=%d cells=%d" % (sc.name, sc.n, sc.grid.n_cells))
    sim = make_sim(sc)
    sim.build()
    sim.forces()
    sim.count_interactions()
    torch_sync()
    log("gpu done")
    ss = O.sorted_f32(sc.grid, sc.cell, sc.pos, sc.vel, sc.info)
    log("oracle sort done")
    g = sim.state_host()
    assert np.array_equal(g["info"], ss["info"]), "sort order"
    assert np.array_equal(g["cell"], ss["cell"])
    assert np.array_equal(g["pos"].view(np.uint32), ss["pos"].view(np.uint32))
    nc = sc.grid.n_cells
    assert np.array_equal(sim.cell_start[:nc].cpu().numpy(), ss["start"])
    assert np.array_equal(sim.cell_end[:nc].cpu().numpy(), ss["end"])
    st = sim.status_host()
    assert st["n_active"] == ss["n_active"] == sc.n and st["overflow"] == 0
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(sc.n, size=n_rows, replace=False)).astype(np.int32)
    lists = O.neighbors_rows(sc.grid, sc.params, ss, rows)
    assert lists.overflow == 0
    fi, bi, fc, bc = gpu_lists_rows(sim, rows)
    col = np.arange(128)[None, :]
    ofi = np.sort(np.where(col < lists.nf[:, None], lists.fl.astype(np.int64), SENT), axis=1)
    obi = np.sort(np.where(col < lists.nb[:, None], lists.bl.astype(np.int64), SENT), axis=1)
    assert np.array_equal(fi, ofi) and np.array_equal(bi, obi), "neighbour sets"
    assert np.array_equal(fc, expected_codes_rows(sc.grid, ss["cell"], fi, rows))
    assert np.array_equal(bc, expected_codes_rows(sc.grid, ss["cell"], bi, rows))
    sto = O.State.lift(ss["cell"], ss["pos"], ss["vel"], ss["info"])
    acc, drho, sa, sd = O.forces_rows(sc.grid, sc.params, sto, rows, lists)
    check_forces(sim.forces_n[: sc.n].cpu().numpy()[rows], acc, drho, sa, sd, label=sc.name + " sampled")
    # the interaction count in full, against the oracle's float32 count (all rows, in chunks)
    total = 0
    for k in range(0, sc.n, 1 << 18):
        r = np.arange(k, min(sc.n, k + (1 << 18)), dtype=np.int32)
        lk = O.neighbors_rows(sc.grid, sc.params, ss, r)
        total += O.count_interactions_rows(sc.grid, sc.params, ss, r, lk)
    assert int(sim.count.item()) == total
    log("%s: interactions %d" % (sc.name, total))


def test_full_size_dam_break_1m():
    _full_size_case(S.dam_break_1m(), n_rows=20000, seed=1)


@pytest.mark.parametrize("variant", [(3, 2, 1, 0.1), (1, 1, 0, 0.0)],
                         ids=["gaussian-monaghan_k-landrini-diffusion", "cubic-morris-golden"])
def test_full_size_model_variants(variant):
    """Two compiled models on the 1.62M dam break (velocities N(0, 0.2 m/s)
    and densities 0.5% noisy, so every viscous and diffusive term is active),
    the LDS brick form the benchmark times, against the oracle on a seeded
    sample of particles."""
    import dataclasses
    kernel, visc, form, delta = variant
    sc = S.dam_break_1m()
    rng = np.random.default_rng(91)
    sc.vel[: sc.n_fluid, :3] = rng.normal(0.0, 0.2, size=(sc.n_fluid, 3)).astype(np.float32)
    sc.vel[:, 3] *= (1.0 + 0.005 * rng.standard_normal(sc.n)).astype(np.float32)
    sc = dataclasses.replace(sc, params=dataclasses.replace(sc.params, kernel=kernel, visc_model=visc, nu=1e-3,
                                                              formulation=form, delta=delta))
    log("full size variant %s: n=%d" % (variant, sc.n))
    sim = make_sim(sc)
    sim.build()
    sim.forces()
    torch_sync()
    ss = O.sorted_f32(sc.grid, sc.cell, sc.pos, sc.vel, sc.info)
    assert np.array_equal(sim.state_host()["info"], ss["info"]), "sort order"
    rows = np.sort(rng.choice(sc.n, size=6000, replace=False)).astype(np.int32)
    lists = O.neighbors_rows(sc.grid, sc.params, ss, rows)
    assert lists.overflow == 0
    sto = O.State.lift(ss["cell"], ss["pos"], ss["vel"], ss["info"])
    acc, drho, sa, sd = O.forces_rows(sc.grid, sc.params, sto, rows, lists)
    exclude = None
    if kernel == O.GAUSSIAN:
        exclude = support_edge_rows(sc, ss, rows=rows, lists=lists)
        log("  %d sampled particles with a pair at the support edge left out" % int(exclude.sum()))
        assert exclude.mean() < 0.005
    check_forces(sim.forces_n[: sc.n].cpu().numpy()[rows], acc, drho, sa, sd, label="dam break 1m %s" % (variant,),
                 exclude=exclude)


@pytest.mark.slow
def test_full_size_channel_16m():
    sc = S.channel_16m()
    log("channel: %d particles" % sc.n)
    sim = make_sim(sc)
    sim.build()
    sim.forces()
    torch_sync()
    ss = O.sorted_f32(sc.grid, sc.cell, sc.pos, sc.vel, sc.info)
    g = sim.state_host()
    assert np.array_equal(g["info"], ss["info"]) and np.array_equal(g["cell"], ss["cell"])
    assert np.array_equal(g["pos"].view(np.uint32), ss["pos"].view(np.uint32))
    assert sim.status_host()["overflow"] == 0
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(sc.n, size=20000, replace=False)).astype(np.int32)
    lists = O.neighbors_rows(sc.grid, sc.params, ss, rows)
    fi, bi, fc, bc = gpu_lists_rows(sim, rows)
    col = np.arange(128)[None, :]
    ofi = np.sort(np.where(col < lists.nf[:, None], lists.fl.astype(np.int64), SENT), axis=1)
    obi = np.sort(np.where(col < lists.nb[:, None], lists.bl.astype(np.int64), SENT), axis=1)
    assert np.array_equal(fi, ofi) and np.array_equal(bi, obi)
    assert np.array_equal(fc, expected_codes_rows(sc.grid, ss["cell"], fi, rows))
    sto = O.State.lift(ss["cell"], ss["pos"], ss["vel"], ss["info"])
    acc, drho, sa, sd = O.forces_rows(sc.grid, sc.params, sto, rows, lists)
    check_forces(sim.forces_n[: sc.n].cpu().numpy()[rows], acc, drho, sa, sd, label="channel_16m sampled")
