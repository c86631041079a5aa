"""GPU checks made at each rebuild, against the oracle: the non-finite count
of the build's status word, the pairs within 2h that reused lists missed
(sph_count_missed_pairs), and the adjoint rollout's refusal to return
gradients from lists that overflowed.

Inputs are seeded clouds; the moved state of the missed-pair test is the
oracle's sorted state plus a seeded displacement (test-side input, not a GPU
output), written into the GPU buffers in that same order after checking that
the GPU sorted the particles identically.  Counts are compared bit-exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import scenes as S

from parity import log, make_sim, torch_sync

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

M_CLOUD = 256
TYPE_SHIFT = 30


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_nonfinite_state_is_reported_by_the_build():
    from paper_2207_11328_amd.abi import SphError
    sc = S.random_cloud(n=900, box=(0.24, 0.2, 0.2), dp=0.02, seed=61)
    pos, vel = sc.pos.copy(), sc.vel.copy()
    vel[5, 3] = np.nan       # density
    vel[9, 0] = np.inf       # velocity
    pos[11, 3] = -np.inf     # mass
    pos[17, 1] = np.nan      # offset (dropped as well)
    vel[17, 2] = np.nan
    vel[400, 1] = -np.inf
    bad = S.Scene(sc.name, sc.grid, sc.params, sc.cell, pos, vel, sc.info, sc.n_fluid, sc.n_boundary)
    ob = O.build_f32(sc.grid, sc.params, sc.cell, pos, vel, sc.info, max_neibs=M_CLOUD)
    log("nonfinite case n=%d oracle nonfinite=%d dropped=%d" % (sc.n, ob["nonfinite"], ob["dropped"]))
    sim = make_sim(bad, max_neibs=M_CLOUD)
    sim.build()
    torch_sync()
    st = sim.status_host()
    assert st["nonfinite"] == ob["nonfinite"] == 5
    assert st["dropped"] == ob["dropped"] == 1
    assert st["n_active"] == ob["n_active"]
    with pytest.raises(SphError, match="non-finite"):
        sim.check_status()
    # the same state without the planted values reports nothing
    ok = make_sim(sc, max_neibs=M_CLOUD)
    ok.build()
    torch_sync()
    assert ok.check_status()["nonfinite"] == 0


def _moved(sc, amp, seed, base=None):
    """Oracle build of the scene (or of `base`, a build_f32 result) and its
    float32 state after a seeded displacement of up to amp dp per axis of
    the fluid particles, in the build's sorted order; no particle leaves a
    closed axis."""
    b = base if base is not None else O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info,
                                                  max_neibs=M_CLOUD)
    rng = np.random.default_rng(seed)
    fluid = (b["info"] >> TYPE_SHIFT) == 0
    d = rng.uniform(-amp, amp, size=(sc.n, 3)) * sc.params.dp * fluid[:, None]
    x = S.decode_positions(sc.grid, b["cell"], b["pos"][:, :3].astype(np.float64) + d)
    L = sc.grid.ncell * sc.grid.cell_size.astype(np.float64)
    for a in range(3):
        if not (sc.grid.periodic >> a) & 1:
            d[(x[:, a] < 0.0) | (x[:, a] >= L[a]), a] = 0.0
    pos = b["pos"].copy()
    pos[:, :3] = (pos[:, :3].astype(np.float64) + d).astype(np.float32)
    return b, pos


@pytest.mark.parametrize("amp,periodic", [(0.05, 0), (0.4, 0), (0.9, 0b011), (0.6, 0b111)])
def test_missed_pairs_match_the_oracle(amp, periodic):
    """Two rebuilds of a moving cloud: each one's count of the previous
    lists' interactions, the new lists' interactions and their difference
    (the missed pairs), and the running total, equal the oracle's."""
    sc = S.random_cloud(n=2400, box=(0.32, 0.3, 0.26), dp=0.02, periodic=periodic, seed=71, boundary_frac=0.25)
    sim = make_sim(sc, max_neibs=M_CLOUD)
    sim.track_missed = True
    sim.build()
    torch_sync()
    old, pos = _moved(sc, amp, seed=81)
    assert np.array_equal(sim.state_host()["info"], old["info"]), "sort order"
    total = 0
    for rnd in range(2):
        log("missed pairs case amp=%.2f periodic=%d round %d" % (amp, periodic, rnd))
        i_old, i_new, missed = O.missed_pairs(sc.grid, sc.params, old, pos, max_neibs=M_CLOUD)
        sim.pos[: sc.n] = torch.from_numpy(pos).to(sim.device)
        sim.build()
        torch_sync()
        sim.check_status()
        got = sim.missed_host()
        total += missed
        log("  gpu %s oracle (%d, %d, %d)" % (got, i_old, i_new, missed))
        assert (got["previous_lists"], got["new_lists"], got["missed"]) == (i_old, i_new, missed)
        assert got["missed_total"] == total
        # the next round starts from the rebuilt state, in the oracle's new order
        nb = O.build_f32(sc.grid, sc.params, old["cell"], pos, old["vel"], old["info"], max_neibs=M_CLOUD)
        assert np.array_equal(sim.state_host()["info"], nb["info"])
        old, pos = _moved(sc, amp, seed=82 + rnd, base=nb)
    if amp <= 0.05:
        assert total == 0
    else:
        assert total > 0


def test_adjoint_rollout_refuses_overflowing_lists():
    """A rollout whose lists overflow (truncated lists are not symmetric, and
    the gather adjoint relies on symmetry) raises instead of returning
    gradients; the same rollout with enough slots runs."""
    from paper_2207_11328_amd.abi import SphError
    from paper_2207_11328_amd.adjoint import AdjointRollout
    sc = S.dam_break(dp=0.04, u0_sigma=0.01, seed=2)
    run = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=12, dt=1e-4,
                         rebuild_every=10, checkpoint_every=10, max_neibs=40)
    with pytest.raises(SphError, match="overflow"):
        run.forward()
    ok = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=12, dt=1e-4,
                        rebuild_every=10, checkpoint_every=10)
    ok.forward()
    t_end = ok.sim.time
    n = ok.n
    g = torch.zeros((n, 4), device=ok.sim.device)
    g[:, 0] = 1.0
    ok.backward(g, torch.zeros_like(g))
    torch_sync()
    # the reverse re-runs forward steps; the clock still reads the rollout's end
    assert ok.sim.time == t_end
    assert abs(t_end - 12 * 1e-4) < 1e-15
