"""sph_forces_noalloc (the allocation-free variant of sph_forces, for
callers that cannot allocate device memory) against sph_forces through the
C ABI: bit-identical derivatives, in both kernel forms, on two calls in a row
where the second has a smaller input, and the refusal of a problem larger
than its fixed scratch before any device call."""
import ctypes as C

import numpy as np
import pytest

from workloads import scenes as S

from parity import log, make_sim, torch_sync

torch = pytest.importorskip("torch")


def test_noalloc_rejects_a_problem_beyond_its_scratch():
    """Host-side check (no device call is made): a capacity whose workspace
    exceeds the fixed scratch is SPH_ERR_SCRATCH."""
    from paper_2207_11328_amd import abi
    g = abi.SphGrid()
    for d in range(3):
        g.cell_size[d] = 0.06
        g.ncell[d] = 100
    p = abi.SphParams()
    p.h, p.r_search, p.rho0, p.gamma, p.c0 = 0.026, 0.06, 1000.0, 7.0, 20.0
    big = abi.SphParticles(0, 9_000_000, None, None, None, None)
    assert abi.sph_forces_workspace_bytes(9_000_000, 10 ** 6) > abi.NOALLOC_SCRATCH_BYTES
    code = abi.lib.sph_forces_noalloc(C.byref(g), C.byref(p), C.byref(big), None, None, 128, None, None, None,
                                      None, None)
    assert code == abi.SPH_ERR_SCRATCH
    assert b"SPH_ERR_SCRATCH" in abi.lib.sph_status_string(code)
    assert abi.lib.sph_forces_noalloc(None, None, None, None, None, 128, None, None, None, None,
                                      None) == abi.SPH_ERR_ARG


@pytest.mark.gpu
def test_noalloc_matches_sph_forces_on_two_calls():
    from paper_2207_11328_amd import abi
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # the second scene is smaller (fewer particles and cells) than the first
    scenes = [S.dam_break(dp=0.016, u0_sigma=0.05, seed=5), S.still_water(dp=0.04, side=0.4)]
    assert scenes[1].n < scenes[0].n and scenes[1].grid.n_cells < scenes[0].grid.n_cells
    for sc in scenes:
        sim = make_sim(sc)
        sim.build()
        sim.check_status()
        need = abi.sph_forces_workspace_bytes(sim.capacity, sim.n_cells)
        assert need <= abi.NOALLOC_SCRATCH_BYTES
        for bricks in (True, False):
            log("noalloc case %s n=%d bricks=%s workspace %d B" % (sc.name, sc.n, bricks, need))
            cs, ce, nb = sim.brick_args(bricks)
            ref = torch.full_like(sim.forces_n, float("nan"))
            got = torch.full_like(sim.forces_n, float("nan"))
            abi.sph_forces(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, ref, sim.ws_forces,
                           None, cs, ce, nb)
            abi.sph_forces_noalloc(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, got, None,
                                   cs, ce, nb)
            torch_sync()
            n = sc.n
            assert torch.isfinite(ref[:n]).all()
            assert torch.equal(got[:n], ref[:n]), float((got[:n] - ref[:n]).abs().max())
        del sim
