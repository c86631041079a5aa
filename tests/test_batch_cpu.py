"""Host side of batching: the per-cell scene table of stacked scenes."""
import numpy as np

from workloads import scenes as S


def test_scene_table_assigns_every_particle_its_scene():
    tanks = S.batched_tanks(n_scenes=5, seed=3, n_min=300, n_max=1200)
    stacked, alpha, subs, ranges = S.stack_scenes(tanks)
    table = S.scene_cells(stacked)
    assert table.shape == (stacked.grid.n_cells,) and table.dtype == np.int32
    scene_of = table[stacked.cell - stacked.grid.cell_base]
    for k, (first, count) in enumerate(ranges):
        assert np.all(scene_of[first:first + count] == k), k
    # every cell has a scene, in stacking order along z
    nx, ny, nz = (int(v) for v in stacked.grid.ncell)
    layers = table.reshape(nz, ny * nx)
    assert np.all(layers == layers[:, :1])
    assert np.all(np.diff(layers[:, 0]) >= 0) and layers[0, 0] == 0 and layers[-1, 0] == len(tanks) - 1
    # the scene's own alpha region lies inside its scene's cells
    for k, t in enumerate(tanks):
        own = alpha == np.float32(t.params.alpha)
        assert np.all(table[own] == k) or np.any(np.float32(tanks[j].params.alpha) == np.float32(t.params.alpha)
                                                 for j in range(len(tanks)) if j != k)
