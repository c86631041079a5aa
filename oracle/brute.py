"""O(N^2) brute-force neighbour sets in numpy (N up to a few thousand).

TEST INFRASTRUCTURE ONLY.  Independent of the cell scan in sph_oracle.c: it
tests every pair of particles, taking the cell difference of the pair as the
nearest periodic image, and evaluates the separation from the cell-relative
float32 encoding with the same operation order as the method's predicate
(section "Optimizing the neighbors search": the search is restricted to the
Moore neighbourhood only because the cell side is at least the radius).
"""
from __future__ import annotations

import numpy as np

TYPE_SHIFT = 30


def _coords(grid, cell):
    nx, ny = int(grid.ncell[0]), int(grid.ncell[1])
    lc = cell.astype(np.int64) - int(grid.cell_base)
    return np.stack([lc % nx, (lc // nx) % ny, lc // (nx * ny)], axis=1)


def pair_r2(grid, cell, pos, fp64=False):
    """[N,N] squared separations x_i - x_j of a float32 encoded state (with
    fp64, of float32 or double offsets, in double)."""
    c = _coords(grid, cell)
    k = c[:, None, :] - c[None, :, :]
    for d in range(3):
        if (grid.periodic >> d) & 1:
            n = int(grid.ncell[d])
            k[:, :, d] = (k[:, :, d] + n // 2) % n - n // 2
    cs = np.asarray(grid.cell_size, dtype=np.float32)
    if fp64:
        # double offsets are taken as given (float32 ones lift exactly)
        o64 = np.asarray(pos)[:, :3].astype(np.float64)
        x = k.astype(np.float64) * cs.astype(np.float64)[None, None, :] + (o64[:, None, :] - o64[None, :, :])
        return (x * x).sum(axis=2)
    o = np.asarray(pos, dtype=np.float32)[:, :3]
    t1 = (o[:, None, :] - o[None, :, :]).astype(np.float32)
    t2 = (k.astype(np.float32) * cs[None, None, :]).astype(np.float32)
    x = (t2 + t1).astype(np.float32)
    xx = (x[:, :, 0] * x[:, :, 0]).astype(np.float32)
    yy = (x[:, :, 1] * x[:, :, 1]).astype(np.float32)
    zz = (x[:, :, 2] * x[:, :, 2]).astype(np.float32)
    return ((xx + yy).astype(np.float32) + zz).astype(np.float32)


def neighbor_sets(grid, r_search, cell, pos, info, fp64=False):
    """List of (fluid ids set, boundary ids set) per particle index, as
    sorted numpy arrays of particle indices."""
    r2 = pair_r2(grid, cell, pos, fp64)
    rs = np.float32(r_search)
    lim = np.float64(rs) ** 2 if fp64 else np.float32(rs * rs)
    n = cell.shape[0]
    typ = (np.asarray(info, dtype=np.uint32) >> TYPE_SHIFT).astype(np.int64)
    valid = np.asarray(cell) >= 0
    adj = (r2 < lim) & valid[:, None] & valid[None, :]
    np.fill_diagonal(adj, False)
    bb = (typ[:, None] == 1) & (typ[None, :] == 1)
    adj &= ~bb
    out = []
    for i in range(n):
        js = np.nonzero(adj[i])[0]
        out.append((js[typ[js] == 0], js[typ[js] == 1]))
    return out
