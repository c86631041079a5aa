"""Write dam_break_64k_gradient.json: the FP64 oracle's gradient of the
differentiable dam break and its finite-difference check.

Workload: the dam break of 64,232 fluid particles (1.6 x 0.67 x 0.6 m box,
0.4 x 0.67 x 0.3 m column, dp = 10.7 mm, initial velocities N(0, 0.01 m/s)
seeded 2), 200 predictor/corrector steps at the time step of the initial
state held fixed, lists rebuilt every 10 steps.  Loss: the mean x of the
front, the ceil(0.01 N_f) fluid particles with the largest x at the end of
the unperturbed run (a frozen set of ids).  Gradients with respect to the
artificial-viscosity coefficient alpha, the sound speed c0 and the initial
velocities, by the oracle's reverse pass, and central finite differences
of FP64 rollouts at a relative step of 1e-4 for alpha and c0 and along a
seeded direction v = N(0, 1) / sqrt(3 N_f) (seed 3) for the velocities.

Calls only oracle/ and workloads/ (the values are the oracle's, never the
GPU library's).  Takes several minutes on a few cores:

    python tests/golden/make_dam_break_64k_gradient.py
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workloads import scenes as S  # noqa: E402

OUT = os.path.join(HERE, "dam_break_64k_gradient.json")
STEPS = 200
REBUILD = 10
EPS = 1e-4
SAMPLE = 2048


class Exact:
    """Parameters handed to the oracle unrounded (finite differences)."""

    exact_values = True

    def __init__(self, p, **kw):
        self._p = p
        self._kw = kw

    def __getattr__(self, k):
        if k in self._kw:
            return self._kw[k]
        v = getattr(self._p, k)
        if isinstance(v, float):
            return O.f32(v)
        if isinstance(v, tuple):
            return tuple(O.f32(t) for t in v)
        return v


def main():
    t0 = time.time()
    sc = S.dam_break_64k()
    p = sc.params
    st0 = O.State.lift(sc.cell, sc.pos, sc.vel, sc.info)
    # the time step of the initial state, held fixed over the run
    b = O.build_f32(sc.grid, p, sc.cell, sc.pos, sc.vel, sc.info)
    st_b = O.State.lift(b["cell"], b["pos"], b["vel"], b["info"])
    acc, _, _, _, _ = O.forces(sc.grid, p, st_b, b["lists"])
    dt = O.dt(p, st_b, acc)
    print("n=%d fluid=%d dt=%.17g (%.0f s)" % (sc.n, sc.n_fluid, dt, time.time() - t0), flush=True)

    def final(params, st):
        out, _ = O.rollout(sc.grid, params, st.copy(), STEPS, rebuild_every=REBUILD, dt_fixed=dt)
        return out

    base = final(p, st0)
    x = O.positions(sc.grid, base)
    fl = base.is_fluid
    ids = (base.info & np.uint32((1 << 30) - 1)).astype(np.int64)
    k = int(math.ceil(0.01 * fl.sum()))
    front = np.sort(ids[fl][np.argsort(-x[fl, 0], kind="stable")[:k]])
    print("front of %d particles (%.0f s)" % (k, time.time() - t0), flush=True)

    def loss(st):
        xs = O.positions(sc.grid, st)
        pid = (st.info & np.uint32((1 << 30) - 1)).astype(np.int64)
        return float(xs[np.isin(pid, front), 0].mean())

    L, adj, gp, _ = O.rollout_adjoint(sc.grid, p, st0, STEPS, dt, O.front_loss(sc.grid, front),
                                      rebuild_every=REBUILD)
    print("reverse: L=%.15g dL/dalpha=%.9e dL/dc0=%.9e (%.0f s)" % (L, gp[0], gp[1], time.time() - t0), flush=True)
    ids0 = (st0.info & np.uint32((1 << 30) - 1)).astype(np.int64)
    fluid0 = st0.is_fluid
    rng = np.random.default_rng(3)
    v = np.zeros((sc.n, 3))
    v[fluid0] = rng.normal(size=(int(fluid0.sum()), 3)) / math.sqrt(3 * int(fluid0.sum()))
    g_u0 = np.where(fluid0[:, None], adj.gu, 0.0)
    dir_rev = float((g_u0 * v).sum())

    fd = {}
    for name in ("alpha", "c0"):
        th = O.f32(getattr(p, name))
        e = EPS * th
        lp = loss(final(Exact(p, **{name: th + e}), st0))
        lm = loss(final(Exact(p, **{name: th - e}), st0))
        fd[name] = (lp - lm) / (2 * e)
        print("fd %s %.9e (%.0f s)" % (name, fd[name], time.time() - t0), flush=True)
    sp, sm = st0.copy(), st0.copy()
    sp.vel = st0.vel + EPS * v
    sm.vel = st0.vel - EPS * v
    fd["u0_dir"] = (loss(final(p, sp)) - loss(final(p, sm))) / (2 * EPS)
    print("fd u0 along v %.9e, reverse %.9e (%.0f s)" % (fd["u0_dir"], dir_rev, time.time() - t0), flush=True)

    fl_idx = np.nonzero(fluid0)[0]
    pick = np.sort(np.random.default_rng(4).choice(fl_idx, size=SAMPLE, replace=False))
    rec = {
        "workload": "dam_break_64k", "particles": sc.n, "fluid": sc.n_fluid, "steps": STEPS,
        "rebuild_every": REBUILD, "dt": dt, "loss": L, "front_ids": front.tolist(),
        "grad_alpha": float(gp[0]), "grad_c0": float(gp[1]),
        "grad_u0_norm": float(np.linalg.norm(g_u0)), "grad_u0_dot_v": dir_rev,
        "fd_eps": EPS, "fd_alpha": fd["alpha"], "fd_c0": fd["c0"], "fd_u0_dot_v": fd["u0_dir"],
        "direction": "v = N(0, 1) / sqrt(3 N_f) on fluid particles in initial storage order, "
                     "numpy default_rng(3).normal",
        "sample_ids": ids0[pick].tolist(), "sample_grad_u0": g_u0[pick].tolist(),
        "seconds": time.time() - t0, "threads": O.threads(),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote %s" % OUT, flush=True)


if __name__ == "__main__":
    main()
