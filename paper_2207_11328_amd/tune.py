"""Autotuner for the LDS brick kernels.

The brick shape (cells per workgroup of the list build, sph_forces and
sph_forces_backward) trades LDS capacity, halo re-reads and waves per
workgroup against each other, and the best choice depends on the workload:
how full the bricks are (free surfaces, walls, many small scenes) and how
dense the particles are.  `autotune` times every supported shape, and the
per-particle global-gather kernel, on the workload itself (one list build
and a few derivative evaluations each, HIP events on the launch stream) and
picks the smallest cost per step,

    t_build / rebuild_every + 2 t_forces    (two derivative calls per step).

Choices are cached in a JSON file keyed by the device and the workload's
shape (particle count, grid, spacing, periodicity, viscosity model, kernel,
formulation, diffusion, list size, per-cell alpha), so a workload is timed
once per device.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import abi
from .sim import Simulation

CACHE_ENV = "SPH_TUNE_CACHE"


def cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_2207_11328_amd", "tune.json")


def workload_key(grid, params, n, max_neibs, cell_alpha, device) -> str:
    name = torch.cuda.get_device_name(torch.device(device))
    parts = [name, "n=%d" % n, "ncell=%s" % ",".join(str(int(v)) for v in grid.ncell),
             "periodic=%d" % int(grid.periodic), "rs=%.6g" % float(params.r_search), "h=%.6g" % float(params.h),
             "visc=%d" % int(params.visc_model), "kernel=%d" % int(getattr(params, "kernel", 0)),
             "form=%d" % int(getattr(params, "formulation", 0)), "diff=%d" % int(getattr(params, "delta", 0.0) != 0.0),
             "M=%d" % int(max_neibs), "alpha_table=%d" % int(cell_alpha is not None)]
    return "|".join(parts)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs a re-tune next time


def _time(fn, reps, stream):
    """Median time [s] of fn() over reps calls, HIP events on `stream`."""
    fn()
    ev = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        ev.append((a, b))
    torch.cuda.synchronize()
    t = sorted(x.elapsed_time(y) * 1e-3 for x, y in ev)
    return t[len(t) // 2]


def autotune(grid, params, cell, pos, vel, info, cell_alpha=None, max_neibs=128, rebuild_every=10, reps=5,
             device="cuda:0", use_cache=True):
    """Returns {"brick": (bx, by, bz), "bricks": bool, "per_step_s": {...},
    "key": ..., "cached": bool}.  bricks False means the per-particle gather
    kernel (then "brick" is the default shape, used by the list build)."""
    n = int(np.asarray(cell).shape[0])
    key = workload_key(grid, params, n, max_neibs, cell_alpha, device)
    path = cache_path()
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            return {"brick": tuple(hit["brick"]), "bricks": bool(hit["bricks"]), "per_step_s": hit["per_step_s"],
                    "key": key, "cached": True}
    shapes = abi.sph_brick_shapes()
    sim = Simulation(grid, params, cell, pos, vel, info, max_neibs=max_neibs, rebuild_every=rebuild_every,
                     device=device, cell_alpha=cell_alpha, brick=shapes[0])
    stream = torch.cuda.current_stream(torch.device(device))
    costs = {}
    for shape in shapes + [None]:
        sim.set_brick(shape or shapes[0])
        t_build = _time(sim.build, max(1, reps // 2), stream)
        sim.check_status()
        t_forces = _time(lambda: sim.forces(bricks=shape is not None), reps, stream)
        label = "gather" if shape is None else "x".join(str(v) for v in shape)
        costs[label] = t_build / max(1, rebuild_every) + 2.0 * t_forces
    del sim
    torch.cuda.empty_cache()
    best = min(costs, key=costs.get)
    choice = {"brick": shapes[0] if best == "gather" else tuple(int(v) for v in best.split("x")),
              "bricks": best != "gather", "per_step_s": costs}
    if use_cache:
        table = _load(path)
        table[key] = {"brick": list(choice["brick"]), "bricks": choice["bricks"], "per_step_s": costs}
        _store(path, table)
    choice.update(key=key, cached=False)
    return choice


def tuned_simulation(grid, params, cell, pos, vel, info, cell_alpha=None, max_neibs=128, rebuild_every=10,
                     device="cuda:0", use_cache=True, **kw):
    """A Simulation with the autotuned brick shape and kernel form; returns
    (simulation, choice)."""
    choice = autotune(grid, params, cell, pos, vel, info, cell_alpha=cell_alpha, max_neibs=max_neibs,
                      rebuild_every=rebuild_every, device=device, use_cache=use_cache)
    sim = Simulation(grid, params, cell, pos, vel, info, max_neibs=max_neibs, rebuild_every=rebuild_every,
                     device=device, cell_alpha=cell_alpha, brick=choice["brick"], use_bricks=choice["bricks"], **kw)
    return sim, choice
