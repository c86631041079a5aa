#!/usr/bin/env python3
"""Benchmark of the WCSPH step on one MI355X.

Workload: the 3D dam break of ~1M fluid particles (1.6 x 0.67 x 0.6 m box,
0.4 x 0.67 x 0.3 m water column, dp = 4.3 mm, 994,635 fluid + 627,096 wall
particles), Wendland kernel h = 1.3 dp, Cole EOS, artificial viscosity
alpha = 0.01, CFL 0.3, lists rebuilt every 10 steps.  Synthetic, seeded
lattice input; nothing is read from disk.

One step = one predictor/corrector step of the hot path: neighbour search
(every 10th step), derivatives twice, device dt, integrator twice.  The
metric is particle interactions evaluated by sph_forces per second of whole
step time (interactions = listed pairs with r < 2h, counted exactly by
replaying the same deterministic trajectory with sph_count_interactions).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 (the build disables packed FP32):
# 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP per FMA x 2.4 GHz = 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# FLOP of one interaction (pair with r < 2h) of the derivative sums, FMA = 2,
# sqrt and reciprocal 1: separation 3, r^2 5, r 1, q - 2 2, m_j F 4, u_ij 3,
# u.x 5, continuity 2, Monaghan term 9, pressure sum 2, coefficient 1,
# acceleration 6 = 43; the Morris laminar term adds 9.
FLOP_PER_INTERACTION = {0: 43, 1: 52}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "forces_traffic_dam_break_1m.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2207_11328_amd", "csrc", f)
                  for f in ("forces.hip", "forces_pairs.hip", "forces_common.h", "sph_model.h", "sph_device.h")]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per sph_forces call from the committed counter summary,
    if it was taken on this workload with the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("sources_sha256") != sources_sha256():
        return None
    return float(rec["bytes_per_call"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 200 timed steps (20 graph units, about 85 ms): shorter windows read
    # 2-4% slower on the 1.62M dam break (0.432 ms per step at 30, 0.415 at
    # 200, 0.414 at 300 in one session)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="dam_break_1m", choices=["dam_break_1m", "dam_break_64k", "still_water_8k"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fwd-bwd", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-m1", action="store_true")
    ap.add_argument("--no-channel", action="store_true")
    ap.add_argument("--no-missed", action="store_true")
    ap.add_argument("--no-channel-adjoint", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--brick", default=None, metavar="BX,BY,BZ",
                    help="use this brick shape for the 1.62M dam break and the batched tanks instead of the "
                         "autotuner's choice (profiling runs: counters distort the tuner's timings)")
    ap.add_argument("--no-fuse", action="store_true",
                    help="take the corrector's derivatives and update as two calls (sph_forces, sph_integrate) "
                         "instead of one (sph_forces_corrector): every k_forces_brick dispatch is then a plain "
                         "sph_forces call (counter passes of that call)")
    ap.add_argument("--gather-probe", type=int, default=0, metavar="MIB",
                    help="only run a gather of MIB MiB in 128-byte rows taken in a random order, three times "
                         "(checks the HBM byte counters' scale on a scattered pattern) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    return ap.parse_args()


def copy_probe(mib):
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "copies": 3}), flush=True)


def hbm_probe(mib=1024, reps=5):
    """Achievable HBM bandwidth: a device-to-device copy of MIB MiB (read +
    write = 2 x MIB MiB moved), timed with HIP events, median of REPS copies
    after one warm-up copy, by the library's stream-copy kernel (the best of
    a few workgroups-per-CU settings) and by torch's copy.  The best is the
    denominator of the derivative call's achievable-HBM fraction, beside the
    8 TB/s data-sheet peak."""
    import torch
    from paper_2207_11328_amd import abi
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return 2 * n / float(np.median(ts)) / 1e9

    rates = {"torch_copy": timed(lambda: dst.copy_(src))}
    for wpc in (1, 2, 4, 8, 16):
        rates["stream_copy_%d_per_cu" % wpc] = timed(lambda: abi.sph_stream_copy(src, dst, n, wpc))
    del src, dst
    torch.cuda.empty_cache()
    best = max(rates, key=rates.get)
    return {"copy_GBps": rates[best], "best": best, "GBps": rates, "bytes_moved": 2 * n, "copies": reps,
            "kind": "device-to-device copy of %d MiB, median of %d" % (mib, reps)}


def make_scene(name):
    from workloads import scenes as S
    return S.CONFIGS[name]()


def cpu_baseline(sc, budget_s):
    """The FP64 oracle's derivative evaluation on the host cores, on the same
    step-0 state: time repeated calls until the budget is used."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    ob = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info)
    t_build = time.perf_counter() - t0
    st = O.State.lift(ob["cell"], ob["pos"], ob["vel"], ob["info"])
    calls, inter, spent = 0, 0, 0.0
    while spent < budget_s or calls == 0:
        t0 = time.perf_counter()
        _, _, _, _, ni = O.forces(sc.grid, sc.params, st, ob["lists"])
        spent += time.perf_counter() - t0
        inter += ni
        calls += 1
    return {
        "value": inter / spent,
        "unit": "interactions/s",
        "cores": O.threads(),
        "kind": "oracle",
        "sample": "%d FP64 oracle derivative call(s) on the full step-0 state (%d particles, %d interactions "
                  "per call; oracle list build %.1f s not included)" % (calls, sc.n, inter // calls, t_build),
    }


def cpu_baseline_one_core(sc):
    """The same FP64 oracle derivative call on one host thread (one call)."""
    from oracle import oracle as O
    ob = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info)
    st = O.State.lift(ob["cell"], ob["pos"], ob["vel"], ob["info"])
    t_all = O.threads()
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        _, _, _, _, ni = O.forces(sc.grid, sc.params, st, ob["lists"])
        t = time.perf_counter() - t0
    finally:
        O.set_threads(t_all)
    return {"value": ni / t, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "sample": "1 FP64 oracle derivative call on the full step-0 state (%d interactions)" % ni}


def m1_forces(sc, choice, warm=10, calls=50, late_step=500):
    """sph_forces alone: the median of `calls` HIP-event-timed calls after
    `warm` warm-up calls, on the step-0 state (lattice) and again after
    `late_step` steps (disordered), each on freshly built lists; the
    interactions of the timed state counted by sph_count_interactions."""
    import torch
    from paper_2207_11328_amd import abi
    from paper_2207_11328_amd.sim import Simulation
    sim = Simulation(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0", brick=choice["brick"],
                     use_bricks=choice["bricks"])
    stream = torch.cuda.current_stream()
    out = {}

    def measure():
        sim.build()
        for _ in range(warm):
            sim.forces()
        ev = []
        for _ in range(calls):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            sim.forces()
            b.record(stream)
            ev.append((a, b))
        torch.cuda.synchronize()
        sim.check_status()
        t = sorted(x.elapsed_time(y) for x, y in ev)[calls // 2] * 1e-3
        abi.sph_count_interactions(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, sim.count)
        inter = int(sim.count.item())
        return {"step": sim.steps_done, "forces_ms_median": t * 1e3, "interactions": inter,
                "interactions_per_s": inter / t}

    out["step_0"] = measure()
    for _ in range(late_step):
        sim.step()
    torch.cuda.synchronize()
    sim.check_status()
    out["step_%d" % late_step] = measure()
    return out


def channel(steps=10, warm=3):
    """The 16.6M-particle channel (periodic in y): whole steps (build every
    10 steps) with the autotuned brick shape; MIPPS = particles x steps/s / 1e6."""
    import torch
    from paper_2207_11328_amd import tune
    from paper_2207_11328_amd.sim import Simulation
    sc = make_scene("channel_16m")
    choice = tune.autotune(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0")
    sim = Simulation(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0", brick=choice["brick"],
                     use_bricks=choice["bricks"])
    for _ in range(warm):
        sim.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sim.check_status()
    return {"workload": "channel_16m", "particles": sc.n, "fluid": sc.n_fluid, "steps": steps,
            "ms_per_step": t / steps * 1e3, "steps_per_s": steps / t, "mipps": sc.n * steps / t / 1e6,
            "brick": list(choice["brick"]), "bricks": choice["bricks"]}


def fwd_bwd(sc, dt, K=10, reps=3, brick=None, use_bricks=True):
    """Cost of the reverse relative to the forward on one K-step block of the
    same workload (fixed dt): t_fwd = K plain steps (one rebuild); t_bwd = the
    reverse of those K steps from stored stage states (sph_integrate_backward
    and sph_forces_backward twice per step, plus the rebuild permutation).
    Also the end-to-end ratios: forward + backward of the rollout with the
    block taped (the default: lists and stage states kept from the forward),
    and with the checkpoint recomputation (no tape)."""
    import torch
    from paper_2207_11328_amd import abi
    from paper_2207_11328_amd.adjoint import AdjointRollout
    run = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=K, dt=dt, rebuild_every=K,
                         checkpoint_every=K, brick=brick, use_bricks=use_bricks, tape_bytes=0)
    taped = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=K, dt=dt, rebuild_every=K,
                           checkpoint_every=K, brick=brick, use_bricks=use_bricks)
    n = run.n
    g = torch.Generator(device=run.sim.device).manual_seed(0)
    seed_p = torch.randn((n, 4), device=run.sim.device, generator=g)
    seed_v = torch.randn((n, 4), device=run.sim.device, generator=g)
    t_f, t_b, t_e2e, t_tape = [], [], [], []
    for _ in range(reps):
        run.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.forward()
        torch.cuda.synchronize()
        t_f.append(time.perf_counter() - t0)
        # stage states of the block (the recomputation the checkpointing does)
        run.reset()
        run.sim.build(perm_out=run.perm)
        stored = []
        for _k in range(K):
            run._advance(stored)
        run.gpos[:n] = seed_p
        run.gvel[:n] = seed_v
        run.grad_params.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.reverse_block(stored)
        abi.sph_unpermute(n, run.perm, run.gpos, run.tmp_p)
        abi.sph_unpermute(n, run.perm, run.gvel, run.tmp_v)
        torch.cuda.synchronize()
        t_b.append(time.perf_counter() - t0)
        del stored
        run.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.forward()
        run.backward(seed_p, seed_v)
        torch.cuda.synchronize()
        t_e2e.append(time.perf_counter() - t0)
        taped.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        taped.forward()
        taped.backward(seed_p, seed_v)
        torch.cuda.synchronize()
        t_tape.append(time.perf_counter() - t0)
    tf, tb, te, tt = min(t_f), min(t_b), min(t_e2e), min(t_tape)
    out = {"workload": sc.name, "particles": sc.n, "block_steps": K, "fwd_ms": tf * 1e3, "bwd_ms": tb * 1e3,
           "fwd_bwd_ratio": (tf + tb) / tf, "fwd_bwd_ratio_end_to_end": tt / tf,
           "fwd_bwd_ratio_with_recompute": te / tf, "taped_blocks": taped.n_taped,
           "tape_bytes_per_block": taped.tape_block_bytes(), "fwd_bwd_steps_per_s": K / (tf + tb)}
    del run, taped
    torch.cuda.empty_cache()
    return out


def fixed_choice(brick):
    """The tuner's result format for a given brick shape (LDS brick kernels)."""
    return {"brick": tuple(int(v) for v in brick), "bricks": True, "per_step_s": {}, "cached": False,
            "fixed": True}


def batched(units=50, warm_units=1, brick=None):
    """128 independent tanks (fluid counts log-uniform in [2k, 60k], column
    aspect 0.3-2, alpha 0.005-0.05) stacked in one grid, advanced by replays
    of a HIP graph holding one rebuild unit (10 steps, each tank with its
    own adaptive dt)."""
    import torch
    from paper_2207_11328_amd import tune
    from workloads import scenes as S
    tanks = S.batched_tanks()
    st, alpha, _, _ = S.stack_scenes(tanks)
    if brick is None:
        sim, choice = tune.tuned_simulation(st.grid, st.params, st.cell, st.pos, st.vel, st.info, cell_alpha=alpha,
                                            device="cuda:0", cell_scene=S.scene_cells(st))
    else:
        from paper_2207_11328_amd.sim import Simulation
        choice = fixed_choice(brick)
        sim = Simulation(st.grid, st.params, st.cell, st.pos, st.vel, st.info, cell_alpha=alpha, device="cuda:0",
                         cell_scene=S.scene_cells(st), brick=choice["brick"])
    sim.capture_unit()
    sim.replay_units(warm_units)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.replay_units(units)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sim.check_status()
    steps = units * sim.rebuild_every
    clocks = sim.time  # each tank's own clock: its own adaptive dt
    return {"scenes": len(tanks), "particles": st.n, "fluid": st.n_fluid, "steps": steps,
            "dt": "per scene", "simulated_time_s": {"min": float(clocks.min()), "max": float(clocks.max())},
            "ms_per_step": t / steps * 1e3, "particle_steps_per_s": st.n * steps / t, "mipps": st.n * steps / t / 1e6,
            "fluid_particle_steps_per_s": st.n_fluid * steps / t, "graph_units": units,
            "tuned": {"brick": list(choice["brick"]), "bricks": choice["bricks"],
                      "per_step_ms": {k: v * 1e3 for k, v in choice["per_step_s"].items()}}}


# list slots for a search-radius skin s (lattice neighbours within r_s =
# 2.6 dp (1 + s) plus margin for the walls)
SKIN_SLOTS = {0.1: 128, 0.15: 160, 0.2: 192, 0.25: 224, 0.3: 256, 0.35: 288, 0.4: 320}


def missed_pairs(steps=1000, skins=(0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4)):
    """Pairs within 2h that the reused lists missed, at every rebuild of a
    1000-step run of the 1.62M dam break (lists rebuilt every 10 steps,
    sph_count_missed_pairs before and after each rebuild).  If the default
    skin (search radius 2h (1 + 0.1)) misses pairs, larger skins are run
    until one misses none."""
    import torch
    from paper_2207_11328_amd.sim import Simulation
    from workloads import scenes as S
    out = {"steps": steps, "rebuild_every": 10, "skins": {}}
    for skin in skins:
        sc = S.dam_break_1m(skin=skin)
        sim = Simulation(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0",
                         max_neibs=SKIN_SLOTS[skin])
        sim.track_missed = True
        per = []
        t0 = time.perf_counter()
        for k in range(steps):
            sim.step()
            if k > 0 and k % sim.rebuild_every == 0:   # a rebuild with counting just ran
                per.append(sim.missed_host()["missed"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = sim.check_status()
        rec = {"search_radius_over_2h": 1.0 + skin, "max_neibs": sim.max_neibs, "max_listed": st["max_neibs"],
               "rebuilds_counted": len(per), "missed_total": int(sum(per)), "missed_max": int(max(per)),
               "rebuilds_with_misses": int(sum(1 for v in per if v > 0)), "missed_per_rebuild": per,
               "wall_s_with_counting": wall}
        out["skins"]["%.2f" % skin] = rec
        del sim
        torch.cuda.empty_cache()
        if rec["missed_total"] == 0:
            out["smallest_skin_without_misses"] = skin
            break
    return out


def channel_adjoint(fwd_steps=100, adj_steps=50, K=10):
    """The 16.6M channel at its stated workload: 100 forward steps (timed),
    then a 50-step adjoint with recomputation (checkpoint every 10 steps,
    fixed dt = the step-0 dt): forward and reverse times and the peak device
    memory of the adjoint run."""
    import torch
    from paper_2207_11328_amd import tune
    from paper_2207_11328_amd.adjoint import AdjointRollout
    from paper_2207_11328_amd.sim import Simulation
    sc = make_scene("channel_16m")
    choice = tune.autotune(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0")
    sim = Simulation(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0", brick=choice["brick"],
                     use_bricks=choice["bricks"])
    sim.build()
    sim.forces()
    sim.step_dt()
    dt0 = float(sim.d_dt.item())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(fwd_steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    sim.check_status()
    del sim
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    run = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=adj_steps, dt=dt0,
                         rebuild_every=K, checkpoint_every=K, brick=choice["brick"], use_bricks=choice["bricks"])
    n = run.n
    g = torch.Generator(device=run.sim.device).manual_seed(0)
    seed_p = torch.randn((n, 4), device=run.sim.device, generator=g)
    seed_v = torch.randn((n, 4), device=run.sim.device, generator=g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.forward()
    torch.cuda.synchronize()
    t_af = time.perf_counter() - t0
    t0 = time.perf_counter()
    gp, gv, gpar = run.backward(seed_p, seed_v)
    torch.cuda.synchronize()
    t_ab = time.perf_counter() - t0
    finite = bool(torch.isfinite(gp).all() and torch.isfinite(gv).all() and torch.isfinite(gpar).all())
    peak = torch.cuda.max_memory_allocated()
    del run
    torch.cuda.empty_cache()
    return {"workload": "channel_16m", "particles": sc.n, "fluid": sc.n_fluid, "forward_steps": fwd_steps,
            "forward_ms_per_step": t_fwd / fwd_steps * 1e3, "forward_mipps": sc.n * fwd_steps / t_fwd / 1e6,
            "adjoint_steps": adj_steps, "checkpoint_every": K, "dt": dt0,
            "adjoint_forward_s": t_af, "adjoint_backward_s": t_ab,
            "backward_over_forward": t_ab / t_af, "gradients_finite": finite,
            "peak_device_memory_gb": peak / 1e9, "brick": list(choice["brick"])}


def adjoint_64k_200(steps=200, C=20, K=10):
    """The differentiable dam break of ~64k fluid particles at its stated
    length: 200 fixed-dt steps (the step-0 dt), checkpoint every 20 steps,
    rebuild every 10; the forward rollout and the reverse, each timed, with
    the blocks taped (the default, device memory permitting) and with the
    recomputation between checkpoints."""
    import torch
    from paper_2207_11328_amd import tune
    from paper_2207_11328_amd.adjoint import AdjointRollout
    from paper_2207_11328_amd.sim import Simulation
    sc = make_scene("dam_break_64k")
    c = tune.autotune(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0")
    s = Simulation(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0", brick=c["brick"],
                   use_bricks=c["bricks"])
    s.build()
    s.forces()
    s.step_dt()
    dt = float(s.d_dt.item())
    del s
    out = {"workload": "dam_break_64k", "particles": sc.n, "steps": steps, "checkpoint_every": C}
    for mode, budget in (("taped", None), ("recompute", 0)):
        run = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=steps, dt=dt,
                             rebuild_every=K, checkpoint_every=C, brick=c["brick"], use_bricks=c["bricks"],
                             tape_bytes=budget)
        n = run.n
        g = torch.Generator(device=run.sim.device).manual_seed(0)
        seed_p = torch.randn((n, 4), device=run.sim.device, generator=g)
        seed_v = torch.randn((n, 4), device=run.sim.device, generator=g)
        best = None
        for _ in range(2):
            run.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run.forward()
            torch.cuda.synchronize()
            t_f = time.perf_counter() - t0
            t0 = time.perf_counter()
            run.backward(seed_p, seed_v)
            torch.cuda.synchronize()
            t_b = time.perf_counter() - t0
            if best is None or t_f + t_b < best[0] + best[1]:
                best = (t_f, t_b)
        t_f, t_b = best
        out[mode] = {"taped_blocks": run.n_taped, "forward_s": t_f, "backward_s": t_b,
                     "fwd_bwd_ratio": (t_f + t_b) / t_f, "fwd_bwd_steps_per_s": steps / (t_f + t_b)}
        del run
        torch.cuda.empty_cache()
    return out


def still_water_vs_oracle(steps=100):
    """The still-water tank (8,000 fluid + 7,548 wall particles, dp = 0.02 m)
    rolled out 100 steps (adaptive dt, rebuild every 10) by the GPU library in
    float32 and by the FP64 oracle on the host (timed): the error of each field
    of the GPU's final state against the oracle's, by particle id."""
    import torch
    from oracle import oracle as O
    from paper_2207_11328_amd.sim import Simulation
    from workloads import scenes as S
    sc = S.still_water(0.02)
    sim = Simulation(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    sim.check_status()
    g = sim.state_host()
    st0 = O.State.lift(sc.cell, sc.pos, sc.vel, sc.info)
    t0 = time.perf_counter()
    ref, t_ref = O.rollout(sc.grid, sc.params, st0, steps, rebuild_every=10)
    t_orc = time.perf_counter() - t0
    mask = np.uint32((1 << 30) - 1)
    gst = O.State.lift(g["cell"], g["pos"], g["vel"], g["info"])
    og = np.argsort(g["info"] & mask)
    oo = np.argsort(ref.info & mask)
    xg, xo = O.positions(sc.grid, gst)[og], O.positions(sc.grid, ref)[oo]
    ug, uo = gst.vel[og], ref.vel[oo]
    rg, ro = gst.rho[og], ref.rho[oo]
    rho0 = O.f32(sc.params.rho0)
    return {"workload": "still_water_8k", "particles": sc.n, "steps": steps,
            "gpu_s": t_gpu, "oracle_s": t_orc, "oracle_cores": O.threads(),
            "time_gpu": sim.time, "time_oracle": t_ref,
            "error": {"position_max_over_dp": float(np.abs(xg - xo).max() / sc.params.dp),
                      "velocity_max_over_umax": float(np.abs(ug - uo).max() / np.abs(uo).max()),
                      "velocity_rms_over_urms": float(np.sqrt(((ug - uo) ** 2).mean() / (uo ** 2).mean())),
                      "density_max_over_rho0": float(np.abs(rg - ro).max() / rho0),
                      "time_rel": abs(sim.time - t_ref) / t_ref}}


# models timed by the variants leg: (label, kernel, visc_model, formulation, delta)
VARIANTS = [
    ("wendland", 0, 0, 0, 0.0), ("cubic_spline", 1, 0, 0, 0.0), ("quadratic", 2, 0, 0, 0.0),
    ("gaussian", 3, 0, 0, 0.0), ("wendland_landrini", 0, 0, 1, 0.0), ("wendland_morris", 0, 1, 0, 0.0),
    ("wendland_monaghan_k", 0, 2, 0, 0.0), ("wendland_diffusion", 0, 0, 0, 0.1),
    ("gaussian_landrini_monaghan_k_diffusion", 3, 2, 1, 0.1),
]


def variants(sim, sc, inter_per_call, reps=20):
    """sph_forces and sph_forces_backward of every model in VARIANTS on the
    same state and lists (the timed run's last), HIP events on the launch
    stream; laminar models at nu = 1e-6 m^2/s."""
    import dataclasses
    import torch
    from paper_2207_11328_amd import abi
    dev = sim.device
    cap = sim.capacity
    gforce = torch.randn((cap, 4), device=dev)
    gpos = torch.zeros((cap, 4), device=dev)
    gvel = torch.zeros((cap, 4), device=dev)
    gpar = torch.zeros(3, dtype=torch.float64, device=dev)
    ws = torch.zeros(abi.sph_forces_backward_workspace_bytes(cap, sim.n_cells), dtype=torch.uint8, device=dev)
    cs, ce, nb = sim.brick_args()
    stream = torch.cuda.current_stream()
    out = {}
    for label, kernel, visc, form, delta in VARIANTS:
        p = abi.params_struct(dataclasses.replace(sc.params, kernel=kernel, visc_model=visc, formulation=form,
                                                  delta=delta, nu=1e-6 if visc else sc.params.nu))

        def fwd():
            abi.sph_forces(sim.g, p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, sim.forces_n,
                           sim.ws_forces, None, cs, ce, nb)

        def bwd():
            abi.sph_forces_backward(sim.g, p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, gforce, gpos,
                                    gvel, gpar, False, ws, None, cs, ce, nb)

        row = {}
        for name, fn in (("forces", fwd), ("backward", bwd)):
            fn()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            row[name + "_ms"] = a.elapsed_time(b) / reps
        row["forces_interactions_per_s"] = inter_per_call / (row["forces_ms"] * 1e-3)
        out[label] = row
    return out


def gather_probe(mib):
    import torch
    rows = (mib << 20) // 128
    src = torch.ones((rows, 32), dtype=torch.float32, device="cuda:0")
    g = torch.Generator(device="cpu").manual_seed(7)
    perm = torch.randperm(rows, generator=g).to("cuda:0")
    torch.cuda.synchronize()
    for _ in range(3):
        dst = src.index_select(0, perm)
    torch.cuda.synchronize()
    # every 128-byte row is read once and written once; the index is 8 bytes a row
    print(json.dumps({"gather_probe_rows": rows, "row_bytes": 128, "index_bytes": rows * 8,
                      "gathers": 3, "checksum": float(dst[:4].sum())}), flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gather_probe:
        gather_probe(args.gather_probe)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the step shards by slabs of "
              "cells with halo exchange, which is not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2207_11328_amd import tune
    from paper_2207_11328_amd.sim import Simulation

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    sc = make_scene(args.workload)
    K, W = args.steps, args.warmup
    brick = tuple(int(v) for v in args.brick.split(",")) if args.brick else None
    choice = (fixed_choice(brick) if brick else
              tune.autotune(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0"))

    def new_sim():
        s = Simulation(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, device="cuda:0",
                       brick=choice["brick"], use_bricks=choice["bricks"])
        if args.no_fuse:
            s.fuse_corrector = False
        return s

    sim = new_sim()
    for _ in range(W):
        sim.step()
    # the timed steps start on a rebuild step (their first step rebuilds, as
    # every 10th does), so that they can be replayed as 10-step graph units
    align = -W % sim.rebuild_every
    for _ in range(align):
        sim.step()
    torch.cuda.synchronize()
    sim.check_status()

    # The timed steps: replays of a HIP graph holding one rebuild unit (the
    # neighbour search and 10 steps, no host launch per kernel) when K is a
    # whole number of units, else launched one by one.
    use_graph = K % sim.rebuild_every == 0
    warm_units = 0
    if use_graph:
        sim.capture_unit()
        # one untimed replay: the first launch of a new graph also uploads it
        sim.replay_units(1)
        warm_units = 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if use_graph:
        sim.replay_units(K // sim.rebuild_every)
    else:
        sim.run(K)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    sim.check_status()

    # The same trajectory again, launched one by one: HIP events around each
    # sph_forces call (the derivative call's own time, for the roofline) and
    # the interactions each call evaluates; its final state must equal the
    # timed run's bit for bit.
    from paper_2207_11328_amd import abi
    rep = new_sim()
    for _ in range(W + align + warm_units * rep.rebuild_every):
        rep.step()
    ev = []  # (start, end) around each sph_forces launch
    inter_dev = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    listed_dev = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    for _ in range(K):
        if rep.steps_done % rep.rebuild_every == 0:
            rep.build()
        for star in (False, True):
            if star:
                rep.integrate(0)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            rep.forces(star)
            b.record()
            ev.append((a, b))
            parts_n = rep.parts_star if star else rep.parts
            abi.sph_count_interactions(rep.g, rep.p, parts_n, rep.neibs, rep.neib_count, rep.max_neibs, rep.count)
            inter_dev += rep.count
            if not star and rep.dt_fixed is None:
                rep.step_dt()
        cnt = rep.neib_count[: rep.n].long()
        listed_dev += 2 * ((cnt & 0xFFFF) + (cnt >> 16)).sum()
        rep.integrate(1)
        rep.steps_done += 1
    torch.cuda.synchronize()
    t_forces_events = [a.elapsed_time(b) * 1e-3 for a, b in ev]
    inter = int(inter_dev.item())
    listed = int(listed_dev.item())
    same = torch.equal(rep.pos, sim.pos) and torch.equal(rep.vel, sim.vel)
    del rep
    torch.cuda.empty_cache()

    n = sc.n
    calls = len(t_forces_events)
    t_forces = float(np.sum(t_forces_events))
    t_forces_avg = t_forces / calls
    # algorithmic bytes of one sph_forces launch: pos, vel (16 B each), count
    # (4 B) and the float4 output per particle, and the listed entries (2 B
    # each in the brick-local lists the LDS kernel reads, 4 B in the global
    # lists of the gather kernel)
    entry_bytes = 2 if choice["bricks"] else 4
    bytes_per_launch = n * (16 + 16 + 4 + 16) + entry_bytes * (listed / calls)
    achieved_gbs = bytes_per_launch / t_forces_avg / 1e9
    flop_per_launch = FLOP_PER_INTERACTION[int(sc.params.visc_model)] * inter / calls
    achieved_tflops = flop_per_launch / t_forces_avg / 1e12
    traffic = measured_traffic(args.workload) if choice["bricks"] else None
    probe = hbm_probe()
    ms_per_step = t_total / K * 1e3
    value = inter / t_total
    out = {
        "metric": "particle-interactions/s in sph_forces; fwd+bwd steps/s vs plain fwd at 1e-5 rel err",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "dam_break_%s" % ("1m" if args.workload == "dam_break_1m" else args.workload),
            "particles": n, "fluid": sc.n_fluid, "boundary": sc.n_boundary,
            "dp": sc.params.dp, "h_over_dp": 1.3, "max_neibs": sim.max_neibs, "rebuild_every": sim.rebuild_every,
            "brick": list(choice["brick"]), "kernel": "lds_bricks" if choice["bricks"] else "gather",
        },
        "tuning": {"cached": choice["cached"], "fixed_by_flag": bool(choice.get("fixed")),
                   "per_step_ms": {k: v * 1e3 for k, v in choice["per_step_s"].items()}},
        "value_definition": "interactions evaluated by sph_forces (pairs with r < 2h, two calls per step) per "
                            "second of WHOLE-STEP time (list build every 10th step, dt, integrator included)",
        "forces_interactions_per_s": inter / t_forces,
        "forces_interactions_per_s_definition": "the same interactions per second of sph_forces time only "
                                                "(HIP events around each call in the timed steps)",
        "forces_ms_avg": t_forces_avg * 1e3,
        "interactions_per_forces_call": inter / calls,
        "listed_per_forces_call": listed / calls,
        "steps_per_s": K / t_total,
        "mipps": n * K / t_total / 1e6,
        "replay_bitwise_identical": bool(same),
        "timing": ("HIP graph replays of %d-step units (neighbour search + steps), after %d untimed warm-up "
                   "steps and one untimed replay of the new graph" % (sim.rebuild_every, W + align)
                   if use_graph else "steps launched one by one"),
        # the derivative call: its algorithmic intensity (on the dam break
        # about 13 FLOP per algorithmic byte) is above the FP32/HBM ridge
        # (9.8), so the FP32 vector roof bounds it; HBM figures beside it
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP32_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": ("sph_forces = k_zero_one (brick counter) + k_forces_brick" if choice["bricks"]
                       else "sph_forces = k_eos + k_forces"),
            "flop_per_launch": flop_per_launch,
            "launch_ms": t_forces_avg * 1e3,
            "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved_gbs / HBM_PEAK_GBS, "bytes_per_launch": bytes_per_launch,
                    "traffic_frac": None if traffic is None else traffic / t_forces_avg / 1e9 / HBM_PEAK_GBS,
                    # the achievable peak measured on this GPU (stream copy)
                    "achievable": probe["copy_GBps"],
                    "frac_of_achievable": achieved_gbs / probe["copy_GBps"],
                    "traffic_frac_of_achievable": (None if traffic is None else
                                                   traffic / t_forces_avg / 1e9 / probe["copy_GBps"]),
                    "probe": probe},
        },
    }
    if not args.no_variants:
        out["variants"] = variants(sim, sc, inter / calls)
    if not args.no_m1:
        out["m1"] = m1_forces(sc, choice)
    if not args.no_batched:
        out["batched"] = batched(brick=brick)
    if not args.no_fwd_bwd:
        dt_now = float(sim.d_dt.item())
        out["adjoint"] = fwd_bwd(sc, dt_now, brick=choice["brick"], use_bricks=choice["bricks"])
        # the differentiable dam break of ~64k fluid particles (the configuration
        # the fwd+bwd cost ratio is quoted on), at its own step-0 dt
        sc64 = make_scene("dam_break_64k")
        c64 = tune.autotune(sc64.grid, sc64.params, sc64.cell, sc64.pos, sc64.vel, sc64.info, device="cuda:0")
        s64 = Simulation(sc64.grid, sc64.params, sc64.cell, sc64.pos, sc64.vel, sc64.info, device="cuda:0",
                         brick=c64["brick"], use_bricks=c64["bricks"])
        s64.build()
        s64.forces()
        s64.step_dt()
        dt64 = float(s64.d_dt.item())
        del s64
        out["adjoint_64k"] = fwd_bwd(sc64, dt64, brick=c64["brick"], use_bricks=c64["bricks"])
        out["adjoint_64k_200_steps"] = adjoint_64k_200()
    del sim
    torch.cuda.empty_cache()
    if not args.no_missed:
        out["missed_pairs"] = missed_pairs()
    if not args.no_channel:
        out["channel"] = channel()
    if not args.no_channel_adjoint:
        out["channel_adjoint"] = channel_adjoint()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
        out["cpu_baseline_1core"] = cpu_baseline_one_core(sc)
        # the oracle's 100-step still-water rollout, timed, and the GPU's
        # per-field error against it
        out["cpu_baseline_still_water"] = still_water_vs_oracle()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
