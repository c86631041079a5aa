"""Step driver over the C ABI: device buffers (torch), rebuild cadence, the
predictor/corrector step with the time step kept on the device.

One step (section "Code structure"; the rebuild cadence of section "Too much
of a good thing?": lists rebuilt every 10 steps by default):

    every K steps: sph_build_neighbors        (re-bin, sort, lists)
    sph_forces(state n)      -> forces_n
    sph_step_dt(state n)     -> dt   (device double)
    sph_integrate(stage 0)   -> state *
    sph_forces(state *)      -> forces_*
    sph_integrate(stage 1)   -> state n+1 (in place), t += dt

The last two calls are one, sph_forces_corrector (the corrector's
derivatives and update in the same kernel, bit for bit the same state n+1;
forces_* is then not written), or sph_forces_corrector_scenes with a step
per scene.  Nothing is synchronised with the
host inside a step.
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi


def _i32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a).view(np.int32) if a.dtype == np.uint32 else np.ascontiguousarray(a, np.int32)


class Simulation:
    """Device state of one scene and the step sequence over the C ABI."""

    def __init__(self, grid, params, cell, pos, vel, info, max_neibs: int = 128, capacity: int | None = None,
                 rebuild_every: int = 10, device: str = "cuda", dt_fixed: float | None = None, cell_alpha=None,
                 brick=None, use_bricks: bool = True, cell_scene=None):
        n = int(np.asarray(cell).shape[0])
        cap = int(capacity or n)
        if cap < n or cap > abi.MAX_CAPACITY:
            raise ValueError("capacity must be in [n, 2^26]")
        self.n = n
        self.capacity = cap
        self.max_neibs = int(max_neibs)
        self.rebuild_every = int(rebuild_every)
        self.grid = grid
        self.params = params
        self.n_cells = int(np.prod(np.asarray(grid.ncell, dtype=np.int64)))
        self.device = torch.device(device)
        dev = self.device

        def z(shape, dtype):
            return torch.zeros(shape, dtype=dtype, device=dev)

        self.cell = z(cap, torch.int32)
        self.info = z(cap, torch.int32)
        self.pos = z((cap, 4), torch.float32)
        self.vel = z((cap, 4), torch.float32)
        self.pos_star = z((cap, 4), torch.float32)
        self.vel_star = z((cap, 4), torch.float32)
        self.forces_n = z((cap, 4), torch.float32)
        self.forces_star = z((cap, 4), torch.float32)
        self.neibs = z(abi.sph_neib_list_entries(cap, self.max_neibs), torch.int32)
        self.neibs_brick = z(abi.sph_neib_brick_entries(cap, self.max_neibs), torch.int16)
        self.neib_count = z(cap, torch.int32)
        self.cell_start = z(max(self.n_cells, 1), torch.int32)
        self.cell_end = z(max(self.n_cells, 1), torch.int32)
        self.status = z(abi.STATUS_WORDS, torch.int32)
        # missed pairs at rebuilds (sph_count_missed_pairs): previous lists'
        # interactions, new lists' interactions, their difference, running total
        self.missed = z(4, torch.int64)
        self.track_missed = False
        self.ws_build = z(abi.sph_build_workspace_bytes(cap, self.n_cells), torch.uint8)
        # scenes sharing the grid, each with its own time step and clock
        # (cell_scene: int32 per cell), or one scene
        self.cell_scene = None
        self.n_scenes = 1
        if cell_scene is not None:
            cs_np = np.ascontiguousarray(cell_scene, np.int32)
            if cs_np.shape != (self.n_cells,):
                raise ValueError("cell_scene must hold one scene index per cell")
            self.n_scenes = int(cs_np.max()) + 1
            if self.n_scenes < 1 or self.n_scenes > abi.MAX_SCENES:
                raise ValueError("cell_scene must name between 1 and %d scenes" % abi.MAX_SCENES)
            self.cell_scene = torch.from_numpy(cs_np).to(dev)
            self.ws_dt = z(abi.sph_dt_scenes_workspace_bytes(self.n_scenes), torch.uint8)
        else:
            self.ws_dt = z(abi.sph_dt_workspace_bytes(), torch.uint8)
        self.ws_forces = z(abi.sph_forces_workspace_bytes(cap, self.n_cells), torch.uint8)
        self.d_dt = z(self.n_scenes, torch.float64)
        self.d_time = z(self.n_scenes, torch.float64)
        self.count = z(1, torch.int64)
        self.dt_fixed = dt_fixed
        if dt_fixed is not None:
            self.d_dt.fill_(float(dt_fixed))

        self.cell[:n] = torch.from_numpy(_i32(cell))
        self.info[:n] = torch.from_numpy(_i32(np.asarray(info, np.uint32)))
        self.pos[:n] = torch.from_numpy(np.ascontiguousarray(pos, np.float32))
        self.vel[:n] = torch.from_numpy(np.ascontiguousarray(vel, np.float32))

        self.cell_alpha = None
        if cell_alpha is not None:
            self.cell_alpha = torch.from_numpy(np.ascontiguousarray(cell_alpha, np.float32)).to(dev)
        self.use_bricks = bool(use_bricks)
        shapes = abi.sph_brick_shapes()
        self.brick_shape = shapes[0] if brick is None else tuple(int(v) for v in brick)
        if self.brick_shape not in shapes:
            raise ValueError("brick shape %s not supported (%s)" % (self.brick_shape, shapes))
        self.g = abi.grid_struct(grid, self.cell_alpha, self.brick_shape)
        self.p = abi.params_struct(params)
        self.parts = abi.particles_struct(n, self.cell, self.pos, self.vel, self.info)
        self.parts_star = abi.particles_struct(n, self.cell, self.pos_star, self.vel_star, self.info)
        self.steps_done = 0
        self._built = False
        # the corrector's derivatives and update in one kernel (with a step
        # per scene for batched scenes)
        self.fuse_corrector = True

    # ------------------------------------------------------------ primitives
    def build(self, stream=None, perm_out=None, status=None):
        """Neighbour search (re-bin, sort, lists).  status: an int32 device
        tensor of STATUS_WORDS words to receive the build's status word
        instead of self.status.  With track_missed set, every rebuild after
        the first also counts the pairs within 2h that the replaced lists
        missed (self.missed)."""
        count = self.track_missed and self._built
        if count:
            abi.sph_count_missed_pairs(self.g, self.p, self.parts, self.neibs, self.neib_count, self.max_neibs,
                                       0, self.missed, stream)
        abi.sph_build_neighbors(self.g, self.p, self.parts, self.neibs, self.neib_count, self.max_neibs,
                                self.cell_start, self.cell_end, self.status if status is None else status,
                                self.ws_build, stream, perm_out, self.neibs_brick)
        if count:
            abi.sph_count_missed_pairs(self.g, self.p, self.parts, self.neibs, self.neib_count, self.max_neibs,
                                       1, self.missed, stream)
        self._built = True

    def set_brick(self, brick):
        """Change the brick shape of the LDS kernels; the lists must be
        rebuilt before the next derivative call."""
        shapes = abi.sph_brick_shapes()
        shape = tuple(int(v) for v in brick)
        if shape not in shapes:
            raise ValueError("brick shape %s not supported (%s)" % (shape, shapes))
        self.brick_shape = shape
        for d in range(3):
            self.g.brick[d] = shape[d]

    def set_params(self, **kw):
        """Change scalar parameters (e.g. alpha, c0) between calls."""
        for k, v in kw.items():
            setattr(self.p, k, float(v))

    def brick_args(self, bricks=None):
        """(cell_start, cell_end, neibs_brick) for the LDS brick kernels, or
        Nones for the per-particle gather kernels."""
        use = self.use_bricks if bricks is None else bricks
        return (self.cell_start, self.cell_end, self.neibs_brick) if use else (None, None, None)

    def forces(self, star: bool = False, stream=None, bricks: bool | None = None):
        """Derivatives of the state n (or *).  bricks: the LDS cell-brick
        kernel (uses the cell ranges and brick-local lists of the last
        build); False: the per-particle global-gather kernel; None: the
        simulation's choice (use_bricks).  The two agree to rounding."""
        parts = self.parts_star if star else self.parts
        out = self.forces_star if star else self.forces_n
        cs, ce, nb = self.brick_args(bricks)
        abi.sph_forces(self.g, self.p, parts, self.neibs, self.neib_count, self.max_neibs, out, self.ws_forces,
                       stream, cs, ce, nb)
        return out

    def corrector(self, stream=None, bricks: bool | None = None, forces=None):
        """The corrector half of the step in one kernel: the derivatives of
        state * and sph_integrate stage 1 (state n -> n+1 in place, t += dt),
        bit for bit forces(True) followed by integrate(1).  forces: a
        [capacity, 4] tensor that also receives the derivatives, or None."""
        cs, ce, nb = self.brick_args(bricks)
        if self.cell_scene is not None:
            abi.sph_forces_corrector_scenes(self.g, self.p, self.parts_star, self.neibs, self.neib_count,
                                            self.max_neibs, self.d_dt, self.cell_scene, self.n_scenes, self.parts,
                                            self.ws_forces, self.d_time, forces, stream, cs, ce, nb)
        else:
            abi.sph_forces_corrector(self.g, self.p, self.parts_star, self.neibs, self.neib_count, self.max_neibs,
                                     self.d_dt, self.parts, self.ws_forces, self.d_time, forces, stream, cs, ce, nb)

    def corrector_half(self, stream=None):
        """The derivatives of state * and the corrector stage: one call
        (corrector) for one scene, else the two separate calls."""
        if self.fuse_corrector:
            self.corrector(stream)
        else:
            self.forces(True, stream)
            self.integrate(1, stream)

    def step_dt(self, stream=None):
        if self.cell_scene is not None:
            abi.sph_step_dt_scenes(self.g, self.p, self.parts, self.forces_n, self.cell_scene, self.n_scenes,
                                   self.d_dt, self.ws_dt, stream)
        else:
            abi.sph_step_dt(self.p, self.parts, self.forces_n, self.d_dt, self.ws_dt, stream)

    def integrate(self, stage: int, stream=None):
        if self.cell_scene is not None:
            if stage == 0:
                abi.sph_integrate_scenes(self.g, self.p, 0, self.d_dt, self.cell_scene, self.n_scenes, self.parts,
                                         None, self.forces_n, self.parts_star, None, stream)
            else:
                abi.sph_integrate_scenes(self.g, self.p, 1, self.d_dt, self.cell_scene, self.n_scenes, self.parts,
                                         self.vel_star, self.forces_star, self.parts, self.d_time, stream)
        elif stage == 0:
            abi.sph_integrate(self.p, 0, self.d_dt, self.parts, None, self.forces_n, self.parts_star,
                              None, stream)
        else:
            abi.sph_integrate(self.p, 1, self.d_dt, self.parts, self.vel_star, self.forces_star, self.parts,
                              self.d_time, stream)

    DIAG_NAMES = ("mass", "mom_x", "mom_y", "mom_z", "force_x", "force_y", "force_z", "volume", "n_fluid",
                  "n_boundary", "max_rel_density", "kinetic")

    def diagnostics(self, with_forces: bool = True, stream=None) -> dict:
        """FP64 conservation sums of the current state (host dict; syncs)."""
        if not hasattr(self, "_diag_out"):
            self._diag_out = torch.zeros(12, dtype=torch.float64, device=self.device)
            self._diag_ws = torch.zeros(abi.sph_diagnostics_workspace_bytes(), dtype=torch.uint8,
                                        device=self.device)
        abi.sph_reduce_diagnostics(self.p, self.parts, self.forces_n if with_forces else None, self._diag_out,
                                   self._diag_ws, stream)
        return dict(zip(self.DIAG_NAMES, self._diag_out.cpu().numpy().tolist()))

    def count_interactions(self, stream=None) -> torch.Tensor:
        abi.sph_count_interactions(self.g, self.p, self.parts, self.neibs, self.neib_count, self.max_neibs,
                                   self.count, stream)
        return self.count

    # ------------------------------------------------------------ step
    def step(self, stream=None):
        if self.steps_done % self.rebuild_every == 0:
            self.build(stream)
        self.forces(False, stream)
        if self.dt_fixed is None:
            self.step_dt(stream)
        self.integrate(0, stream)
        self.corrector_half(stream)
        self.steps_done += 1

    def run(self, steps: int, stream=None):
        for _ in range(steps):
            self.step(stream)

    # ------------------------------------------------------------ HIP graph
    def capture_unit(self):
        """Record one rebuild unit (the neighbour search plus rebuild_every
        steps, about 6 + 5 K launches) into a HIP graph.  Nothing is
        executed while capturing; replay_units() then advances K steps per
        graph launch with no per-kernel launch overhead.  Must be called on a
        rebuild boundary.  The graph reads and writes this object's buffers,
        so it stays valid for the object's lifetime."""
        if self.steps_done % self.rebuild_every != 0:
            raise RuntimeError("capture_unit must start on a rebuild step")
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                self.build()
                for _ in range(self.rebuild_every):
                    self.forces(False)
                    if self.dt_fixed is None:
                        self.step_dt()
                    self.integrate(0)
                    self.corrector_half()
        torch.cuda.current_stream(self.device).wait_stream(side)
        self.graph = graph
        return graph

    def replay_units(self, units: int):
        for _ in range(units):
            self.graph.replay()
            self.steps_done += self.rebuild_every

    # ------------------------------------------------------------ host views
    @staticmethod
    def status_dict(words) -> dict:
        s = np.asarray(words)
        return {"n_active": int(s[abi.STATUS_N_ACTIVE]), "max_neibs": int(s[abi.STATUS_MAX_NEIBS]),
                "overflow": int(s[abi.STATUS_OVERFLOW]), "dropped": int(s[abi.STATUS_DROPPED]),
                "nonfinite": int(s[abi.STATUS_NONFINITE])}

    def status_host(self) -> dict:
        return self.status_dict(self.status.cpu().numpy())

    def raise_on_status(self, st: dict):
        """SphError for a build whose lists overflowed or whose state held
        non-finite values (particles that left the grid are not an error)."""
        if st["nonfinite"] > 0:
            raise abi.SphError("non-finite state: %d particles have a non-finite offset, mass, velocity or "
                               "density" % st["nonfinite"])
        if st["overflow"] > 0:
            raise abi.SphError("neighbour list overflow: %d particles need more than %d slots (max %d)"
                               % (st["overflow"], self.max_neibs, st["max_neibs"]))

    def check_status(self):
        st = self.status_host()
        self.raise_on_status(st)
        return st

    def missed_host(self) -> dict:
        m = self.missed.cpu().numpy()
        return {"previous_lists": int(m[0]), "new_lists": int(m[1]), "missed": int(m[2]), "missed_total": int(m[3])}

    def state_host(self) -> dict:
        n = self.n
        return {
            "cell": self.cell[:n].cpu().numpy(),
            "pos": self.pos[:n].cpu().numpy(),
            "vel": self.vel[:n].cpu().numpy(),
            "info": self.info[:n].cpu().numpy().view(np.uint32),
        }

    def lists_host(self):
        """(neibs [max_neibs, n] uint32 in slot-major order, neib_count [n] uint32)."""
        M = self.max_neibs
        t = self.neibs.view(-1, M, 64).cpu().numpy().view(np.uint32)  # [tile, slot, lane]
        nb = t.transpose(1, 0, 2).reshape(M, -1)[:, : self.n]
        cnt = self.neib_count[: self.n].cpu().numpy().view(np.uint32)
        return np.ascontiguousarray(nb), cnt

    @property
    def time(self):
        """Simulated time (host; syncs): a float, or one per scene."""
        if self.cell_scene is not None:
            return self.d_time.cpu().numpy()
        return float(self.d_time.item())
