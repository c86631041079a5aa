"""Differentiable fixed-dt rollouts over the C ABI.

The last K-step blocks of the rollout, as many as a device-memory budget
allows (`tape_bytes`; by default half of the free device memory), are taped:
their build writes its lists into buffers of their own and the forward keeps
their sort permutation, particle order and stage states y^n and y*, so the
reverse replays them without rebuilding or re-running anything.  For the
blocks before them the forward keeps a checkpoint of the full particle state
every `checkpoint_every` steps (a multiple of the rebuild interval K); the
reverse walks those checkpoint segments backwards; inside a segment it
re-runs the forward once to recover the state before each rebuild, then for
every block (last to first): restores the pre-rebuild state, rebuilds (the
same lists and the same sort permutation as the forward, the build being
deterministic), re-runs the K steps keeping the stage states, and applies
the reverse step

    sph_integrate_backward(1) -> sph_forces_backward(y*) ->
    sph_integrate_backward(0) -> sph_forces_backward(y^n)

K times, then carries the adjoint back across the rebuild with
sph_unpermute.  The time step is frozen (treated as a constant), so the
reverse differentiates exactly the function the forward evaluates.

`SPHRollout` wraps a rollout as a torch.autograd.Function of the initial
velocities and of (alpha, c0).
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi
from .sim import Simulation


class AdjointRollout:
    def __init__(self, grid, params, cell, pos, vel, info, steps: int, dt: float, rebuild_every: int = 10,
                 checkpoint_every: int = 20, max_neibs: int = 128, device: str = "cuda", brick=None,
                 use_bricks: bool = True, tape_bytes: int | None = None):
        if checkpoint_every % rebuild_every != 0:
            raise ValueError("checkpoint_every must be a multiple of rebuild_every")
        self.steps = int(steps)
        self.K = int(rebuild_every)
        self.C = int(checkpoint_every)
        self.dt = float(dt)
        self.sim = Simulation(grid, params, cell, pos, vel, info, max_neibs=max_neibs, rebuild_every=rebuild_every,
                              device=device, dt_fixed=dt, brick=brick, use_bricks=use_bricks)
        s = self.sim
        n, cap, dev = s.n, s.capacity, s.device

        def z(shape, dtype=torch.float32):
            return torch.zeros(shape, dtype=dtype, device=dev)

        self.gpos, self.gvel = z((cap, 4)), z((cap, 4))
        self.gpos_s, self.gvel_s = z((cap, 4)), z((cap, 4))
        self.gforce = z((cap, 4))
        self.tmp_p, self.tmp_v = z((cap, 4)), z((cap, 4))
        self.perm = z(cap, torch.int32)
        self.ws_back = z(abi.sph_forces_backward_workspace_bytes(cap, s.n_cells), torch.uint8)
        self.grad_params = z(3, torch.float64)
        # status word of every build of the forward and of the reverse (the
        # reverse rebuilds each block's lists); checked once at the end of each
        n_builds = max(1, (self.steps + self.K - 1) // self.K)
        self.fwd_status = z((n_builds, abi.STATUS_WORDS), torch.int32)
        self.bwd_status = z((n_builds, abi.STATUS_WORDS), torch.int32)
        self.initial = self._snapshot()
        self.checkpoints = {}
        self.n = n
        # the tape: the last n_taped blocks (buffers allocated once, reused
        # by every forward)
        n_blocks = (self.steps + self.K - 1) // self.K
        if tape_bytes is None:
            free, _total = torch.cuda.mem_get_info(torch.device(dev))
            tape_bytes = free // 2
        per_block = self.tape_block_bytes()
        self.n_taped = int(min(n_blocks, max(0, int(tape_bytes) // per_block)))
        self.first_taped = n_blocks - self.n_taped  # block index
        self.tape = {}
        for b in range(self.first_taped, n_blocks):
            self.tape[b] = {
                "neibs": torch.empty_like(s.neibs), "neib_count": torch.empty_like(s.neib_count),
                "neibs_brick": torch.empty_like(s.neibs_brick), "cell_start": torch.empty_like(s.cell_start),
                "cell_end": torch.empty_like(s.cell_end), "perm": torch.empty_like(self.perm),
                "cell": torch.empty_like(s.cell), "info": torch.empty_like(s.info), "stored": None,
            }
        self._own_lists = (s.neibs, s.neib_count, s.neibs_brick, s.cell_start, s.cell_end)

    def tape_block_bytes(self) -> int:
        """Device bytes of one taped block: its lists, cell ranges,
        permutation and particle order, and the K steps' stage states."""
        s = self.sim
        lists = sum(t.numel() * t.element_size()
                    for t in (s.neibs, s.neib_count, s.neibs_brick, s.cell_start, s.cell_end))
        order = 3 * s.cell.numel() * s.cell.element_size()
        stages = self.K * 4 * s.pos.numel() * s.pos.element_size()
        return lists + order + stages

    def _use_lists(self, bufs):
        """Point the simulation's list buffers at bufs (neibs, neib_count,
        neibs_brick, cell_start, cell_end): every call reads them from there."""
        s = self.sim
        s.neibs, s.neib_count, s.neibs_brick, s.cell_start, s.cell_end = bufs

    def _tape_lists(self, b):
        t = self.tape[b]
        return (t["neibs"], t["neib_count"], t["neibs_brick"], t["cell_start"], t["cell_end"])

    # ------------------------------------------------------------ state helpers
    def _snapshot(self):
        s = self.sim
        return tuple(t.clone() for t in (s.cell, s.pos, s.vel, s.info, s.d_time))

    def _restore(self, snap):
        s = self.sim
        for dst, src in zip((s.cell, s.pos, s.vel, s.info, s.d_time), snap):
            dst.copy_(src)

    def _check_builds(self, status, n_builds):
        """Raise SphError if any build overflowed its lists (a truncated list
        is not symmetric, and the gather adjoint assumes it is) or met a
        non-finite state."""
        for row in status[:n_builds].cpu().numpy():
            self.sim.raise_on_status(self.sim.status_dict(row))

    def _advance(self, store=None):
        """One predictor/corrector step on the current lists (no rebuild),
        the corrector as the simulation's step takes it (one fused call for
        one scene, bit for bit the separate calls)."""
        s = self.sim
        if store is not None:
            store.append([s.pos.clone(), s.vel.clone(), None, None])
        s.forces(False)
        s.integrate(0)
        if store is not None:
            store[-1][2] = s.pos_star.clone()
            store[-1][3] = s.vel_star.clone()
        s.corrector_half()

    def reset(self, vel0=None, alpha=None, c0=None):
        """Back to the initial state, optionally with new initial velocities
        (device float[n][3], initial particle order) and parameters."""
        self._restore(self.initial)
        if vel0 is not None:
            self.sim.vel[: self.n, :3] = vel0.to(self.sim.vel.dtype)
        kw = {}
        if alpha is not None:
            kw["alpha"] = float(alpha)
        if c0 is not None:
            kw["c0"] = float(c0)
        if kw:
            self.sim.set_params(**kw)
        self.sim.d_time.zero_()
        self.checkpoints = {}

    # ------------------------------------------------------------ forward
    def forward(self):
        s = self.sim
        self.fwd_status.zero_()
        self._use_lists(self._own_lists)
        stored = None
        for k in range(self.steps):
            b = k // self.K
            if k % self.C == 0 and b < self.first_taped:
                self.checkpoints[k] = self._snapshot()
            if k % self.K == 0:
                if b < self.first_taped:
                    s.build(status=self.fwd_status[b])
                    stored = None
                else:
                    t = self.tape[b]
                    self._use_lists(self._tape_lists(b))
                    s.build(perm_out=t["perm"], status=self.fwd_status[b])
                    t["cell"].copy_(s.cell)
                    t["info"].copy_(s.info)
                    stored = t["stored"] = []
            self._advance(stored)
        self._check_builds(self.fwd_status, (self.steps + self.K - 1) // self.K)
        return s

    # ------------------------------------------------------------ reverse
    def _reverse_step(self, pos_n, vel_n, pos_s, vel_s):
        s = self.sim
        pn = abi.particles_struct(s.n, s.cell, pos_n, vel_n, s.info)
        ps = abi.particles_struct(s.n, s.cell, pos_s, vel_s, s.info)
        abi.sph_integrate_backward(s.p, 1, s.d_dt, pn, self.gpos, self.gvel, self.gpos_s, self.gvel_s, self.gforce)
        cs, ce, nb = s.brick_args()
        bk = dict(cell_start=cs, cell_end=ce, neibs_brick=nb)
        abi.sph_forces_backward(s.g, s.p, ps, s.neibs, s.neib_count, s.max_neibs, self.gforce, self.gpos_s,
                                self.gvel_s, self.grad_params, True, self.ws_back, **bk)
        abi.sph_integrate_backward(s.p, 0, s.d_dt, pn, self.gpos, self.gvel, self.gpos_s, self.gvel_s, self.gforce)
        abi.sph_forces_backward(s.g, s.p, pn, s.neibs, s.neib_count, s.max_neibs, self.gforce, self.gpos,
                                self.gvel, self.grad_params, True, self.ws_back, **bk)

    def _carry_back(self, perm):
        """Adjoint across a rebuild: from the sorted order it made back to
        the order before it."""
        n = self.n
        abi.sph_unpermute(n, perm, self.gpos, self.tmp_p)
        abi.sph_unpermute(n, perm, self.gvel, self.tmp_v)
        self.gpos, self.tmp_p = self.tmp_p, self.gpos
        self.gvel, self.tmp_v = self.tmp_v, self.gvel

    def reverse_block(self, stored):
        """Reverse the steps of one block given their stored stage states."""
        for pos_n, vel_n, pos_s, vel_s in reversed(stored):
            self._reverse_step(pos_n, vel_n, pos_s, vel_s)

    def backward(self, gpos_final, gvel_final):
        """Adjoint of the final state (device float[n][4] each, final sorted
        order; grad_pos xyz = dL/d(offset), grad_vel = (dL/du, dL/drho)) ->
        adjoint of the initial state (initial particle order) and
        dL/d(alpha, c0, nu) (device double[3])."""
        s = self.sim
        n = s.n
        final = self._snapshot()  # the final state, put back at the end
        self.bwd_status.zero_()
        self.gpos.zero_()
        self.gvel.zero_()
        self.gpos[:n] = gpos_final
        self.gvel[:n] = gvel_final
        self.grad_params.zero_()
        # the taped blocks, last to first: their lists, order and stage states
        # as the forward left them
        for b in sorted(self.tape, reverse=True):
            t = self.tape[b]
            if t["stored"] is None:
                raise RuntimeError("backward() needs a forward() of the rollout first")
            self._use_lists(self._tape_lists(b))
            s.cell.copy_(t["cell"])
            s.info.copy_(t["info"])
            self.reverse_block(t["stored"])
            self._carry_back(t["perm"])
        self._use_lists(self._own_lists)
        # the blocks before them from the checkpoints
        taped_from = self.first_taped * self.K
        for c in sorted(self.checkpoints, reverse=True):
            end = min(c + self.C, self.steps, taped_from)
            blocks = list(range(c, end, self.K))
            self._restore(self.checkpoints[c])
            pre = {}
            for b in blocks:
                pre[b] = self._snapshot()
                if b != blocks[-1]:
                    s.build(status=self.bwd_status[b // self.K])
                    for _ in range(self.K):
                        self._advance()
            for b in reversed(blocks):
                self._restore(pre[b])
                s.build(perm_out=self.perm, status=self.bwd_status[b // self.K])
                stored = []
                for _ in range(b, min(b + self.K, end)):
                    self._advance(stored)
                self.reverse_block(stored)
                self._carry_back(self.perm)
        self._restore(final)
        if self.tape:
            self._use_lists(self._tape_lists(max(self.tape)))
        self._check_builds(self.bwd_status, (self.steps + self.K - 1) // self.K)
        return self.gpos[:n], self.gvel[:n], self.grad_params

    # ------------------------------------------------------------ outputs
    def outputs_by_id(self):
        """Final positions (double, physical), velocities and densities in
        particle-id order, and the id order of the sorted state."""
        s = self.sim
        n = s.n
        g = s.grid
        ids = (s.info[:n].long() & ((1 << 30) - 1))
        nx, ny = int(g.ncell[0]), int(g.ncell[1])
        lc = s.cell[:n].long() - int(g.cell_base)
        c = torch.stack([lc % nx, (lc // nx) % ny, lc // (nx * ny)], dim=1).double()
        cs = torch.tensor(np.asarray(g.cell_size, np.float32).astype(np.float64), device=s.device)
        org = torch.tensor(np.asarray(g.origin, np.float64), device=s.device)
        x = org[None, :] + (c + 0.5) * cs[None, :] + s.pos[:n, :3].double()
        order = torch.argsort(ids)
        return x[order], s.vel[:n, :3][order], s.vel[:n, 3][order], order


class SPHRollout(torch.autograd.Function):
    """(initial velocities [n,3] in id order, alpha, c0) -> final (x, u, rho)
    in id order.  Backward runs the checkpointed adjoint."""

    @staticmethod
    def forward(ctx, vel0, alpha, c0, runner: AdjointRollout):
        runner.reset(vel0.detach(), float(alpha), float(c0))
        runner.forward()
        x, u, rho, order = runner.outputs_by_id()
        ctx.runner = runner
        ctx.order = order
        ctx.param_like = (alpha, c0)
        return x, u.clone(), rho.clone()

    @staticmethod
    def backward(ctx, gx, gu, grho):
        runner = ctx.runner
        order = ctx.order
        n = runner.n
        dev = runner.sim.device
        gp = torch.zeros((n, 4), dtype=torch.float32, device=dev)
        gv = torch.zeros((n, 4), dtype=torch.float32, device=dev)
        if gx is not None:
            gp[order, :3] = gx.float()
        if gu is not None:
            gv[order, :3] = gu.float()
        if grho is not None:
            gv[order, 3] = grho.float()
        g0p, g0v, gparams = runner.backward(gp, gv)
        a, c = ctx.param_like
        ga = gparams[0].to(device=a.device, dtype=a.dtype) if torch.is_tensor(a) else None
        gc = gparams[1].to(device=c.device, dtype=c.dtype) if torch.is_tensor(c) else None
        return g0v[:, :3].clone(), ga, gc, None
