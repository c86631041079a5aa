"""GPU parity of the adjoint entry points (sph_forces_backward,
sph_integrate_backward, sph_unpermute) and of the checkpointed rollout
gradient against the FP64 oracle reverse.

Tolerance of sph_forces_backward: the same bar as the derivatives, 1e-5 of
the condition scale, per particle and component: |g_gpu - g_oracle| <= 1e-5
S, where S is the oracle reverse evaluated with every factor in absolute
value (oracle.forces_reverse_scales: the sum over the pairs of both roles of
the magnitudes of each term's factors); a float evaluation in any order errs
by a few units of rounding (u = 6e-8) times about the number of terms, i.e.
well inside 1e-5 S.  The parameter derivatives (float64 sums of float32
terms) take the same bar against their own scales.
The 24-step rollout gradient differs from the FP64 oracle's by the float32
trajectory error (bounds set from the measured agreement, with margin)."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import scenes as S

from parity import compare_build, log, make_sim, support_edge_rows, torch_sync

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


ADJ_TOL = 1e-5


def _cmp(name, got, ref, scale, tol=ADJ_TOL):
    """|got - ref| <= tol scale for every element (no element left out)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.asarray(scale, np.float64)
    d = np.abs(got - ref)
    assert np.all(np.abs(ref) <= scale * (1 + 1e-12) + 1e-300), name + ": scale below the value"
    e = np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d > 0, np.inf, 0.0))
    m = np.abs(ref).max()
    log("%s: max |d|/S %.2e  (normwise |d|/max|ref| %.2e)" % (name, e.max(), d.max() / m if m > 0 else d.max()))
    assert e.max() <= tol, (name, e.max())


# random clouds at about lattice density with 192 slots: the gather form of
# the adjoint needs symmetric lists, which a truncated (overflowing) list is not
SCENES = {
    "cloud_av": (lambda: S.random_cloud(n=1100, box=(0.26, 0.2, 0.2), dp=0.02, seed=51, boundary_frac=0.25,
                                        u_sigma=0.3, rho_sigma=0.01, alpha=0.3), 192),
    "cloud_laminar_periodic": (lambda: S.random_cloud(n=1200, box=(0.26, 0.24, 0.2), dp=0.02, seed=52,
                                                      boundary_frac=0.2, u_sigma=0.3, rho_sigma=0.01, alpha=0.1,
                                                      visc_model=1, nu=2e-3, periodic=0b111), 192),
    "dam_break_64k": (lambda: S.dam_break_64k(), 128),
}


CASES = [(name, "bricks", None, 0.0) for name in SCENES] + [(name, "gather", None, 0.0) for name in SCENES] + \
    [("cloud_laminar_periodic", "bricks", (3, 3, 3), 0.0), ("cloud_av", "bricks", (3, 2, 3), 0.0)] + \
    [("cloud_av", "bricks", None, 0.1), ("cloud_laminar_periodic", "gather", None, 0.1),
     ("dam_break_64k", "bricks", None, 0.1)]


def _case_id(c):
    shape = "" if c[2] is None else "-" + "x".join(map(str, c[2]))
    return "%s-%s%s%s" % (c[0], c[1], shape, "-diffusion" if c[3] else "")


@pytest.mark.parametrize("name,form,shape,delta", CASES, ids=[_case_id(c) for c in CASES])
def test_forces_backward_parity(name, form, shape, delta):
    """Both forms of the adjoint (LDS bricks in two halves along y, also for
    odd brick heights; per-particle gather) against the FP64 oracle reverse,
    also with the density diffusion term."""
    import dataclasses
    make, M = SCENES[name]
    sc = make()
    if delta:
        sc = dataclasses.replace(sc, params=dataclasses.replace(sc.params, delta=delta))
    log("case %s n=%d bricks=%s shape=%s delta=%s" % (name, sc.n, form == "bricks", shape, delta))
    _backward_parity(sc, M, form == "bricks", shape, name)


def _backward_parity(sc, M, bricks, shape, name):
    sim = make_sim(sc, max_neibs=M, brick=shape)
    sim.build()
    torch_sync()
    ob = compare_build(sc, sim, max_neibs=M)
    assert ob["lists"].overflow == 0
    st = O.State.lift(ob["cell"], ob["pos"], ob["vel"], ob["info"])
    rng = np.random.default_rng(7)
    gf = np.zeros((sc.n, 4), np.float32)
    gf[:, :3] = rng.normal(size=(sc.n, 3))
    gf[:, 3] = rng.normal(size=sc.n) * 1e-3
    adj, gp = O.forces_reverse(sc.grid, sc.params, st, ob["lists"], gf[:, :3].astype(np.float64),
                               gf[:, 3].astype(np.float64))
    scl, sp = O.forces_reverse_scales(sc.grid, sc.params, st, ob["lists"], gf[:, :3].astype(np.float64),
                                      gf[:, 3].astype(np.float64))
    from paper_2207_11328_amd import abi
    dev = sim.device
    gforce = torch.from_numpy(gf).to(dev)
    gpos = torch.full((sim.capacity, 4), 7.0, device=dev)
    gvel = torch.zeros((sim.capacity, 4), device=dev)
    gparams = torch.zeros(3, dtype=torch.float64, device=dev)
    ws = torch.zeros(abi.sph_forces_backward_workspace_bytes(sim.capacity, sim.n_cells), dtype=torch.uint8,
                     device=dev)
    bk = dict(cell_start=sim.cell_start, cell_end=sim.cell_end, neibs_brick=sim.neibs_brick) if bricks else {}
    abi.sph_forces_backward(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, gforce, gpos, gvel,
                            gparams, False, ws, **bk)
    torch_sync()
    gp_gpu = gpos[: sc.n].cpu().numpy()
    gv_gpu = gvel[: sc.n].cpu().numpy()
    assert np.all(gp_gpu[:, 3] == 7.0), "w of grad_pos must be left untouched"
    keep = slice(None)
    if int(getattr(sc.params, "kernel", 0)) == O.GAUSSIAN:
        # pairs at the edge of the truncated Gaussian's support (see support_edge_rows)
        edge = support_edge_rows(sc, ob)
        log("%s: %d of %d particles within 2e-6 of 2h of a neighbour left out" % (name, edge.sum(), sc.n))
        assert edge.mean() < 0.005
        keep = ~edge
    _cmp(name + " dL/do", gp_gpu[keep, :3], adj.go[keep], scl.go[keep])
    _cmp(name + " dL/du", gv_gpu[keep, :3], adj.gu[keep], scl.gu[keep])
    _cmp(name + " dL/drho", gv_gpu[keep, 3], adj.grho[keep], scl.grho[keep])
    g = gparams.cpu().numpy()
    log("%s params gpu %s oracle %s |d|/S %s" % (name, g, gp, np.abs(g - gp) / np.where(sp > 0, sp, 1.0)))
    for k in range(3):
        assert abs(g[k] - gp[k]) <= ADJ_TOL * sp[k], (k, g[k], gp[k], sp[k])
    # accumulate mode adds to what is there; deterministic bit for bit
    gpos2 = gpos.clone()
    gvel2 = gvel.clone()
    gparams2 = gparams.clone()
    abi.sph_forces_backward(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, gforce, gpos2,
                            gvel2, gparams2, True, ws, **bk)
    torch_sync()
    assert torch.allclose(gvel2, 2 * gvel, rtol=1e-6, atol=0)
    assert torch.allclose(gparams2, 2 * gparams, rtol=1e-12, atol=0)
    abi.sph_forces_backward(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, gforce, gpos2,
                            gvel2, gparams2, False, ws, **bk)
    torch_sync()
    assert torch.equal(gvel2, gvel) and torch.equal(gparams2, gparams)


# every compiled model: kernel x laminar term x formulation x diffusion
VARIANTS = [(k, v, f, d) for k in range(4) for v in range(3) for f in range(2) for d in (0.0, 0.1)]


def _variant_id(v):
    return "%s-%s-%s%s" % (["wendland", "cubic", "quadratic", "gaussian"][v[0]], ["av", "morris", "monaghan_k"][v[1]],
                           ["golden", "landrini"][v[2]], "-diffusion" if v[3] else "")


def _variant_case(name, variant, bricks):
    import dataclasses
    kernel, visc, form, delta = variant
    make, M = SCENES[name]
    sc = make()
    sc = dataclasses.replace(sc, params=dataclasses.replace(sc.params, kernel=kernel, visc_model=visc, nu=2e-3,
                                                              formulation=form, delta=delta))
    log("case %s %s bricks=%s n=%d" % (name, _variant_id(variant), bricks, sc.n))
    _backward_parity(sc, M, bricks, None, name + " " + _variant_id(variant))


@pytest.mark.parametrize("variant", VARIANTS, ids=[_variant_id(v) for v in VARIANTS])
def test_model_variants_backward_bricks(variant):
    """The adjoint of every compiled model (kernel, formulation, laminar
    term, diffusion) in the LDS brick form against the oracle reverse,
    parameter derivatives included."""
    _variant_case("cloud_av", variant, True)


BACK_GATHER = [(1, 1, 1, 0.1), (2, 2, 0, 0.0), (3, 2, 1, 0.1), (0, 2, 1, 0.0), (3, 1, 0, 0.0)]


@pytest.mark.parametrize("variant", BACK_GATHER, ids=[_variant_id(v) for v in BACK_GATHER])
def test_model_variants_backward_gather(variant):
    """A spread of the models in the per-particle gather form of the adjoint,
    on the periodic cloud."""
    _variant_case("cloud_laminar_periodic", variant, False)


BACK_DAM = [(1, 2, 1, 0.1), (3, 1, 0, 0.0)]


@pytest.mark.parametrize("variant", BACK_DAM, ids=[_variant_id(v) for v in BACK_DAM])
def test_model_variants_backward_dam_break(variant):
    _variant_case("dam_break_64k", variant, True)


def test_backward_brick_skip_any_workspace_contents():
    """The adjoint skips the bricks whose particles all have empty lists as the
    derivative kernel does (its prologue writes their zero adjoint unless the
    call accumulates): bit-identical results whatever the workspace held,
    in both modes, on the 64k dam break."""
    from paper_2207_11328_amd import abi
    sc = S.dam_break_64k()
    sim = make_sim(sc, max_neibs=128)
    sim.build()
    torch_sync()
    dev = sim.device
    assert int((sim.neib_count[: sc.n] == 0).sum()) > 1000
    g = torch.Generator(device=dev).manual_seed(5)
    gforce = torch.randn((sim.capacity, 4), device=dev, generator=g)
    bk = dict(cell_start=sim.cell_start, cell_end=sim.cell_end, neibs_brick=sim.neibs_brick)
    nbytes = abi.sph_forces_backward_workspace_bytes(sim.capacity, sim.n_cells)

    def run(fill, accumulate, base):
        ws = torch.full((nbytes,), fill, dtype=torch.uint8, device=dev)
        gpos = base[0].clone()
        gvel = base[1].clone()
        gpar = torch.zeros(3, dtype=torch.float64, device=dev)
        abi.sph_forces_backward(sim.g, sim.p, sim.parts, sim.neibs, sim.neib_count, sim.max_neibs, gforce, gpos,
                                gvel, gpar, accumulate, ws, **bk)
        torch_sync()
        return gpos, gvel, gpar

    start = (torch.full((sim.capacity, 4), float("nan"), device=dev), torch.full((sim.capacity, 4), float("nan"),
                                                                                  device=dev))
    start[0][:, 3] = 3.0
    ref = run(0, False, start)
    assert torch.isfinite(ref[0][: sc.n]).all() and torch.isfinite(ref[1][: sc.n]).all()
    assert (ref[0][: sc.n, 3] == 3.0).all()
    for fill in (0xFF, 0x01):
        got = run(fill, False, start)
        for x, y in zip(ref, got):
            assert torch.equal(x[: sc.n] if x.dim() == 2 else x, y[: sc.n] if y.dim() == 2 else y), fill
    acc0 = run(0, True, ref[:2])
    acc1 = run(0xFF, True, ref[:2])
    for x, y in zip(acc0, acc1):
        assert torch.equal(x, y)
    empty = sim.neib_count[: sc.n] == 0
    assert torch.equal(acc0[0][: sc.n][empty], ref[0][: sc.n][empty])
    assert torch.equal(acc0[1][: sc.n][empty], ref[1][: sc.n][empty])


def test_integrate_backward_parity():
    sc = S.random_cloud(n=800, box=(0.2, 0.2, 0.2), dp=0.02, seed=53, boundary_frac=0.3, u_sigma=0.2)
    sim = make_sim(sc, max_neibs=192)
    sim.build()
    torch_sync()
    ob = compare_build(sc, sim, max_neibs=192)
    st = O.State.lift(ob["cell"], ob["pos"], ob["vel"], ob["info"])
    from paper_2207_11328_amd import abi
    dev = sim.device
    rng = np.random.default_rng(8)
    dt = 3e-4
    sim.d_dt.fill_(dt)
    n, cap = sc.n, sim.capacity
    gp = np.zeros((n, 4), np.float32)
    gv = np.zeros((n, 4), np.float32)
    gp[:, :3] = rng.normal(size=(n, 3))
    gv[:, :3] = rng.normal(size=(n, 3))
    gv[:, 3] = rng.normal(size=n)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    tgp, tgv = T(np.zeros((cap, 4), np.float32)), T(np.zeros((cap, 4), np.float32))
    tgp[:n], tgv[:n] = T(gp), T(gv)
    tps, tvs, tgf = (torch.zeros((cap, 4), device=dev) for _ in range(3))
    abi.sph_integrate_backward(sim.p, 1, sim.d_dt, sim.parts, tgp, tgv, tps, tvs, tgf)
    torch_sync()
    adj_next = O.Adj(gp[:, :3].astype(np.float64), gv[:, :3].astype(np.float64), gv[:, 3].astype(np.float64))
    base1, gu_star, abar1, dbar1 = O.integrate_reverse(1, dt, st, adj_next)
    u = 2.0 ** -24
    assert np.allclose(tgf[:n, :3].cpu().numpy(), abar1, rtol=2 * u, atol=0)
    assert np.allclose(tgf[:n, 3].cpu().numpy(), dbar1, rtol=2 * u, atol=0)
    assert np.allclose(tvs[:n, :3].cpu().numpy(), gu_star, rtol=2 * u, atol=0)
    assert np.all(tps[:n].cpu().numpy() == 0) and np.all(tvs[:n, 3].cpu().numpy() == 0)
    # stage 0 with a random dL/dy*
    sp = rng.normal(size=(n, 4)).astype(np.float32)
    sv = rng.normal(size=(n, 4)).astype(np.float32)
    tps[:n], tvs[:n] = T(sp), T(sv)
    abi.sph_integrate_backward(sim.p, 0, sim.d_dt, sim.parts, tgp, tgv, tps, tvs, tgf)
    torch_sync()
    adj_star = O.Adj(sp[:, :3].astype(np.float64), sv[:, :3].astype(np.float64), sv[:, 3].astype(np.float64))
    base0, _, abar0, dbar0 = O.integrate_reverse(0, dt, st, adj_star)
    got_p = tgp[:n, :3].cpu().numpy().astype(np.float64)
    got_v = tgv[:n].cpu().numpy().astype(np.float64)
    assert np.allclose(got_p, gp[:, :3] + base0.go, rtol=4 * u, atol=4 * u * np.abs(gp[:, :3]).max())
    assert np.allclose(got_v[:, :3], gv[:, :3] + base0.gu, rtol=4 * u, atol=4 * u * 3)
    assert np.allclose(got_v[:, 3], gv[:, 3] + base0.grho, rtol=4 * u, atol=4 * u * 3)
    assert np.allclose(tgf[:n, :3].cpu().numpy(), abar0, rtol=2 * u, atol=0)
    assert np.allclose(tgf[:n, 3].cpu().numpy(), dbar0, rtol=2 * u, atol=0)


def test_unpermute_inverts_the_build_permutation():
    sc = S.shuffled(S.random_cloud(n=1400, box=(0.3, 0.2, 0.2), dp=0.02, seed=54), seed=2)
    sim = make_sim(sc, max_neibs=192)
    from paper_2207_11328_amd import abi
    perm = torch.zeros(sim.capacity, dtype=torch.int32, device=sim.device)
    before = sim.vel.clone()
    sim.build(perm_out=perm)
    torch_sync()
    ob = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, 192)
    assert np.array_equal(perm[: sc.n].cpu().numpy(), ob["perm"])
    back = torch.zeros_like(sim.vel)
    abi.sph_unpermute(sc.n, perm, sim.vel, back)
    torch_sync()
    assert torch.equal(back[: sc.n], before[: sc.n])


def _front(sc, steps, dt):
    st0 = O.State.lift(sc.cell, sc.pos, sc.vel, sc.info)
    base, _ = O.rollout(sc.grid, sc.params, st0.copy(), steps, rebuild_every=10, dt_fixed=dt)
    x = O.positions(sc.grid, base)
    fl = base.is_fluid
    ids = (base.info & np.uint32((1 << 30) - 1)).astype(np.int64)
    k = int(np.ceil(0.01 * fl.sum()))
    return ids[fl][np.argsort(-x[fl, 0])[:k]], st0


@pytest.mark.parametrize("variant", [None, (1, 2, 1, 0.1)], ids=["default", "cubic-monaghan_k-landrini-diffusion"])
def test_rollout_gradient_matches_oracle_reverse(variant):
    """Differentiable dam break (reduced size), 24 fixed-dt steps, rebuild
    every 10, checkpoint every 20: dL/d(alpha, c0, u0) of L = mean x of the
    front particles, through torch.autograd, against the FP64 oracle; for the
    default model and for a variant (cubic spline, Landrini-Morris, Monaghan
    K laminar term, density diffusion)."""
    import dataclasses
    from paper_2207_11328_amd.adjoint import AdjointRollout, SPHRollout
    sc = S.dam_break(dp=0.04, u0_sigma=0.01, seed=2)
    if variant is not None:
        kernel, visc, form, delta = variant
        sc = dataclasses.replace(sc, params=dataclasses.replace(sc.params, kernel=kernel, visc_model=visc, nu=1e-3,
                                                                  formulation=form, delta=delta))
    steps, dt = 24, 1.5e-4
    front, st0 = _front(sc, steps, dt)
    L_o, adj_o, gp_o, _ = O.rollout_adjoint(sc.grid, sc.params, st0, steps, dt, O.front_loss(sc.grid, front))
    runner = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=steps, dt=dt,
                            rebuild_every=10, checkpoint_every=20)
    dev = runner.sim.device
    vel0 = torch.from_numpy(sc.vel[:, :3].copy()).to(dev).requires_grad_(True)
    alpha = torch.tensor(float(np.float32(sc.params.alpha)), dtype=torch.float64, requires_grad=True)
    c0 = torch.tensor(float(np.float32(sc.params.c0)), dtype=torch.float64, requires_grad=True)
    x, u, rho = SPHRollout.apply(vel0, alpha, c0, runner)
    sel = torch.from_numpy(np.asarray(front)).to(dev)
    L = x[sel, 0].mean()
    L.backward()
    torch_sync()
    log("loss gpu %.12f oracle %.12f" % (L.item(), L_o))
    assert abs(L.item() - L_o) < 1e-6
    ga, gc = alpha.grad.item(), c0.grad.item()
    log("dL/dalpha gpu %.6e oracle %.6e ; dL/dc0 gpu %.6e oracle %.6e" % (ga, gp_o[0], gc, gp_o[1]))
    # measured: 1.1e-6 and 2.9e-6 (alpha), <= 4e-7 (c0), 1.6e-7 (u0, normwise)
    assert abs(ga - gp_o[0]) <= 2e-5 * abs(gp_o[0])
    assert abs(gc - gp_o[1]) <= 2e-5 * abs(gp_o[1])
    gu = vel0.grad.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(gu - adj_o.gu) / np.linalg.norm(adj_o.gu)
    log("dL/du0 relative L2 error %.3e" % rel)
    assert rel <= 2e-6


def test_taped_blocks_match_recomputation():
    """The reverse of taped blocks (lists, order and stage states kept from
    the forward) gives the same bits as the reverse that rebuilds and re-runs
    them from checkpoints: 24 steps, rebuild every 10, checkpoint every 20,
    with no block, the last block and every block taped."""
    from paper_2207_11328_amd.adjoint import AdjointRollout
    sc = S.dam_break(dp=0.04, u0_sigma=0.01, seed=2)
    steps, dt = 24, 1.5e-4
    runs = {}
    for name in ("none", "last", "all"):
        r = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=steps, dt=dt,
                           rebuild_every=10, checkpoint_every=20, tape_bytes=0)
        budget = {"none": 0, "last": r.tape_block_bytes(), "all": 3 * r.tape_block_bytes()}[name]
        r = AdjointRollout(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info, steps=steps, dt=dt,
                           rebuild_every=10, checkpoint_every=20, tape_bytes=budget)
        assert r.n_taped == {"none": 0, "last": 1, "all": 3}[name]
        g = torch.Generator(device=r.sim.device).manual_seed(5)
        seed_p = torch.randn((r.n, 4), device=r.sim.device, generator=g)
        seed_v = torch.randn((r.n, 4), device=r.sim.device, generator=g)
        final = []
        for rep in range(2):  # a second forward/backward on the same buffers
            r.reset()
            r.forward()
            final.append(r.sim.pos[: r.n].clone())
            gp, gv, gpar = r.backward(seed_p, seed_v)
            runs[(name, rep)] = (gp.cpu().numpy().copy(), gv.cpu().numpy().copy(), gpar.cpu().numpy().copy())
            # the final state is back in place after the reverse
            assert torch.equal(r.sim.pos[: r.n], final[-1])
        del r
    ref = runs[("none", 0)]
    for key, val in runs.items():
        for a, b in zip(ref, val):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), key
    log("taped and recomputed reverses agree bit for bit")
