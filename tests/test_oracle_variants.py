"""Pins of the oracle's kernel and formulation variants: the cubic-spline,
quadratic and truncated Gaussian smoothing kernels (listing l:ktemplate and
the kernel options of "The SPH in GPUSPH"), the Landrini-Morris formulation
(eq. mass-cont-sph2, eq. ns-sph2) and Monaghan's K form of the laminar
viscosity (section "Minimizing complexity").

As in the other pin files, nothing here compares the oracle with itself:
normalisation and derivative identities are checked by quadrature and finite
differences, the formulations by invariants they have by construction and by
their continuum limits on a lattice.
"""
import copy
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from workloads import scenes as S

KINDS = [O.WENDLAND, O.CUBIC_SPLINE, O.QUADRATIC, O.GAUSSIAN]


# ------------------------------------------------------------------ kernels
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("h", [0.026, 1.0, 3.7e-3])
def test_kernel_unit_integral(kind, h):
    """Every smoothing kernel integrates to one over its support of radius 2h."""
    val, err = integrate.quad(lambda r: 4.0 * math.pi * r * r * O.kernel_W(kind, r, h), 0.0, 2.0 * h,
                              points=[h], epsabs=0.0, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-11


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("q", [0.05, 0.4, 0.9, 0.999, 1.001, 1.3, 1.7, 1.99])
def test_kernel_F_and_dF_are_derivatives(kind, q):
    """F = (1/r) dW/dr and dF/dr, by central differences of W and F."""
    h = 0.031
    r = q * h
    e = 1e-7 * h
    dW = (O.kernel_W(kind, r + e, h) - O.kernel_W(kind, r - e, h)) / (2 * e)
    F = O.kernel_F(kind, r, h)
    assert abs(dW / r - F) <= 2e-7 * abs(F)
    dF = (O.kernel_F(kind, r + e, h) - O.kernel_F(kind, r - e, h)) / (2 * e)
    G = O.kernel_dF(kind, r, h)
    assert abs(dF - G) <= 2e-6 * abs(G)


@pytest.mark.parametrize("kind", KINDS)
def test_kernel_support_sign_and_monotonicity(kind):
    """Zero from r = 2h on; W > 0 and decreasing inside (F < 0)."""
    h = 0.5
    for q in (2.0, 2.0 + 1e-12, 2.5, 7.0):
        assert O.kernel_W(kind, q * h, h) == 0.0
        assert O.kernel_F(kind, q * h, h) == 0.0
        assert O.kernel_dF(kind, q * h, h) == 0.0
    qs = np.linspace(1e-3, 2.0 - 1e-9, 400)
    W = np.array([O.kernel_W(kind, q * h, h) for q in qs])
    F = np.array([O.kernel_F(kind, q * h, h) for q in qs])
    assert np.all(W > 0) and np.all(np.diff(W) < 0) and np.all(F < 0)
    # W is continuous at the edge of the support
    assert O.kernel_W(kind, (2.0 - 1e-9) * h, h) < 1e-6 * O.kernel_W(kind, 0.0, h)


def test_cubic_spline_is_twice_continuously_differentiable_at_q1():
    """The M4 spline's two pieces join with equal W, F and dF/dr at q = 1,
    and W(0) : W(h) : W(1.5h) = 1 : 1/4 : 1/32 (its piecewise cubic shape)."""
    h = 0.2
    e = 1e-12
    for f in (O.kernel_W, O.kernel_F, O.kernel_dF):
        a, b = f(O.CUBIC_SPLINE, (1 - e) * h, h), f(O.CUBIC_SPLINE, (1 + e) * h, h)
        assert abs(a - b) <= 1e-9 * abs(a)
    W0 = O.kernel_W(O.CUBIC_SPLINE, 0.0, h)
    assert abs(O.kernel_W(O.CUBIC_SPLINE, h, h) / W0 - 0.25) < 1e-14
    assert abs(O.kernel_W(O.CUBIC_SPLINE, 1.5 * h, h) / W0 - 1.0 / 32.0) < 1e-14


def test_gaussian_is_the_truncated_exponential():
    """W(q) proportional to exp(-q^2) - exp(-4) (the d-truncated Gaussian of
    the listing with d = 2h), and F(r) = -(2/h^2) C exp(-q^2), with
    C = W(0) / (1 - exp(-4)): its F does not vanish at the edge."""
    h = 0.3
    W0 = O.kernel_W(O.GAUSSIAN, 0.0, h)
    C = W0 / (1.0 - math.exp(-4.0))
    for q in (0.3, 1.0, 1.6, 1.999):
        assert abs(O.kernel_W(O.GAUSSIAN, q * h, h) - C * (math.exp(-q * q) - math.exp(-4.0))) < 1e-13 * W0
        assert abs(O.kernel_F(O.GAUSSIAN, q * h, h) + 2.0 * C * math.exp(-q * q) / h ** 2) < 1e-13 * C / h ** 2


def test_quadratic_kernel_is_a_parabola_with_a_flat_edge():
    """W is a quadratic in q that vanishes with zero slope at q = 2 (so it is
    c (2 - q)^2): W(q)/W(0) = (1 - q/2)^2."""
    h = 0.7
    W0 = O.kernel_W(O.QUADRATIC, 0.0, h)
    for q in (0.1, 0.8, 1.5, 1.9):
        assert abs(O.kernel_W(O.QUADRATIC, q * h, h) / W0 - (1.0 - 0.5 * q) ** 2) < 1e-14


def _lattice_vectors(R):
    m = int(math.ceil(R)) + 1
    r = np.arange(-m, m + 1)
    a, b, c = np.meshgrid(r, r, r, indexing="ij")
    v = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
    s = (v * v).sum(axis=1)
    return v[(s > 0) & (s < R * R)]


@pytest.mark.parametrize("kind", KINDS)
def test_kernel_gradient_lattice_moment(kind):
    """sum_j dp^3 x_z^2 F over a cubic lattice at h = 1.3 dp approximates the
    continuum -1 (integration by parts of a unit-integral kernel) to the
    kernel's lattice error; the odd moments vanish by symmetry."""
    dp = 0.02
    h = 1.3 * dp
    v = _lattice_vectors(2.6) * dp
    r = np.linalg.norm(v, axis=1)
    F = np.array([O.kernel_F(kind, x, h) for x in r])
    Mzz = float((dp ** 3 * v[:, 2] ** 2 * F).sum())
    assert -1.06 < Mzz < -0.97, Mzz
    assert np.all(np.abs((dp ** 3 * v * F[:, None]).sum(axis=0)) < 1e-12)


# ------------------------------------------------------------------ lattice scenes
def _lattice(n, dp, **kw):
    """A cubic lattice of n^3 fluid particles, no walls, g = 0; returns the
    built lists, the lifted state (sorted order), positions and the mask of
    particles whose kernel support lies entirely inside the lattice."""
    kw.setdefault("g", (0.0, 0.0, 0.0))
    p = S.sph_params(dp, **kw)
    lo = np.array([0.1, 0.1, 0.1])
    xf = S.lattice(n, n, n, dp, lo=tuple(lo))
    grid = S.make_grid((0, 0, 0), tuple(lo * 2 + n * dp), p.r_search)
    sc = S._assemble("lattice", grid, p, xf, np.zeros((0, 3)), H=0.0)
    b = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info)
    st = O.State.lift(b["cell"], b["pos"], b["vel"], b["info"])
    x = O.positions(sc.grid, st)
    lo_x, hi_x = xf.min(axis=0), xf.max(axis=0)
    margin = 2.0 * O.f32(p.h) + 0.5 * dp
    inner = np.all((x > lo_x + margin) & (x < hi_x - margin), axis=1)
    return sc, b, st, x, inner


def _with(params, **kw):
    q = copy.deepcopy(params)
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def _eos_inverse(P, p):
    """Density with Cole pressure P (test-side inverse of the equation of state)."""
    B = O.f32(p.rho0) * O.f32(p.c0) ** 2 / O.f32(p.gamma)
    return O.f32(p.rho0) * (1.0 + P / B) ** (1.0 / O.f32(p.gamma))


# ------------------------------------------------------------------ Landrini-Morris formulation
def test_landrini_continuity_depends_on_density_only_through_rho_i():
    """With particle volumes m_j/rho_j held fixed, the Landrini-Morris
    continuity rate divided by rho_i is the same for any density field (the
    field enters only through rho_i, eq. mass-cont-sph2); the golden-rule
    rate is not (its weight is m_j)."""
    dp = 0.02
    sc, b, st, x, inner = _lattice(8, dp, alpha=0.0)
    rng = np.random.default_rng(71)
    st.vel = rng.normal(0.0, 0.2, size=(st.n, 3))
    rates = {}
    for form in (0, 1):
        p = _with(sc.params, formulation=form)
        out = []
        for k in range(2):
            s = st.copy()
            s.rho = 1000.0 * (1.0 + 0.2 * rng.uniform(-1, 1, size=st.n))
            s.mass = s.rho * dp ** 3
            acc, drho, sa, sd, ni = O.forces(sc.grid, p, s, b["lists"])
            out.append((drho / s.rho, sd / s.rho))
        rates[form] = out
    (r1, s1), (r2, s2) = rates[1]
    assert np.all(np.abs(r1 - r2) <= 1e-13 * np.maximum(s1, s2))
    (g1, t1), (g2, t2) = rates[0]
    assert np.max(np.abs(g1 - g2) / np.maximum(t1, t2)) > 1e-2


def test_landrini_continuity_is_minus_rho_div_u_for_a_linear_field():
    """u = eps (x - c) on a lattice with a rough density field and volumes
    dp^3: Drho_i/Dt = rho_i eps tr(M) for every interior particle, where M is
    the lattice moment of the kernel gradient (-> -rho_i div u = -3 eps rho_i)."""
    dp = 0.02
    sc, b, st, x, inner = _lattice(11, dp, alpha=0.0, formulation=1)
    eps = 0.37
    c = x.mean(axis=0)
    st.vel = eps * (x - c)
    rng = np.random.default_rng(72)
    st.rho = 1000.0 * (1.0 + 0.2 * rng.uniform(-1, 1, size=st.n))
    st.mass = st.rho * dp ** 3
    acc, drho, sa, sd, ni = O.forces(sc.grid, sc.params, st, b["lists"])
    assert inner.sum() >= 27
    ratio = drho[inner] / (-3.0 * eps * st.rho[inner])
    # one lattice constant for all (the float32 encoding moves the lattice by ~1e-8)
    assert np.all(np.abs(ratio - ratio[0]) < 1e-7)
    assert abs(ratio[0] - 0.9789) < 1e-3  # the Wendland lattice moment, 2% from the continuum


def test_landrini_momentum_is_linear_in_pressure_at_fixed_volumes():
    """With volumes m_j/rho_j held fixed, rho_i a_i of the Landrini-Morris
    form is linear in the pressure field (eq. ns-sph2 weights P_i + P_j by
    the volume only): pressure fields P1, P2 and P1 + P2, each realised
    through the equation of state, give rho3 a3 = rho1 a1 + rho2 a2 for every
    particle, interior or not.  The golden rule breaks this."""
    dp = 0.02
    sc, b, st, x, inner = _lattice(8, dp, alpha=0.0)
    B = O.f32(sc.params.rho0) * O.f32(sc.params.c0) ** 2 / 7.0
    rng = np.random.default_rng(73)
    P1 = B * rng.uniform(0.0, 1.0, size=st.n)
    P2 = B * rng.uniform(0.0, 1.0, size=st.n)

    def rho_a(P, form):
        s = st.copy()
        s.rho = _eos_inverse(P, sc.params)
        s.mass = s.rho * dp ** 3
        acc, drho, sa, sd, ni = O.forces(sc.grid, _with(sc.params, formulation=form), s, b["lists"])
        return s.rho[:, None] * acc, s.rho[:, None] * sa

    a1, s1 = rho_a(P1, 1)
    a2, s2 = rho_a(P2, 1)
    a3, s3 = rho_a(P1 + P2, 1)
    assert np.all(np.abs(a3 - a1 - a2) <= 1e-12 * (s1 + s2 + s3))
    g1, t1 = rho_a(P1, 0)
    g2, t2 = rho_a(P2, 0)
    g3, t3 = rho_a(P1 + P2, 0)
    assert np.max(np.abs(g3 - g1 - g2) / (t1 + t2 + t3)) > 1e-3


def test_landrini_momentum_for_a_linear_pressure_field():
    """P = P0 + G.(x - c) realised through the equation of state (so the
    density varies by several percent), volumes dp^3: every interior particle
    gets a_i = M G / rho_i with M the lattice moment (-> -grad P / rho)."""
    dp = 0.02
    sc, b, st, x, inner = _lattice(11, dp, alpha=0.0, formulation=1, c0=5.0)
    B = O.f32(sc.params.rho0) * O.f32(sc.params.c0) ** 2 / 7.0
    G = np.array([0.3, -0.2, 0.45]) * B / (11 * dp)
    c = x.mean(axis=0)
    P = 0.8 * B + (x - c) @ G
    st.rho = _eos_inverse(P, sc.params)
    assert st.rho.max() / st.rho.min() > 1.05
    st.mass = st.rho * dp ** 3
    acc, drho, sa, sd, ni = O.forces(sc.grid, sc.params, st, b["lists"])
    expect = -0.978896 * G[None, :] / st.rho[inner][:, None]
    # the float32 encoding moves the lattice by ~1e-8 relative, which the
    # cancelling 2 P_i sum_j V_j x_ij F_ij (P_i ~ 0.8 B) turns into ~1e-6 of the result
    assert np.all(np.abs(acc[inner] - expect) <= 1e-5 * np.abs(expect).max())


def test_landrini_equals_golden_rule_at_uniform_density():
    """At uniform density (P_i + P_j)/(rho_i rho_j) = P_i/rho_i^2 + P_j/rho_j^2
    and rho_i/rho_j = 1: the two formulations coincide, viscosity, laminar
    term and all."""
    sc = S.random_cloud(n=900, box=(0.2, 0.2, 0.2), dp=0.02, seed=74, boundary_frac=0.25, u_sigma=0.3,
                        rho_sigma=0.0, alpha=0.2, visc_model=1, nu=1e-3)
    sc.vel[:, 3] = np.float32(1012.0)
    b = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info)
    st = O.State.lift(b["cell"], b["pos"], b["vel"], b["info"])
    a0, d0, sa0, sd0, _ = O.forces(sc.grid, sc.params, st, b["lists"])
    a1, d1, sa1, sd1, _ = O.forces(sc.grid, _with(sc.params, formulation=1), st, b["lists"])
    assert np.all(np.abs(a1 - a0) <= 1e-14 * sa0) and np.all(np.abs(d1 - d0) <= 1e-14 * sd0)
    assert np.abs(a0).max() > 0 and np.abs(d0).max() > 0


# ------------------------------------------------------------------ Monaghan K form
@pytest.mark.parametrize("kind,tol", [(O.GAUSSIAN, 0.09), (O.WENDLAND, 0.15)])
@pytest.mark.parametrize("flow", ["shear", "compressive"])
def test_laminar_forms_on_quadratic_flows(kind, tol, flow):
    """Interior particles of a uniform lattice under u_x = s y^2 (divergence
    free: nu lap u = 2 nu s) and u_x = s x^2 (lap u + 2 grad div u = 6 s):
    Morris gives nu lap u for both, Monaghan's K form
    nu (lap u + 2 grad div u) with K = d + 2 = 5, to the kernel's lattice
    error at h = 1.3 dp (up to 8% for the Gaussian, 13% for Wendland; a
    wrong K or the Morris form in its place is off by a factor 2 or 3)."""
    dp = 0.02
    nu = 1e-3
    s = 3.0
    out = {}
    for visc in (1, 2):
        sc, b, st, x, inner = _lattice(11, dp, alpha=0.0, visc_model=visc, nu=nu, kernel=kind, eps_visc=1e-8)
        c = x.mean(axis=0)
        st.vel = np.zeros((st.n, 3))
        axis = 1 if flow == "shear" else 0
        st.vel[:, 0] = s * (x[:, axis] - c[axis]) ** 2
        st.rho[:] = 1000.0
        st.mass[:] = 1000.0 * dp ** 3
        acc, *_ = O.forces(sc.grid, sc.params, st, b["lists"])
        out[visc] = acc[inner]
        assert np.all(np.abs(acc[inner, 1:]) < 1e-6 * nu * s)  # zero up to the float32 encoding
    assert np.all(np.abs(out[1][:, 0] / (2 * nu * s) - 1.0) < tol)
    want = 2 * nu * s if flow == "shear" else 6 * nu * s
    assert np.all(np.abs(out[2][:, 0] / want - 1.0) < tol), out[2][:3, 0] / want


def test_monaghan_k_form_is_central_and_ignores_rigid_rotation():
    """Monaghan's K form acts along x_ij and is proportional to u_ij . x_ij:
    it conserves angular momentum for any configuration, and gives nothing
    for a rigid rotation (u_ij . x_ij = 0 for every pair)."""
    sc = S.random_cloud(n=900, box=(0.2, 0.2, 0.2), dp=0.02, seed=75, boundary_frac=0.2, u_sigma=0.3,
                        rho_sigma=0.01, alpha=0.0, visc_model=2, nu=1e-2)
    b = O.build_f32(sc.grid, sc.params, sc.cell, sc.pos, sc.vel, sc.info)
    st = O.State.lift(b["cell"], b["pos"], b["vel"], b["info"])
    x = O.positions(sc.grid, st)
    p0 = _with(sc.params, visc_model=0)
    a2, _, sa2, _, _ = O.forces(sc.grid, sc.params, st, b["lists"])
    a0, *_ = O.forces(sc.grid, p0, st, b["lists"])
    lam = a2 - a0
    L = (st.mass[:, None] * np.cross(x, lam)).sum(axis=0)
    scale = (st.mass * np.linalg.norm(x, axis=1) * np.linalg.norm(sa2, axis=1)).sum()
    assert np.all(np.abs(L) <= 1e-13 * scale) and np.abs(lam).max() > 0
    w = np.array([0.4, -1.1, 0.7])
    st.vel = np.cross(w[None, :], x - x.mean(axis=0))
    a2, _, sa2, _, _ = O.forces(sc.grid, sc.params, st, b["lists"])
    a0, *_ = O.forces(sc.grid, p0, st, b["lists"])
    assert np.all(np.abs(a2 - a0) <= 1e-13 * sa2)
