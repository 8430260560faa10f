"""Pins for the oracle's right-hand side and RK4: free-stream preservation,
discrete conservation, design-order convergence to exact time derivatives
(an Euler entropy wave and pure heat conduction), the closed-form initial
kinetic-energy decay of the Taylor-Green vortex, axis-permutation symmetry,
one-dimensional reduction and the equivalence of the reference-state form
with the textbook form (checked against extended precision)."""

import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.rhs import Params, rhs, rk4_step
from paper_2401_06132_amd import inputs

G = 1.4


def _fields(m, fn):
    return {t: np.ascontiguousarray(np.moveaxis(fn(m.upts_coords(t)), -1, 1)) for t in m.types}


def _integral(m, U):
    return sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, U[t]) for t in m.types)


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
@pytest.mark.parametrize("p", [2, 3])
def test_free_stream_preservation(kind, p):
    m = Mesh(2, 2, 2, p, kind)
    U = {t: u for t, u in zip(m.types, inputs.uniform_state([(m.nelem[t], m.refs[t].nu) for t in m.types]))}
    for pref in (0.0, inputs.P0):
        du = rhs(m, U, Params(pref=pref))
        # flux magnitude ~ p0 + rho v^2 ~ 72; the RHS must vanish to rounding
        assert max(np.abs(du[t]).max() for t in m.types) < 1e-12 * 72 * 10


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
def test_discrete_conservation(kind):
    m = Mesh(2, 3, 2, 3, kind)
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
    du = rhs(m, U, Params(pref=inputs.P0))
    tot = _integral(m, du)
    scale = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, np.abs(du[t])) for t in m.types)
    assert np.all(np.abs(tot) <= 1e-13 * scale)


def _entropy_wave(x, a=0.5, p=1.0):
    s = x[..., 0] + x[..., 1] + x[..., 2]
    rho = 1 + 0.2 * np.sin(s)
    E = p / (G - 1) + 0.5 * rho * 3 * a * a
    u = np.stack([rho, rho * a, rho * a, rho * a, E], -1)
    drho = -3 * a * 0.2 * np.cos(s)
    du = np.stack([drho, a * drho, a * drho, a * drho, 1.5 * a * a * drho], -1)
    return u, du


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
@pytest.mark.parametrize("p", [2, 3])
def test_entropy_wave_convergence(kind, p):
    """Euler (mu = 0): rho = 1 + 0.2 sin(x+y+z), uniform v and p is an exact
    solution; the RHS error must fall at about the design rate."""
    errs = []
    for N in (4, 8):
        m = Mesh(N, N, N, p, kind)
        U = _fields(m, lambda x: _entropy_wave(x)[0])
        ex = _fields(m, lambda x: _entropy_wave(x)[1])
        du = rhs(m, U, Params(mu=0.0, tau=0.0))
        errs.append(max(np.abs(du[t] - ex[t]).max() for t in m.types))
    assert np.log2(errs[0] / errs[1]) > p - 0.3


def test_heat_conduction_convergence():
    """v = 0, uniform p, rho = 1 + 0.2 sin x: only the heat flux acts,
    dE/dt = mu gamma p / (Pr (gamma-1)) d2(1/rho)/dx2."""
    mu, Pr = 0.05, 0.71

    def fld(x):
        s = x[..., 0]
        rho = 1 + 0.2 * np.sin(s)
        z = np.zeros_like(s)
        u = np.stack([rho, z, z, z, np.full_like(s, 1.0 / (G - 1))], -1)
        lap = 2 * (0.2 * np.cos(s)) ** 2 / rho ** 3 + 0.2 * np.sin(s) / rho ** 2
        return u, np.stack([z, z, z, z, mu * G / (Pr * (G - 1)) * lap], -1)

    errs = []
    for N in (4, 8, 16):
        m = Mesh(N, 2, 2, 3, "hex")
        du = rhs(m, _fields(m, lambda x: fld(x)[0]), Params(mu=mu, prandtl=Pr))
        ex = _fields(m, lambda x: fld(x)[1])
        errs.append(max(np.abs(du[t] - ex[t]).max() for t in m.types))
    assert errs[2] < 2e-3 * 0.05 / 0.05 and np.log2(errs[1] / errs[2]) > 1.5


@pytest.mark.parametrize("kind,tol", [("hex", 1e-3), ("prism", 1e-2)])
def test_tgv_initial_kinetic_energy_decay(kind, tol):
    """d/dt int rho|v|^2/2 at t=0 equals -mu int |omega|^2 = -mu (3/4)(2 pi)^3
    for the divergence-free Taylor-Green field."""
    m = Mesh(8, 8, 8, 3, kind)
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types], noise_amp=0))}
    du = rhs(m, U, Params(pref=inputs.P0))
    dke = 0.0
    for t in m.types:
        r = m.refs[t]
        # evaluate the integrand of the discrete fields at the quadrature points
        u = np.einsum("qu,evu->evq", r.M7, U[t])
        d = np.einsum("qu,evu->evq", r.M7, du[t])
        v = u[:, 1:4] / u[:, 0:1]
        dk = np.einsum("eiq,eiq->eq", v, d[:, 1:4]) - 0.5 * np.einsum("eiq,eiq->eq", v, v) * d[:, 0]
        dke += np.einsum("e,q,eq->", m.detJ[t], r.qwts, dk)
    exact = -(1.0 / 1600.0) * 0.75 * (2 * np.pi) ** 3
    assert abs(dke / exact - 1) < tol


def test_axis_permutation_symmetry():
    """Swapping x and y in the state (and the x/y momenta) swaps them in the
    RHS.  The L/R rule is symmetric under the swap on the periodic box."""
    rng = np.random.default_rng(5)
    k = rng.standard_normal((5, 3))

    def f(x):
        out = []
        for c in range(5):
            out.append(0.05 * np.sin(k[c, 0] * 0 + x[..., 0] + 2 * x[..., 1]) * np.cos(x[..., 2] + c)
                       + 0.03 * np.cos(x[..., 0] - x[..., 1] + c))
        u = np.stack(out, -1)
        u[..., 0] += 1.0
        u[..., 4] += 2.5
        return u

    def fswap(x):
        xs = x[..., [1, 0, 2]]
        u = f(xs)
        return u[..., [0, 2, 1, 3, 4]]

    m = Mesh(3, 3, 2, 2, "hex")
    par = Params(mu=0.01)
    d1 = rhs(m, _fields(m, f), par)["hex"]
    d2 = rhs(m, _fields(m, fswap), par)["hex"]
    X = m.upts_coords("hex").reshape(-1, 3)
    key = {tuple(np.round(x, 9)): i for i, x in enumerate(X)}
    idx = np.array([key[tuple(np.round(x[[1, 0, 2]], 9))] for x in X])
    D1 = d1.transpose(0, 2, 1).reshape(-1, 5)
    D2 = d2.transpose(0, 2, 1).reshape(-1, 5)
    np.testing.assert_allclose(D2, D1[idx][:, [0, 2, 1, 3, 4]], atol=1e-12 * np.abs(D1).max())


def test_one_dimensional_reduction():
    """A state that depends on x only, with v_y = v_z = 0.  The mass,
    x-momentum and energy RHS must be exactly independent of y and z.  The
    y/z momenta carry only the lifted difference between the collocated face
    flux f(u^f) and the face trace of the projected flux (flux anti-aliasing
    projects the volume flux but not the interface flux); that defect is a
    projection error and must fall at least at rate p + 1."""
    def f(x):
        s = x[..., 0]
        rho = 1 + 0.1 * np.sin(s)
        vx = 0.3 * np.cos(s)
        p = 2 + 0.1 * np.sin(2 * s)
        z = np.zeros_like(s)
        return np.stack([rho, rho * vx, z, z, p / (G - 1) + 0.5 * rho * vx * vx], -1)

    cross = []
    for N in (4, 8):
        m = Mesh(N, 3, 2, 3, "hex")
        du = rhs(m, _fields(m, f), Params(mu=0.01))["hex"]
        X = m.upts_coords("hex")[..., 0].reshape(-1)
        D = du.transpose(0, 2, 1).reshape(-1, 5)
        for xv in np.unique(np.round(X, 10)):
            sel = np.abs(X - xv) < 1e-9
            assert np.ptp(D[sel][:, [0, 1, 4]], axis=0).max() < 1e-12
        cross.append(np.abs(du[:, 2:4]).max())
    assert cross[0] < 1e-3 and np.log2(cross[0] / cross[1]) > 4.0


@pytest.mark.parametrize("kind", ["hex", "prism"])
def test_reference_state_form_is_the_accurate_one(kind):
    """At Mach 0.1 the textbook form carries p0 ~ 71 through the derivative
    operators.  Against an extended-precision evaluation (longdouble
    arithmetic; both forms are the same function), the float64
    reference-state form is accurate to < 5e-13 relative per variable while
    the float64 textbook form is several times worse.  (What single precision
    reaches is measured with the kernels' own split in test_fp32_split.py.)"""
    m = Mesh(2, 2, 2, 2, kind)
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
    ref = rhs(m, {t: U[t].astype(np.longdouble) for t in m.types}, Params(pref=inputs.P0), dtype=np.longdouble)
    good = rhs(m, U, Params(pref=inputs.P0))
    plain = rhs(m, U, Params(pref=0.0))
    eg, ep = [], []
    for t in m.types:
        sc = np.abs(ref[t]).max(axis=(0, 2))
        eg.append((np.abs(good[t] - ref[t]).max(axis=(0, 2)) / sc).astype(np.float64))
        ep.append((np.abs(plain[t] - ref[t]).max(axis=(0, 2)) / sc).astype(np.float64))
    eg, ep = np.max(eg), np.max(ep)
    assert eg < 5e-13
    assert ep > 3 * eg


def test_rk4_fourth_order_in_time():
    m = Mesh(2, 2, 2, 2, "hex")
    U0 = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types], noise_amp=0))}
    par = Params(pref=inputs.P0)
    T = 0.02

    def run(nsteps):
        U = U0
        for _ in range(nsteps):
            U = rk4_step(m, U, par, T / nsteps)
        return U["hex"]

    ref = run(32)
    e1 = np.abs(run(4) - ref).max()
    e2 = np.abs(run(8) - ref).max()
    assert 12 < e1 / e2 < 20
    # conserved integrals are preserved by the step
    c0, c1 = _integral(m, U0), _integral(m, {"hex": ref})
    assert np.all(np.abs(c1 - c0) <= 1e-13 * np.abs(c0).max())


# ---- the AA-off configuration (flux evaluated at the solution points) ----

@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
def test_aa_off_free_stream_and_conservation(kind):
    m = Mesh(2, 3, 2, 3, kind)
    U = {t: u for t, u in zip(m.types, inputs.uniform_state([(m.nelem[t], m.refs[t].nu) for t in m.types]))}
    du = rhs(m, U, Params(pref=inputs.P0, aa=False))
    assert max(np.abs(du[t]).max() for t in m.types) < 1e-12 * 72 * 10
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
    du = rhs(m, U, Params(pref=inputs.P0, aa=False))
    tot = _integral(m, du)
    scale = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, np.abs(du[t])) for t in m.types)
    assert np.all(np.abs(tot) <= 1e-13 * scale)


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
@pytest.mark.parametrize("p", [2, 3])
def test_aa_off_equals_aa_for_polynomial_flux(kind, p):
    """Inviscid, uniform velocity and pressure, density a polynomial of
    degree p on each element: the flux is then itself of degree p, so
    interpolating it to the quadrature points and projecting back is exact
    and the anti-aliased RHS equals the one with the flux at the solution
    points.  (A plausible slip in either path -- a missing metric factor, a
    transposed operator -- breaks the equality.)"""
    m = Mesh(2, 2, 3, p, kind)
    rng = np.random.default_rng(3)
    U = {}
    for t in m.types:
        x = m.upts_coords(t)
        # per element: rho = c0 + c . (x - centre), degree 1 <= p, plus a
        # per-element product term of degree 2 <= p
        cen = x.mean(axis=1, keepdims=True)
        d = x - cen
        c = rng.uniform(-0.1, 0.1, size=(x.shape[0], 1, 3))
        rho = 1.0 + (c * d).sum(-1) + 0.05 * d[..., 0] * d[..., 2]
        v = np.array([0.3, -0.2, 0.1])
        pr = inputs.P0
        E = pr / (G - 1) + 0.5 * rho * float(v @ v)
        U[t] = np.ascontiguousarray(np.stack([rho, rho * v[0], rho * v[1], rho * v[2], E], 1))
    a = rhs(m, U, Params(mu=0.0, pref=inputs.P0, aa=True))
    b = rhs(m, U, Params(mu=0.0, pref=inputs.P0, aa=False))
    for t in m.types:
        sc = np.abs(a[t]).max()
        assert sc > 1e-3
        assert np.abs(a[t] - b[t]).max() <= 1e-11 * sc, (t, np.abs(a[t] - b[t]).max() / sc)


@pytest.mark.parametrize("kind", ["hex", "prism"])
def test_aa_off_entropy_wave_convergence(kind):
    """Design order without anti-aliasing: the entropy wave's exact time
    derivative is approached at rate >= p (p = 3)."""
    errs = []
    for n in (2, 4):
        m = Mesh(n, n, n, 3, kind, lo=-np.pi, hi=np.pi)
        U, dU = {}, {}
        for t in m.types:
            u, du = _entropy_wave(m.upts_coords(t))
            U[t] = np.ascontiguousarray(np.moveaxis(u, -1, 1))
            dU[t] = np.moveaxis(du, -1, 1)
        got = rhs(m, U, Params(mu=0.0, aa=False))
        errs.append(max(np.abs(got[t] - dU[t]).max() for t in m.types))
    rate = np.log2(errs[0] / errs[1])
    assert rate > 3.0, (errs, rate)
