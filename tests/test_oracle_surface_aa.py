"""Pins for the oracle's surface-flux anti-aliasing (flux points replaced by
face quadrature points, section 2.1.1 and table "operatorms").

  * the rebuilt lifting M3 is the DG lifting of the face Lagrange basis
    through the quadrature points, checked against explicit Lagrange
    polynomials integrated with a 16-point rule (hexahedra);
  * M3 applied to samples of a polynomial reproduces the exactly integrated
    lift Mass^-1 int l_u g dS up to the degree the face rule integrates
    (hexahedra and prisms, every face);
  * free-stream preservation and discrete conservation;
  * a state whose interface fluxes are continuous polynomials of degree <= p
    on every face (a shear flow with a piecewise-linear profile) gives the
    same right-hand side with and without surface-flux anti-aliasing;
  * design-order convergence to the exact time derivative of an entropy wave.
"""

import numpy as np
import pytest

from oracle import quadrature
from oracle.elements import RefElement
from oracle.mesh import Mesh
from oracle.rhs import Params, rhs
from paper_2401_06132_amd import inputs


def _lagrange(nodes, x):
    """Values of the Lagrange polynomials through `nodes` at x: (len(x), len(nodes))."""
    nodes = np.asarray(nodes, float)
    x = np.asarray(x, float)
    out = np.ones((len(x), len(nodes)))
    for j, xj in enumerate(nodes):
        for k, xk in enumerate(nodes):
            if k != j:
                out[:, j] *= (x - xk) / (xj - xk)
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_hex_lifting_is_dg_lift_of_quadrature_point_basis(p):
    """M3[u, f] = (1/mass_u) int_face l_u L_f, where L_f is the face Lagrange
    polynomial through the GL(m) x GL(m) quadrature points and the hex mass
    matrix of the GL(n) nodal basis is diag(w_i w_j w_k)."""
    r = RefElement("hex", p, surf_aa=True)
    n, m = p + 1, p + 3
    gl, glw = quadrature.gauss_legendre(n)
    gm, _ = quadrature.gauss_legendre(m)
    x16, w16 = np.polynomial.legendre.leggauss(16)
    Ln = _lagrange(gl, x16)  # solution basis along a line
    Lm = _lagrange(gm, x16)  # face basis along a line
    end = _lagrange(gl, [-1.0, 1.0])  # (2, n)
    M3 = np.asarray(r.M3, float)
    for f in range(6):
        axis, side = f // 2, f % 2
        cols = np.nonzero(r.fface == f)[0]
        assert len(cols) == m * m
        for u in range(n ** 3):
            ijk = (u % n, (u // n) % n, u // (n * n))
            tang = [a for a in range(3) if a != axis]
            # int_{-1}^{1} l_j L_a  for the two tangential directions
            Ia = (w16 * Ln[:, ijk[tang[0]]]) @ Lm
            Ib = (w16 * Ln[:, ijk[tang[1]]]) @ Lm
            mass = glw[ijk[0]] * glw[ijk[1]] * glw[ijk[2]]
            want = end[side, ijk[axis]] * np.outer(Ib, Ia).reshape(-1) / mass  # index a + m b
            np.testing.assert_allclose(M3[u, cols], want, rtol=0, atol=1e-12 * np.abs(want).max())


def _face_exact_lift(r, f, g, npts=14):
    """Mass^-1 int_face(f) l_u g dS_ref with a high-order rule on the face
    (GL x GL on quadrilaterals, collapsed GL x GL on the triangle)."""
    from oracle import basis
    fc = r.faces[f]
    x, w = np.polynomial.legendre.leggauss(npts)
    A, B = np.meshgrid(x, x, indexing="ij")
    WA = np.outer(w, w)
    if fc["kind"] == "quad":
        s, t, ww = A.ravel(), B.ravel(), WA.ravel() * fc["jac"]
        xs = fc["map"](s, t)
        gv = g(s, t)
    else:
        # collapsed square -> triangle: xi = (1+a)(1-b)/2 - 1, eta = b
        xi = 0.5 * (1 + A) * (1 - B) - 1
        eta = B
        ww = (WA * 0.5 * (1 - B)).ravel() * fc["jac"]
        xs = fc["map"](xi.ravel(), eta.ravel())
        gv = g(xi.ravel(), eta.ravel())
    Lv, _ = basis.nodal(r.etype, r.p, r.upts, xs)
    rhs_ = np.asarray(Lv, float).T @ (ww * gv)
    return np.linalg.solve(np.asarray(r.mass, float), rhs_)


@pytest.mark.parametrize("etype", ["hex", "prism"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_lifting_of_polynomials_is_exact_to_rule_degree(etype, p):
    """Quadrilateral faces: GL(m)^2 integrates l_u g exactly for g of degree
    2m - 1 - p per direction; triangles: the (p+1)^2 conical rule is exact to
    total degree 2p + 1, so g of total degree p + 1."""
    r = RefElement(etype, p, surf_aa=True)
    rng = np.random.default_rng(7 + p)
    M3 = np.asarray(r.M3, float)
    m = p + 3
    for f, fc in enumerate(r.faces):
        cols = np.nonzero(r.fface == f)[0]
        if fc["kind"] == "quad":
            deg = 2 * m - 1 - p
            ca, cb = rng.standard_normal(deg + 1), rng.standard_normal(deg + 1)

            def g(s, t, ca=ca, cb=cb):
                return np.polynomial.polynomial.polyval(s, ca) * np.polynomial.polynomial.polyval(t, cb)
            # the face parameters (s, t) of each flux point, recovered from the map
            k = m
            gm, _ = quadrature.gauss_legendre(k)
            s = np.array([gm[a] for b in range(k) for a in range(k)])
            t = np.array([gm[b] for b in range(k) for a in range(k)])
            np.testing.assert_allclose(fc["map"](s, t), r.fpts[cols], atol=1e-14)
        else:
            deg = p + 1
            coef = rng.standard_normal((deg + 1, deg + 1))
            coef[np.add.outer(np.arange(deg + 1), np.arange(deg + 1)) > deg] = 0.0

            def g(xi, eta, coef=coef):
                return np.polynomial.polynomial.polyval2d(xi, eta, coef)
            tq, _ = quadrature.triangle_conical(p + 1)
            s, t = tq[:, 0], tq[:, 1]
            np.testing.assert_allclose(fc["map"](s, t), r.fpts[cols], atol=1e-14)
        got = M3[:, cols] @ g(s, t)
        want = _face_exact_lift(r, f, g)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
def test_free_stream_and_conservation(kind):
    m = Mesh(2, 2, 2, 3, kind, surf_aa=True)
    U = {t: u for t, u in zip(m.types, inputs.uniform_state([(m.nelem[t], m.refs[t].nu) for t in m.types]))}
    du = rhs(m, U, Params(pref=inputs.P0))
    assert max(np.abs(du[t]).max() for t in m.types) < 1e-12 * 72 * 10
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
    for aa in (True, False):
        du = rhs(m, U, Params(pref=inputs.P0, aa=aa))
        tot = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, du[t]) for t in m.types)
        scale = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, np.abs(du[t])) for t in m.types)
        assert np.all(np.abs(tot) <= 1e-13 * scale)


def _shear_state(x, h, lo):
    """rho = 1, p = 1, v = (0, 0.3 tri(x), 0) with tri the piecewise-linear
    wave that is 0 and 1 at alternate element boundaries along x."""
    s = (x[..., 0] - lo) / h
    k = np.floor(s + 1e-12)
    frac = s - k
    tri = np.where(k.astype(int) % 2 == 0, frac, 1.0 - frac)
    vy = 0.3 * tri
    rho = np.ones_like(vy)
    E = 1.0 / 0.4 + 0.5 * vy * vy
    z = np.zeros_like(vy)
    return np.stack([rho, z, rho * vy, z, E], -1)


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
def test_polynomial_interface_flux_is_unchanged(kind):
    """The shear flow is continuous, so the Rusanov and LDG penalty terms
    vanish; every interface flux is a polynomial of degree <= 3 on each face
    (inviscid y-flux cubic in x, the viscous fluxes at most linear), which
    the GL(n)^2 flux points already integrate exactly at p = 3; hence the two
    point sets give the same right-hand side to rounding."""
    p, N = 3, 4
    out = []
    for saa in (False, True):
        m = Mesh(N, 2, 2, p, kind, surf_aa=saa)
        h = (m.hi - m.lo) / N
        U = {t: np.ascontiguousarray(np.moveaxis(_shear_state(m.upts_coords(t), h, m.lo), -1, 1)) for t in m.types}
        out.append(rhs(m, U, Params(mu=0.05)))
    scale = max(np.abs(out[0][t]).max() for t in out[0])
    assert scale > 1e-3
    for t in out[0]:
        np.testing.assert_allclose(out[1][t], out[0][t], rtol=0, atol=1e-11 * scale)


def _entropy_wave(x, a=0.5, p=1.0):
    s = x[..., 0] + x[..., 1] + x[..., 2]
    rho = 1 + 0.2 * np.sin(s)
    E = p / 0.4 + 0.5 * rho * 3 * a * a
    u = np.stack([rho, rho * a, rho * a, rho * a, E], -1)
    drho = -3 * a * 0.2 * np.cos(s)
    du = np.stack([drho, a * drho, a * drho, a * drho, 1.5 * a * a * drho], -1)
    return u, du


@pytest.mark.parametrize("kind", ["hex", "prism"])
def test_entropy_wave_convergence(kind):
    p = 2
    errs = []
    for N in (4, 8):
        m = Mesh(N, N, N, p, kind, surf_aa=True)
        U = {t: np.ascontiguousarray(np.moveaxis(_entropy_wave(m.upts_coords(t))[0], -1, 1)) for t in m.types}
        ex = {t: np.ascontiguousarray(np.moveaxis(_entropy_wave(m.upts_coords(t))[1], -1, 1)) for t in m.types}
        du = rhs(m, U, Params(mu=0.0, tau=0.0))
        errs.append(max(np.abs(du[t] - ex[t]).max() for t in m.types))
    assert np.log2(errs[0] / errs[1]) > p - 0.3
