"""Pins for the oracle's pyramids: the conical-product rule against the
closed-form pyramid moments, the node set (count, interior, invariance under
the square's symmetries, unisolvence), the solution space (its gradients
against finite differences, the rational members that define it, polynomial
traces on the faces), the weak-form divergence taken for pyramids, and the
right-hand side on pyramid and hexahedron/pyramid meshes (free stream,
discrete conservation, entropy-wave convergence).  The generic operator
identities are pinned for pyramids in test_oracle_operators.py."""

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import basis, quadrature
from oracle.elements import RefElement
from oracle.mesh import Mesh
from oracle.rhs import Params, rhs
from paper_2401_06132_amd import inputs
from test_oracle_tet import _entropy_wave


def _pyramid_monomial(a, b, c):
    """int over the reference pyramid of xi^a eta^b zeta^c, exactly.  The
    section at height zeta is the square of half width s = (1 - zeta)/2, on
    which xi^a eta^b integrates to (2/(a+1)) (2/(b+1)) s^(a+b+2) for even a, b
    (zero otherwise); with zeta = 1 - 2s,
    int_{-1}^{1} s^(a+b+2) zeta^c dzeta = 2 sum_j C(c, j) (-2)^j / (a+b+3+j)."""
    if a % 2 or b % 2:
        return Fraction(0)
    sq = Fraction(2, a + 1) * Fraction(2, b + 1)
    z = sum(Fraction(math.comb(c, j) * (-2) ** j, a + b + 3 + j) for j in range(c + 1))
    return sq * 2 * z


def test_pyramid_volume_closed_form():
    assert _pyramid_monomial(0, 0, 0) == Fraction(8, 3)  # base 4, height 2


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_pyramid_rule_exact_to_degree_2k_minus_1(k):
    x, w = quadrature.pyramid_conical(k)
    assert len(w) == k ** 3 and np.all(w > 0)
    s = (1 - x[:, 2]) / 2
    assert np.all(np.abs(x[:, 0]) < s) and np.all(np.abs(x[:, 1]) < s) and np.all(np.abs(x[:, 2]) < 1)
    for a in range(2 * k):
        for b in range(2 * k - a):
            for c in range(2 * k - a - b):
                want = float(_pyramid_monomial(a, b, c))
                got = np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c)
                assert abs(got - want) < 1e-13 * max(1.0, abs(want)), (a, b, c)
    assert abs(np.sum(w * x[:, 2] ** (2 * k)) - float(_pyramid_monomial(0, 0, 2 * k))) > 1e-10


def _d4(x):
    """The eight images of points under the square's symmetry group."""
    out = []
    for sw in (False, True):
        y = x[:, [1, 0, 2]] if sw else x
        for sx in (1, -1):
            for sy in (1, -1):
                out.append(y * np.array([sx, sy, 1]))
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_pyramid_nodes(p):
    x = quadrature.pyramid_nodes(p)
    assert len(x) == (p + 1) * (p + 2) * (2 * p + 3) // 6
    s = (1 - x[:, 2]) / 2
    assert np.all(np.abs(x[:, 0]) < s) and np.all(np.abs(x[:, 1]) < s) and np.all(np.abs(x[:, 2]) < 1)
    base = {tuple(r) for r in np.round(x, 12)}
    for y in _d4(x):
        assert {tuple(r) for r in np.round(y, 12)} == base
    V, _ = basis.eval_basis("pyr", p, x)
    sv = np.linalg.svd(np.asarray(V, float), compute_uv=False)
    assert sv.min() / sv.max() > 1e-3


def _interior_points(n, rng):
    z = rng.uniform(-0.95, 0.9, n)
    s = (1 - z) / 2
    return np.stack([rng.uniform(-0.95, 0.95, n) * s, rng.uniform(-0.95, 0.95, n) * s, z], axis=1)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_pyramid_basis_gradient_and_dimension(p):
    rng = np.random.default_rng(3)
    x = _interior_points(40, rng)
    V, G = basis.eval_basis("pyr", p, x)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (np.asarray(basis.eval_basis("pyr", p, x + e)[0], float) -
              np.asarray(basis.eval_basis("pyr", p, x - e)[0], float)) / (2 * h)
        np.testing.assert_allclose(np.asarray(G[d], float), fd, atol=1e-6 * np.abs(fd).max())
    # the modes are linearly independent: rank = dimension of the space
    y = _interior_points(400, rng)
    Vy = np.asarray(basis.eval_basis("pyr", p, y)[0], float)
    assert np.linalg.matrix_rank(Vy, tol=1e-9 * np.abs(Vy).max()) == (p + 1) * (p + 2) * (2 * p + 3) // 6


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_pyramid_space_members(p):
    """The space holds the rational functions xi^i eta^j s^(max(i,j) - i - j),
    s = (1 - zeta)/2, i, j <= p, and P_p: the nodal interpolant reproduces
    each of them at arbitrary points."""
    r = RefElement("pyr", p)
    rng = np.random.default_rng(5)
    y = _interior_points(60, rng)
    L, DL = basis.nodal("pyr", p, r.upts, y)
    L, DL = np.asarray(L, float), np.asarray(DL, float)

    def rat(x, i, j):
        s = (1 - x[:, 2]) / 2
        return x[:, 0] ** i * x[:, 1] ** j * s ** (max(i, j) - i - j)

    for i in range(p + 1):
        for j in range(p + 1):
            f = rat(r.upts, i, j)
            assert np.abs(L @ f - rat(y, i, j)).max() < 1e-12, (i, j)
    for a in range(p + 1):
        for b in range(p + 1 - a):
            for c in range(p + 1 - a - b):
                def f(x):
                    return x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c
                assert np.abs(L @ f(r.upts) - f(y)).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_pyramid_traces_are_face_polynomials(p):
    """Trace of any member of the space: Q_p on the base and P_p on every
    triangle, so the face's own nodal values determine it (conforming with
    hexahedron and tetrahedron faces)."""
    r = RefElement("pyr", p)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(r.nu)
    # base: the GL(n)^2 tensor interpolant of the base flux-point values
    st = rng.uniform(-1, 1, (30, 2))
    yb = np.stack([st[:, 0], st[:, 1], -np.ones(30)], axis=1)
    Lb = np.asarray(basis.nodal("pyr", p, r.upts, yb)[0], float)
    fb = np.asarray(r.M0, float)[r.fface == 0] @ u  # values at the base points, index a + n b
    lx = np.asarray(basis.line_nodal(r.gl, st[:, 0]), float)
    ly = np.asarray(basis.line_nodal(r.gl, st[:, 1]), float)
    n = p + 1
    tensor = np.einsum("qa,qb,ba->q", lx, ly, fb.reshape(n, n))
    assert np.abs(Lb @ u - tensor).max() < 1e-11 * np.abs(u).max()
    # triangles: the P_p interpolant of the face's triangle-node values
    tq = rng.uniform(-1, 1, (60, 2))
    tq = tq[tq.sum(axis=1) <= 0][:20]
    Lt = np.asarray(basis.tri_nodal(p, r.tri_nodes, tq), float)
    for f in range(1, 5):
        yf = r.faces[f]["map"](tq[:, 0], tq[:, 1])
        Lf = np.asarray(basis.nodal("pyr", p, r.upts, yf)[0], float)
        ff = np.asarray(r.M0, float)[r.fface == f] @ u
        assert np.abs(Lf @ u - Lt @ ff).max() < 1e-11 * np.abs(u).max()


def test_pyramid_space_not_closed_under_differentiation():
    """The premise of the weak-form reading: d/dxi of a member can leave the
    space (here 4 xi eta/(1-zeta) -> 2 eta/(1-zeta)), so the collocated strong
    divergence differs from the weak form on pyramids."""
    p = 1
    r = RefElement("pyr", p)
    rng = np.random.default_rng(9)
    y = _interior_points(30, rng)
    L = np.asarray(basis.nodal("pyr", p, r.upts, y)[0], float)

    def g(x):
        return 2 * x[:, 1] / (1 - x[:, 2])
    assert np.abs(L @ g(r.upts) - g(y)).max() > 1e-2


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_pyramid_weak_divergence(p):
    """Kq (with anti-aliasing) and Ku (without) plus the lifting of the normal
    flux give the exact derivative at the solution points for every flux
    F in P_p (integration by parts, exact quadrature), and are conservative:
    w_u^T Kq_d = 0."""
    r = RefElement("pyr", p)
    rng = np.random.default_rng(11)
    terms = [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]
    coef = rng.standard_normal(len(terms))

    def F(x):
        return sum(cf * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for cf, (a, b, c) in zip(coef, terms))

    def dF(x, d):
        out = np.zeros(len(x))
        for cf, e in zip(coef, terms):
            if e[d]:
                ee = list(e)
                ee[d] -= 1
                out += cf * e[d] * x[:, 0] ** ee[0] * x[:, 1] ** ee[1] * x[:, 2] ** ee[2]
        return out

    M3 = np.asarray(r.M3, float)
    for d in range(3):
        lift = M3 @ (r.fnorm[:, d] * F(r.fpts))
        want = dF(r.upts, d)
        sc = np.abs(want).max() + np.abs(F(r.upts)).max()
        assert np.abs(np.asarray(r.Kq[d], float) @ F(r.qpts) + lift - want).max() < 1e-11 * sc
        assert np.abs(np.asarray(r.Ku[d], float) @ F(r.upts) + lift - want).max() < 1e-11 * sc
        assert np.abs(np.asarray(r.wu @ r.Kq[d], float)).max() < 1e-14 * np.abs(np.asarray(r.Kq[d], float)).max()


@pytest.mark.parametrize("kind", ["pyr", "hex_pyr", "hex_pyr_tet", "hex_prism_pyr_tet"])
@pytest.mark.parametrize("p", [1, 3])
def test_free_stream_and_conservation(kind, p):
    m = Mesh(2, 2, 3, p, kind)
    U = {t: u for t, u in zip(m.types, inputs.uniform_state([(m.nelem[t], m.refs[t].nu) for t in m.types]))}
    for pref in (0.0, inputs.P0):
        for aa in (True, False):
            du = rhs(m, U, Params(pref=pref, aa=aa))
            assert max(np.abs(du[t]).max() for t in m.types) < 1e-12 * 72 * 10
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
    for aa in (True, False):
        du = rhs(m, U, Params(pref=inputs.P0, aa=aa))
        tot = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, du[t]) for t in m.types)
        scale = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, np.abs(du[t])) for t in m.types)
        assert np.all(np.abs(tot) <= 1e-13 * scale)


def test_transition_cells():
    """hex_pyr_tet: the element counts of the layering (hexahedra below, one
    pyramid and ten tetrahedra per transition cell, six tetrahedra per Kuhn
    cell), every element of positive volume and the cells filled exactly."""
    nx, ny, nz = 2, 3, 5
    m = Mesh(nx, ny, nz, 1, "hex_pyr_tet")
    kh = nz // 2
    cells = nx * ny
    assert m.nelem["hex"] == cells * kh
    assert m.nelem["pyr"] == cells * 2
    assert m.nelem["tet"] == cells * (2 * 10 + 6 * (nz - kh - 2))
    vol = {"hex": 8.0, "tet": 4.0 / 3.0, "pyr": 8.0 / 3.0}
    total = sum(vol[t] * m.detJ[t].sum() for t in m.types)
    assert np.all(np.concatenate([m.detJ[t] for t in m.types]) > 0)
    assert abs(total - (2 * np.pi) ** 3) < 1e-10
    with pytest.raises(ValueError):
        Mesh(2, 2, 2, 1, "hex_pyr_tet")


@pytest.mark.parametrize("kind,sizes", [("pyr", (2, 4)), ("hex_pyr", (2, 4)), ("hex_pyr_tet", (3, 6)),
                                        ("hex_prism_pyr_tet", (3, 6))])
def test_entropy_wave_convergence(kind, sizes):
    """Euler entropy wave: the RHS error falls at about the design rate."""
    p = 2
    errs = []
    for N in sizes:
        m = Mesh(N, N, N, p, kind)
        U = {t: np.ascontiguousarray(np.moveaxis(_entropy_wave(m.upts_coords(t))[0], -1, 1)) for t in m.types}
        ex = {t: np.ascontiguousarray(np.moveaxis(_entropy_wave(m.upts_coords(t))[1], -1, 1)) for t in m.types}
        du = rhs(m, U, Params(mu=0.0, tau=0.0))
        errs.append(max(np.abs(du[t] - ex[t]).max() for t in m.types))
    assert np.log2(errs[0] / errs[1]) > p - 0.3
