"""Pins for the oracle's point sets, quadrature rules and operator matrices.

Each check compares against something other than the oracle itself: values
printed in the paper, closed-form integrals, polynomial exactness, the
Radau form of the DG correction functions, and integration-by-parts /
tensor-product identities that a dropped term, a sign slip or a transposed
operand would break.
"""

import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import basis, quadrature
from oracle.elements import RefElement

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_points.txt")


def _golden():
    out = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        out[k] = np.array([float(x) for x in v])
    return out


def test_gauss_legendre_matches_paper_printed_nodes():
    g = _golden()
    for n, key in [(3, "gl3"), (4, "gl4")]:
        x, w = quadrature.gauss_legendre(n)
        np.testing.assert_allclose(x, g[key], atol=1e-15)
        assert abs(w.sum() - 2.0) < 1e-15
    assert abs(g["gl3"][2] - math.sqrt(0.6)) < 1e-16


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_gauss_legendre_exactness(n):
    x, w = quadrature.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    # degree 2n is not integrated exactly
    assert abs(np.dot(w, x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6


def _tri_monomial_integral(a, b):
    # int over {xi,eta >= -1, xi+eta <= 0} of xi^a eta^b; xi = 2x-1, eta = 2y-1
    # on the unit triangle, int x^i y^j = i! j! / (i+j+2)!
    from fractions import Fraction
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = math.comb(a, i) * math.comb(b, j) * 2 ** i * 2 ** j * (-1) ** (a - i + b - j)
            tot += Fraction(c * math.factorial(i) * math.factorial(j), math.factorial(i + j + 2))
    return float(4 * tot)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_conical_triangle_rule_exact_to_degree_2k_minus_1(k):
    pts, w = quadrature.triangle_conical(k)
    assert len(w) == k * k
    assert np.all(pts[:, 0] >= -1) and np.all(pts[:, 1] >= -1) and np.all(pts.sum(1) <= 1e-15)
    for a in range(2 * k):
        for b in range(2 * k - a):
            val = np.dot(w, pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(val - _tri_monomial_integral(a, b)) < 1e-13
    # a degree-2k monomial is missed
    errs = [abs(np.dot(w, pts[:, 0] ** a * pts[:, 1] ** (2 * k - a)) - _tri_monomial_integral(a, 2 * k - a))
            for a in range(2 * k + 1)]
    assert max(errs) > 1e-8


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_triangle_nodes_symmetric_and_unisolvent(p):
    t = quadrature.triangle_nodes(p)
    assert len(t) == (p + 1) * (p + 2) // 2
    assert np.all(t >= -1 - 1e-15) and np.all(t.sum(1) <= 1e-15)
    # barycentric coordinates; the set must be invariant under all six vertex permutations
    lam = np.stack([-(t[:, 0] + t[:, 1]) / 2, (1 + t[:, 0]) / 2, (1 + t[:, 1]) / 2], axis=1)
    import itertools
    key = lambda L: np.round(L, 12)[np.lexsort(np.round(L, 12).T[::-1])]  # noqa: E731
    for perm in itertools.permutations(range(3)):
        np.testing.assert_allclose(key(lam[:, perm]), key(lam), atol=1e-12)
    # strictly interior, and the interpolatory quadrature weights are positive
    assert np.all(lam > 1e-3)
    tq, tw = quadrature.triangle_conical(p + 1)
    w = basis.tri_nodal(p, t, tq).T @ tw
    assert np.all(w > 0) and abs(w.sum() - 2.0) < 1e-13
    # the construction reduces to the equispaced lattice for an equispaced master grid
    V = basis.tri_nodal(p, t, t)
    np.testing.assert_allclose(V, np.eye(len(t)), atol=1e-12)
    if p == 1:
        # GL(2) master grid: v = (1 -+ 1/sqrt 3)/2, vertex-type node (i=1,j=k=0)
        v0, v1 = (1 - 1 / math.sqrt(3)) / 2, (1 + 1 / math.sqrt(3)) / 2
        x = (1 + 2 * v1 - 2 * v0) / 3
        assert np.min(np.linalg.norm(t - np.array([2 * x - 1, 2 * ((1 + 2 * v0 - v1 - v0) / 3) - 1]), axis=1)) < 1e-14


def test_gll_closed_form():
    np.testing.assert_allclose(quadrature.gauss_lobatto_legendre(3), [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(quadrature.gauss_lobatto_legendre(4), [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1],
                               atol=1e-15)
    np.testing.assert_allclose(quadrature.gauss_lobatto_legendre(5), [-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1],
                               atol=1e-15)


def _random_poly(etype, p, rng):
    """A random polynomial of the element's solution space, as monomials."""
    if etype == "hex":
        terms = [(a, b, c) for a in range(p + 1) for b in range(p + 1) for c in range(p + 1)]
    elif etype in ("tet", "pyr"):  # P_p (inside the pyramid space)
        terms = [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]
    else:
        terms = [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1)]
    coef = rng.standard_normal(len(terms))

    def f(x):
        return sum(cf * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for cf, (a, b, c) in zip(coef, terms))

    def grad(x):
        g = np.zeros((3, len(x)))
        for cf, (a, b, c) in zip(coef, terms):
            if a:
                g[0] += cf * a * x[:, 0] ** (a - 1) * x[:, 1] ** b * x[:, 2] ** c
            if b:
                g[1] += cf * b * x[:, 0] ** a * x[:, 1] ** (b - 1) * x[:, 2] ** c
            if c:
                g[2] += cf * c * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** (c - 1)
        return g

    return f, grad


CASES = [(t, p) for t in ("hex", "prism", "tet", "pyr") for p in (1, 2, 3, 4)]


@pytest.fixture(scope="module")
def refs():
    return {c: RefElement(*c) for c in CASES}


@pytest.mark.parametrize("case", CASES)
def test_interpolation_and_derivative_exactness(refs, case):
    r = refs[case]
    rng = np.random.default_rng(1)
    for _ in range(3):
        f, g = _random_poly(r.etype, r.p, rng)
        fu = f(r.upts)
        scale = np.abs(fu).max()
        assert np.abs(r.M0 @ fu - f(r.fpts)).max() < 1e-13 * scale * 10
        assert np.abs(r.M7 @ fu - f(r.qpts)).max() < 1e-13 * scale * 10
        np.testing.assert_allclose(np.einsum("dsu,u->ds", r.Dg, fu), g(r.upts), atol=1e-12 * scale * 10)


@pytest.mark.parametrize("case", CASES)
def test_projection_is_left_inverse_of_interpolation(refs, case):
    r = refs[case]
    np.testing.assert_allclose(r.M8 @ r.M7, np.eye(r.nu), atol=1e-13)


@pytest.mark.parametrize("case", CASES)
def test_quadrature_weights_and_volume(refs, case):
    r = refs[case]
    vol = {"hex": 8.0, "prism": 4.0, "tet": 4.0 / 3.0, "pyr": 8.0 / 3.0}[r.etype]
    assert abs(r.qwts.sum() - vol) < 1e-13
    assert abs(r.wu.sum() - vol) < 1e-13


@pytest.mark.parametrize("case", [c for c in CASES if c[0] != "pyr"])
def test_divergence_operator_is_weak_form(refs, case):
    """(M1 - M3 M2) M9 = -Mass^-1 sum_d D_{q,d}^T W_q: the FR-DG divergence with
    the projected flux equals integration by parts against the test functions,
    with the face terms removed exactly by the lifting.  Pyramids: the
    identity needs a space closed under differentiation, which theirs is not;
    their weak form is pinned in test_oracle_pyr.py."""
    r = refs[case]
    _, Dq = basis.nodal(r.etype, r.p, r.upts, r.qpts)
    for d in range(3):
        fu = r.M8  # M9 block for component d
        lhs = r.Dg[d] @ fu - r.M3 @ (r.fnorm[:, d][:, None] * (r.M0 @ fu))
        rhs = -np.linalg.solve(r.mass.astype(np.float64), (Dq[d].T * r.qwts[None, :]).astype(np.float64))
        np.testing.assert_allclose(lhs, rhs, atol=1e-11 * np.abs(rhs).max())


@pytest.mark.parametrize("case", CASES)
def test_lifting_preserves_face_integrals(refs, case):
    """w_u^T M3 = face quadrature weights of each flux point (int of its face
    nodal basis function): lifting puts exactly the face integral in the
    element."""
    r = refs[case]
    wf = r.wu @ r.M3
    for f, fc in enumerate(r.faces):
        sel = r.fface == f
        area = {"quad": 4.0, "tri": 2.0}[fc["kind"]] * fc["jac"]
        assert abs(wf[sel].sum() - area) < 1e-13
        assert np.all(wf[sel] > 0)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_hex_lifting_equals_radau_correction_derivative(refs, p):
    """DG correction functions in 1-D are the right/left Radau polynomials
    g_R = (P_{p+1} + P_p)/2, g_L = (-1)^{p+1} (P_{p+1} - P_p)/2 (Huynh 2007);
    the hex lifting of a flux point on face xi=+1 (resp. -1) into the solution
    points of its line is g_R'(x_i) (resp. -g_L'(x_i)), zero elsewhere."""
    r = refs[("hex", p)]
    n = p + 1
    x = r.gl
    cR = np.zeros(p + 2)
    cR[p + 1] = 0.5
    cR[p] = 0.5
    cL = np.zeros(p + 2)
    cL[p + 1] = 0.5 * (-1) ** (p + 1)
    cL[p] = -0.5 * (-1) ** (p + 1)
    dgR = npleg.legval(x, npleg.legder(cR))
    dgL = npleg.legval(x, npleg.legder(cL))
    for face, dg in [(1, dgR), (0, -dgL)]:
        cols = np.nonzero(r.fface == face)[0]
        for b in range(n):
            for a in range(n):
                col = r.M3[:, cols[a + n * b]]
                expect = np.zeros(r.nu)
                for i in range(n):
                    expect[i + n * (a + n * b)] = dg[i]
                np.testing.assert_allclose(col, expect, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_hex_operators_factor_into_1d(refs, p):
    r = refs[("hex", p)]
    gl, glw = quadrature.gauss_legendre(p + 1)
    gq, gqw = quadrature.gauss_legendre(p + 3)
    I1 = basis.line_nodal(gl, gq)
    np.testing.assert_allclose(r.M7, np.kron(I1, np.kron(I1, I1)), atol=1e-13)
    P1 = (I1.T * gqw[None, :]) / glw[:, None]  # W_u^-1 I^T W_q
    np.testing.assert_allclose(r.M8, np.kron(P1, np.kron(P1, P1)), atol=1e-13)
    # the paper's orthonormal-basis form of the projection (psi = normalised Legendre)
    k = np.arange(p + 1)
    psi_u = npleg.legvander(gl, p) * np.sqrt((2 * k + 1) / 2.0)
    psi_q = npleg.legvander(gq, p) * np.sqrt((2 * k + 1) / 2.0)
    np.testing.assert_allclose(psi_u @ (psi_q.T * gqw[None, :]), P1, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_prism_operators_factor_into_triangle_times_line(refs, p):
    r = refs[("prism", p)]
    gl, glw = quadrature.gauss_legendre(p + 1)
    gq, gqw = quadrature.gauss_legendre(p + 3)
    tq, tqw = quadrature.triangle_conical(p + 1)
    L = basis.line_nodal(gl, gq)
    T = basis.tri_nodal(p, r.tri_nodes, tq)
    np.testing.assert_allclose(r.M7, np.kron(L, T), atol=1e-13)
    PL = (L.T * gqw[None, :]) / glw[:, None]
    Mt = T.T @ (tqw[:, None] * T)
    PT = np.linalg.solve(Mt.astype(np.float64), (T.T * tqw[None, :]).astype(np.float64))
    np.testing.assert_allclose(r.M8, np.kron(PL, PT), atol=1e-12)


@pytest.mark.parametrize("p,key", [(2, "ws2"), (3, "ws3")])
def test_prism_rhs_independent_of_the_triangle_point_set(p, key):
    """With flux and surface-flux anti-aliasing on affine prisms every term
    of the RHS is a projection or a DG lift of quantities evaluated at fixed
    quadrature points, so du as a polynomial does not depend on where the
    solution and flux points sit in the triangle.  The oracle on the
    triangle points the paper prints (section 2.1 and section 4.1 figures)
    and on its own point set must give the same polynomial: this pins the
    prism's nodal basis, interpolation, projection and lifting operators
    against a second point set that the oracle did not construct."""
    from oracle.mesh import Mesh
    from oracle.rhs import Params, rhs
    from paper_2401_06132_amd import inputs

    ws = _golden()[key].reshape(-1, 2)
    assert len(ws) == (p + 1) * (p + 2) // 2
    mb = Mesh(2, 2, 2, p, "prism", surf_aa=True)
    mw = Mesh(2, 2, 2, p, "prism", tri_nodes=ws, surf_aa=True)
    rb, rw = mb.refs["prism"], mw.refs["prism"]
    Ub = inputs.element_state([mb.upts_coords("prism")], seed=4)[0]
    L_bw, _ = basis.nodal("prism", p, rb.upts, rw.upts)  # own basis at the paper's points
    L_wb, _ = basis.nodal("prism", p, rw.upts, rb.upts)
    Uw = np.einsum("wu,evu->evw", np.asarray(L_bw, float), Ub)
    par = Params(pref=inputs.P0, aa=True)
    db = rhs(mb, {"prism": Ub}, par)["prism"]
    dw = rhs(mw, {"prism": Uw}, par)["prism"]
    got = np.einsum("bw,evw->evb", np.asarray(L_wb, float), dw)
    err = np.abs(got - db).max(axis=(0, 2)) / np.abs(db).max(axis=(0, 2))
    assert np.all(err < 1e-12), err
    # without surface-flux anti-aliasing the interface flux is collocated
    # at the flux points, which differ: the two results must differ
    mb0 = Mesh(2, 2, 2, p, "prism")
    mw0 = Mesh(2, 2, 2, p, "prism", tri_nodes=ws)
    d0 = np.einsum("bw,evw->evb", np.asarray(L_wb, float), rhs(mw0, {"prism": Uw}, par)["prism"])
    assert np.abs(d0 - rhs(mb0, {"prism": Ub}, par)["prism"]).max() > 1e-6
