"""Pins for the oracle's tetrahedra: the conical-product rule against the
closed-form simplex integrals, the node set (count, interior, invariance
under the tetrahedron's symmetries, unisolvence), and the right-hand side on
tetrahedral and prism/tetrahedron meshes (free stream, discrete conservation,
entropy-wave convergence).  The operator identities (interpolation and
derivative exactness, projection, weak-form divergence, lifting) are pinned
for tetrahedra in test_oracle_operators.py."""

import itertools
import math

import numpy as np
import pytest

from oracle import basis, quadrature
from oracle.mesh import Mesh
from oracle.rhs import Params, rhs
from paper_2401_06132_amd import inputs


def _simplex_monomial(a, b, c):
    """int over the reference tetrahedron of xi^a eta^b zeta^c, from the unit
    simplex moments x^i y^j z^k -> i! j! k! / (i+j+k+3)! and xi = 2x - 1."""
    tot = 0.0
    for i in range(a + 1):
        for j in range(b + 1):
            for k in range(c + 1):
                coef = math.comb(a, i) * math.comb(b, j) * math.comb(c, k) * 2 ** (i + j + k) * \
                    (-1) ** (a - i + b - j + c - k)
                tot += coef * math.factorial(i) * math.factorial(j) * math.factorial(k) / math.factorial(i + j + k + 3)
    return 8.0 * tot


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_tetrahedron_rule_exact_to_degree_2k_minus_1(k):
    x, w = quadrature.tetrahedron_conical(k)
    assert len(w) == k ** 3 and np.all(w > 0)
    assert np.all(x > -1) and np.all(x.sum(axis=1) < -1)
    for a in range(2 * k):
        for b in range(2 * k - a):
            for c in range(2 * k - a - b):
                want = _simplex_monomial(a, b, c)
                got = np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c)
                assert abs(got - want) < 1e-14 * max(1.0, abs(want)) * 10, (a, b, c)
    # not exact one degree higher (the rule is not accidentally stronger)
    errs = [abs(np.sum(w * x[:, 2] ** (2 * k)) - _simplex_monomial(0, 0, 2 * k))]
    assert max(errs) > 1e-10


def _bary(x):
    lam = np.empty((len(x), 4))
    lam[:, 1:] = (x + 1.0) / 2.0
    lam[:, 0] = 1.0 - lam[:, 1:].sum(axis=1)
    return lam


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tetrahedron_nodes(p):
    x = quadrature.tetrahedron_nodes(p)
    assert len(x) == (p + 1) * (p + 2) * (p + 3) // 6
    lam = _bary(x)
    assert np.all(lam > 0)
    key = lambda L: np.round(L, 12)  # noqa: E731
    base = {tuple(r) for r in key(lam)}
    for perm in itertools.permutations(range(4)):
        assert {tuple(r) for r in key(lam[:, perm])} == base
    V, _ = basis.eval_basis("tet", p, x)
    sv = np.linalg.svd(np.asarray(V, float), compute_uv=False)
    assert sv.min() / sv.max() > 1e-5  # Legendre products: 2e-4 at p = 4


@pytest.mark.parametrize("kind", ["tet", "prism_tet"])
@pytest.mark.parametrize("p", [1, 3])
def test_free_stream_and_conservation(kind, p):
    m = Mesh(2, 2, 2, p, kind)
    U = {t: u for t, u in zip(m.types, inputs.uniform_state([(m.nelem[t], m.refs[t].nu) for t in m.types]))}
    for pref in (0.0, inputs.P0):
        du = rhs(m, U, Params(pref=pref))
        assert max(np.abs(du[t]).max() for t in m.types) < 1e-12 * 72 * 10
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
    for aa in (True, False):
        du = rhs(m, U, Params(pref=inputs.P0, aa=aa))
        tot = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, du[t]) for t in m.types)
        scale = sum(np.einsum("e,u,evu->v", m.detJ[t], m.refs[t].wu, np.abs(du[t])) for t in m.types)
        assert np.all(np.abs(tot) <= 1e-13 * scale)


def _entropy_wave(x, a=0.5, p=1.0):
    s = x[..., 0] + x[..., 1] + x[..., 2]
    rho = 1 + 0.2 * np.sin(s)
    E = p / 0.4 + 0.5 * rho * 3 * a * a
    u = np.stack([rho, rho * a, rho * a, rho * a, E], -1)
    drho = -3 * a * 0.2 * np.cos(s)
    du = np.stack([drho, a * drho, a * drho, a * drho, 1.5 * a * a * drho], -1)
    return u, du


@pytest.mark.parametrize("kind", ["tet", "prism_tet"])
def test_entropy_wave_convergence(kind):
    """Euler entropy wave: the RHS error falls at about the design rate."""
    p = 2
    errs = []
    for N in (3, 6):
        m = Mesh(N, N, N, p, kind)
        U = {t: np.ascontiguousarray(np.moveaxis(_entropy_wave(m.upts_coords(t))[0], -1, 1)) for t in m.types}
        ex = {t: np.ascontiguousarray(np.moveaxis(_entropy_wave(m.upts_coords(t))[1], -1, 1)) for t in m.types}
        du = rhs(m, U, Params(mu=0.0, tau=0.0))
        errs.append(max(np.abs(du[t] - ex[t]).max() for t in m.types))
    assert np.log2(errs[0] / errs[1]) > p - 0.3
