"""One-dimensional rules, the conical-product triangle, tetrahedron and
pyramid rules and the node sets used by the oracle.  Test infrastructure
only (see package header).

Paper: section 2.1 allows any solution/flux point set; hexahedra use
Gauss-Legendre points (the printed coordinates are the 3- and 4-point
Gauss-Legendre nodes, figures "ufn" and "prism2toprims3").  Prisms are a
triangle times a Gauss-Legendre line (section 4.1).  The paper prints
triangle points only for p = 2 and p = 3, so the triangle node set is a
reading: the Blyth-Pozrikidis construction on Gauss-Legendre master points,
used for every order; the tetrahedron and pyramid sets are readings too.
"""

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import roots_jacobi


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [-1, 1]; exact to degree 2n-1."""
    x, w = npleg.leggauss(n)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gauss_lobatto_legendre(n):
    """n-point Gauss-Lobatto-Legendre nodes on [-1, 1] (endpoints included):
    the endpoints plus the roots of P'_{n-1}."""
    if n < 2:
        raise ValueError("GLL needs at least two points")
    c = np.zeros(n)
    c[-1] = 1.0
    interior = np.sort(npleg.legroots(npleg.legder(c))) if n > 2 else np.array([])
    return np.concatenate([[-1.0], interior, [1.0]])


def gauss_jacobi(n, alpha, beta):
    """n-point Gauss-Jacobi rule for the weight (1-x)^alpha (1+x)^beta."""
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def triangle_conical(k):
    """Conical-product (collapsed-coordinate) rule on the reference triangle
    {xi, eta >= -1, xi + eta <= 0} with k*k points, exact for total degree
    2k-1: Gauss-Legendre in a, Gauss-Jacobi(1,0) in b, with
    xi = (1+a)(1-b)/2 - 1, eta = b and dxi deta = (1-b)/2 da db.
    Ordering: b index outer, a index inner."""
    a, wa = gauss_legendre(k)
    b, wb = gauss_jacobi(k, 1.0, 0.0)
    pts = np.empty((k * k, 2))
    wts = np.empty(k * k)
    for j in range(k):
        for i in range(k):
            pts[j * k + i] = (0.5 * (1.0 + a[i]) * (1.0 - b[j]) - 1.0, b[j])
            wts[j * k + i] = 0.5 * wa[i] * wb[j]
    return pts, wts


def triangle_nodes(p):
    """(p+1)(p+2)/2 nodes on the reference triangle, Blyth-Pozrikidis
    construction on the Gauss-Legendre master grid v_m = (1 + t_m)/2,
    t_m = GL(p+1) nodes:
        x = (1 + 2 v_i - v_j - v_k)/3,  y = (1 + 2 v_j - v_i - v_k)/3,
    k = p - i - j, on the unit right triangle, mapped to (-1,-1),(1,-1),(-1,1).
    Ordering: j outer (0..p), i inner (0..p-j)."""
    if p == 0:
        return np.array([[-1.0 / 3.0, -1.0 / 3.0]])
    v = 0.5 * (1.0 + gauss_legendre(p + 1)[0])
    pts = []
    for j in range(p + 1):
        for i in range(p + 1 - j):
            k = p - i - j
            x = (1.0 + 2.0 * v[i] - v[j] - v[k]) / 3.0
            y = (1.0 + 2.0 * v[j] - v[i] - v[k]) / 3.0
            pts.append((2.0 * x - 1.0, 2.0 * y - 1.0))
    return np.array(pts)


def tetrahedron_conical(k):
    """Conical-product (collapsed-coordinate) rule on the reference
    tetrahedron {xi, eta, zeta >= -1, xi + eta + zeta <= -1} with k^3 points,
    exact for total degree 2k-1: Gauss-Legendre in a, Gauss-Jacobi(1,0) in b,
    Gauss-Jacobi(2,0) in c, with
        zeta = c,  eta = (1+b)(1-c)/2 - 1,  xi = (1+a)(1-b)(1-c)/4 - 1,
        dxi deta dzeta = (1-b)(1-c)^2/8 da db dc.
    Ordering: c outer, b, a inner."""
    a, wa = gauss_legendre(k)
    b, wb = gauss_jacobi(k, 1.0, 0.0)
    c, wc = gauss_jacobi(k, 2.0, 0.0)
    pts = np.empty((k ** 3, 3))
    wts = np.empty(k ** 3)
    for l in range(k):
        for j in range(k):
            for i in range(k):
                q = (l * k + j) * k + i
                pts[q] = (0.25 * (1 + a[i]) * (1 - b[j]) * (1 - c[l]) - 1.0, 0.5 * (1 + b[j]) * (1 - c[l]) - 1.0, c[l])
                wts[q] = wa[i] * wb[j] * wc[l] / 8.0
    return pts, wts


# vertices of the reference tetrahedron
TET_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])


def tetrahedron_nodes(p):
    """(p+1)(p+2)(p+3)/6 nodes in the reference tetrahedron (the paper prints
    none; a reading): the three-dimensional form of the Blyth-Pozrikidis
    construction on the Gauss-Legendre master grid v_m = (1 + t_m)/2,
    t_m = GL(p+1) nodes.  For i + j + k + l = p the barycentric coordinates
        lambda_1 = (1 + 3 v_i - v_j - v_k - v_l)/4   (vertex 1, and likewise
        lambda_2 from j, lambda_3 from k, lambda_0 from l)
    sum to one; the node is sum_a lambda_a V_a.  Ordering: k outer, j, i inner."""
    if p == 0:
        return TET_VERTS.mean(axis=0)[None, :]
    v = 0.5 * (1.0 + gauss_legendre(p + 1)[0])
    pts = []
    for k in range(p + 1):
        for j in range(p + 1 - k):
            for i in range(p + 1 - k - j):
                l = p - i - j - k
                idx = (l, i, j, k)
                s = sum(v[t] for t in idx)
                lam = [(1.0 + 4.0 * v[t] - s) / 4.0 for t in idx]
                pts.append(sum(lam[a] * TET_VERTS[a] for a in range(4)))
    return np.array(pts)


def pyramid_conical(k):
    """Conical-product (collapsed-coordinate) rule on the reference pyramid
    (square base [-1,1]^2 at zeta = -1, apex (0, 0, 1)) with k^3 points:
    Gauss-Legendre in a and b, Gauss-Jacobi(2,0) in c, with
        xi = a (1-c)/2,  eta = b (1-c)/2,  zeta = c,
        dxi deta dzeta = (1-c)^2/4 da db dc.
    A monomial xi^i eta^j zeta^l becomes a^i b^j times a polynomial of degree
    i + j + l in c, so the rule is exact for total degree 2k-1 (and for
    products of two functions of the pyramid space of order k-1, which are
    polynomials of degree <= 2k-2 in each collapsed coordinate).
    Ordering: c outer, b, a inner."""
    a, wa = gauss_legendre(k)
    c, wc = gauss_jacobi(k, 2.0, 0.0)
    pts = np.empty((k ** 3, 3))
    wts = np.empty(k ** 3)
    for l in range(k):
        for j in range(k):
            for i in range(k):
                q = (l * k + j) * k + i
                s = 0.5 * (1.0 - c[l])
                pts[q] = (a[i] * s, a[j] * s, c[l])
                wts[q] = wa[i] * wa[j] * wc[l] / 4.0
    return pts, wts


# vertices of the reference pyramid: the base square counter-clockwise, then the apex
PYR_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [1.0, 1.0, -1.0], [-1.0, 1.0, -1.0], [0.0, 0.0, 1.0]])


def pyramid_nodes(p):
    """(p+1)(p+2)(2p+3)/6 solution points in the reference pyramid (the paper
    prints none; a reading): p+1 layers at the heights zeta_l = t_l, the
    Gauss-Legendre(p+1) nodes in increasing order; layer l holds the tensor
    Gauss-Legendre(p+1-l) grid of the collapsed coordinates (a, b), i.e. the
    points (a_i (1-zeta_l)/2, b_j (1-zeta_l)/2, zeta_l).  Every layer is
    unisolvent for Q_{p-l} in (a, b) and the heights are distinct, which
    makes the set unisolvent for the pyramid space.  Ordering: l outer, j,
    i inner."""
    t = gauss_legendre(p + 1)[0]
    pts = []
    for l in range(p + 1):
        g = gauss_legendre(p + 1 - l)[0]
        s = 0.5 * (1.0 - t[l])
        for j in range(p + 1 - l):
            for i in range(p + 1 - l):
                pts.append((g[i] * s, g[j] * s, t[l]))
    return np.array(pts)
