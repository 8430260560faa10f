"""Polynomial bases of the solution spaces.  Test infrastructure only.

The nodal basis l_zeta of section 2.1 is built as l = (Vandermonde)^-T psi
for any basis psi of the space; interpolation is independent of that choice.
The oracle uses Legendre products, which are well conditioned and have no
singularity on the triangle:
  hex    Q_p : P_a(xi) P_b(eta) P_c(zeta), a, b, c <= p
  prism      : P_a(xi) P_b(eta) P_c(zeta), a + b <= p, c <= p
  tet    P_p : P_a(xi) P_b(eta) P_c(zeta), a + b + c <= p
  pyr        : the rational pyramid space (Bergot, Cohen & Durufle 2010),
               spanned in the collapsed coordinates a = 2 xi/(1-zeta),
               b = 2 eta/(1-zeta), c = zeta by
               P_i(a) P_j(b) (1-c)^max(i,j) P_k(c),  i, j <= p, k <= p - max(i,j).
               It contains P_p; its trace on the base is Q_p and on each
               triangular face P_p, so it conforms with hexahedron,
               prism and tetrahedron faces.
The paper's L2 projection (eq. FR-tdivtpcorfq) is evaluated with the
basis-independent mass-matrix form in elements.py.
"""

import numpy as np
from numpy.polynomial import legendre as npleg

# Operators are built in extended precision and rounded once by the caller:
# a Vandermonde inverse at p = 4 loses ~1e-14 (prism: ~3e-13) in float64,
# which would otherwise dominate the oracle's own rounding.
EXT = np.longdouble


def inv(A):
    """Inverse of a small dense matrix by Gauss-Jordan elimination with
    partial pivoting, in the matrix's own precision (numpy.linalg has no
    extended-precision path)."""
    A = np.array(A, dtype=EXT, copy=True)
    n = A.shape[0]
    B = np.eye(n, dtype=EXT)
    for c in range(n):
        piv = c + int(np.argmax(np.abs(A[c:, c])))
        if A[piv, c] == 0:
            raise np.linalg.LinAlgError("singular matrix")
        A[[c, piv]] = A[[piv, c]]
        B[[c, piv]] = B[[piv, c]]
        d = A[c, c]
        A[c] /= d
        B[c] /= d
        f = A[:, c].copy()
        f[c] = 0
        A -= np.outer(f, A[c])
        B -= np.outer(f, B[c])
    return B


def legendre_values(kmax, x):
    """P_0..P_kmax at x and their first derivatives: arrays (kmax+1, len(x)),
    in extended precision."""
    x = np.asarray(x, dtype=EXT)
    vals = np.empty((kmax + 1, x.size), dtype=EXT)
    ders = np.empty((kmax + 1, x.size), dtype=EXT)
    for k in range(kmax + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        vals[k] = npleg.legval(x, c)
        ders[k] = npleg.legval(x, npleg.legder(c)) if k > 0 else 0.0
    return vals, ders


def modes(etype, p):
    if etype == "hex":
        return [(a, b, c) for c in range(p + 1) for b in range(p + 1) for a in range(p + 1)]
    if etype == "prism":
        return [(a, b, c) for c in range(p + 1) for b in range(p + 1) for a in range(p + 1 - b)]
    if etype == "tet":
        return [(a, b, c) for c in range(p + 1) for b in range(p + 1 - c) for a in range(p + 1 - b - c)]
    if etype == "pyr":
        return [(a, b, c) for b in range(p + 1) for a in range(p + 1) for c in range(p + 1 - max(a, b))]
    raise ValueError(etype)


def _pyr_basis(p, pts):
    """Pyramid space basis values and gradients (see the module header).
    The points must avoid the apex zeta = 1."""
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    om = 1 - z
    a, b = 2 * x / om, 2 * y / om
    va, da = legendre_values(p, a)
    vb, db = legendre_values(p, b)
    vc, dc = legendre_values(p, z)
    md = modes("pyr", p)
    V = np.empty((len(pts), len(md)), dtype=EXT)
    G = np.empty((3, len(pts), len(md)), dtype=EXT)
    for k, (i, j, l) in enumerate(md):
        mu = max(i, j)
        C = om ** mu * vc[l]
        # dC/dc; (1-c)^mu differentiates to -mu (1-c)^(mu-1)
        dC = om ** mu * dc[l] - (mu * om ** (mu - 1) * vc[l] if mu > 0 else 0)
        V[:, k] = va[i] * vb[j] * C
        # d a/d xi = 2/(1-c), d a/d zeta = a/(1-c); likewise b
        G[0, :, k] = da[i] * vb[j] * C * 2 / om
        G[1, :, k] = va[i] * db[j] * C * 2 / om
        G[2, :, k] = (da[i] * a * vb[j] + va[i] * db[j] * b) * C / om + va[i] * vb[j] * dC
    return V, G


def eval_basis(etype, p, pts):
    """Basis values V[pt, mode] and gradients G[d, pt, mode] at pts (N, 3)."""
    pts = np.asarray(pts, dtype=EXT)
    if etype == "pyr":
        return _pyr_basis(p, pts)
    vx, dx = legendre_values(p, pts[:, 0])
    vy, dy = legendre_values(p, pts[:, 1])
    vz, dz = legendre_values(p, pts[:, 2])
    md = modes(etype, p)
    V = np.empty((len(pts), len(md)), dtype=EXT)
    G = np.empty((3, len(pts), len(md)), dtype=EXT)
    for k, (a, b, c) in enumerate(md):
        V[:, k] = vx[a] * vy[b] * vz[c]
        G[0, :, k] = dx[a] * vy[b] * vz[c]
        G[1, :, k] = vx[a] * dy[b] * vz[c]
        G[2, :, k] = vx[a] * vy[b] * dz[c]
    return V, G


def nodal(etype, p, nodes, pts):
    """Nodal basis l_zeta (l_zeta(nodes_sigma) = delta) evaluated at pts:
    L[pt, zeta] and gradients DL[d, pt, zeta]."""
    Vn, _ = eval_basis(etype, p, nodes)
    V, G = eval_basis(etype, p, pts)
    Vinv = inv(Vn)
    return V @ Vinv, np.einsum("dpm,mz->dpz", G, Vinv)


def tri_nodal(p, nodes2, pts2):
    """Nodal basis of P_p on the triangle (2-D points)."""
    md = [(a, b) for b in range(p + 1) for a in range(p + 1 - b)]

    def ev(q):
        vx, _ = legendre_values(p, q[:, 0])
        vy, _ = legendre_values(p, q[:, 1])
        return np.stack([vx[a] * vy[b] for a, b in md], axis=1)

    return ev(np.asarray(pts2)) @ inv(ev(np.asarray(nodes2)))


def line_nodal(nodes1, pts1):
    """1-D Lagrange basis through nodes1 evaluated at pts1: L[pt, node]."""
    n = len(nodes1)
    vn, _ = legendre_values(n - 1, nodes1)
    v, _ = legendre_values(n - 1, pts1)
    return v.T @ inv(vn.T)
