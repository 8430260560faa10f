"""Polynomial bases of the solution spaces.  Test infrastructure only.

The nodal basis l_zeta of section 2.1 is built as l = (Vandermonde)^-T psi
for any basis psi of the space; interpolation is independent of that choice.
The oracle uses Legendre products, which are well conditioned and have no
singularity on the triangle:
  hex    Q_p : P_a(xi) P_b(eta) P_c(zeta), a, b, c <= p
  prism      : P_a(xi) P_b(eta) P_c(zeta), a + b <= p, c <= p
The paper's L2 projection (eq. FR-tdivtpcorfq) is evaluated with the
basis-independent mass-matrix form in elements.py.
"""

import numpy as np
from numpy.polynomial import legendre as npleg


def legendre_values(kmax, x):
    """P_0..P_kmax at x and their first derivatives: arrays (kmax+1, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    vals = np.empty((kmax + 1, x.size))
    ders = np.empty((kmax + 1, x.size))
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
    raise ValueError(etype)


def eval_basis(etype, p, pts):
    """Basis values V[pt, mode] and gradients G[d, pt, mode] at pts (N, 3)."""
    pts = np.asarray(pts, dtype=np.float64)
    vx, dx = legendre_values(p, pts[:, 0])
    vy, dy = legendre_values(p, pts[:, 1])
    vz, dz = legendre_values(p, pts[:, 2])
    md = modes(etype, p)
    V = np.empty((len(pts), len(md)))
    G = np.empty((3, len(pts), len(md)))
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
    Vinv = np.linalg.inv(Vn)
    return V @ Vinv, np.einsum("dpm,mz->dpz", G, Vinv)


def tri_nodal(p, nodes2, pts2):
    """Nodal basis of P_p on the triangle (2-D points)."""
    md = [(a, b) for b in range(p + 1) for a in range(p + 1 - b)]

    def ev(q):
        vx, _ = legendre_values(p, q[:, 0])
        vy, _ = legendre_values(p, q[:, 1])
        return np.stack([vx[a] * vy[b] for a, b in md], axis=1)

    return ev(np.asarray(pts2)) @ np.linalg.inv(ev(np.asarray(nodes2)))


def line_nodal(nodes1, pts1):
    """1-D Lagrange basis through nodes1 evaluated at pts1: L[pt, node]."""
    n = len(nodes1)
    vn, _ = legendre_values(n - 1, nodes1)
    v, _ = legendre_values(n - 1, pts1)
    return v.T @ np.linalg.inv(vn.T)
