"""Periodic box meshes, affine metrics and flux-point pairing.
Test infrastructure only.

Box [lo, hi]^3 split into nx*ny*nz cells, cell index c = i + nx (j + ny k).
  kind "hex"   : one axis-aligned hexahedron per cell.
  kind "prism" : two prisms per cell.  The cell's x-z square is split by the
                 diagonal from (x0+h, z0) to (x0, z0+h) and extruded along y,
                 so each z = const cell face is one full prism quadrilateral
                 (required for conforming hex-prism interfaces).  Prism "A"
                 holds the corner (x0, z0), prism "B" the corner (x0+h, z0+h).
                 Maps (positive Jacobian):
                   A: x = x0 + (eta+1) h/2, y = y0 + (zeta+1) h/2, z = z0 + (xi+1) h/2
                   B: x = x0 + h - (eta+1) h/2, y = y0 + (zeta+1) h/2, z = z0 + h - (xi+1) h/2
  kind "mixed" : hexahedra in cells whose centre has z < 0, prisms elsewhere.
  kind "tet"   : six tetrahedra per cell (Kuhn subdivision of the cube
                 mirrored in x: in unit coordinates u = ((x0+h-x)/h, (y-y0)/h,
                 (z-z0)/h) the tetrahedra are u_a >= u_b >= u_c for the six
                 orders (a, b, c) of the axes, vertices 0, e_a, e_a + e_b,
                 (1,1,1) in that order mapped to V0..V3 (V1 and V2 swapped
                 where that gives a negative Jacobian)).  Every cell face is
                 cut along the same diagonal as its opposite face, so the
                 tetrahedra are conforming across cells and the period; the
                 y faces are cut along the prisms' diagonal.
  kind "prism_tet" : prisms in cells whose centre has y < 0, tetrahedra
                 elsewhere (prism triangles meet tetrahedron faces).
  kind "pyr"   : six pyramids per cell, one on each cell face (its base)
                 with the apex at the cell centre; the pyramid on face f
                 (x-, x+, y-, y+, z-, z+ in that order) maps reference
                 (xi, eta, zeta) to B + xi e1 + eta e2 + (1+zeta)/2 (C - B),
                 B the face centre, C the cell centre and e1, e2 the face's
                 half edges, ordered so that e1 x e2 points into the cell
                 (x-: (y, z); x+: (z, y); y-: (z, x); y+: (x, z); z-: (x, y);
                 z+: (y, x)).  Bases meet hexahedron faces or other bases
                 (GL(n)^2 points on the same square); triangles meet the
                 neighbouring pyramids of the same cell.
  kind "hex_pyr" : hexahedra in cells whose centre has z < 0, pyramids
                 elsewhere.
  kind "hex_pyr_tet" : hexahedra, pyramids and tetrahedra (nz >= 3).  Layers
                 k < nz // 2 hold hexahedra and layers between nz // 2 and
                 nz - 1 tetrahedra (the Kuhn cells of "tet").  Layer nz // 2
                 and the last layer hold transition cells: one pyramid on the
                 cell face towards the hexahedra (z- in layer nz // 2, z+ in
                 the last layer, which meets the first hexahedron layer
                 across the period) and ten tetrahedra.  Those are the
                 pyramids of the five other faces with the apex at the cell
                 centre, each cut in two along the face diagonal that the
                 Kuhn cells use there: the diagonal joining the face's
                 corners with the smallest and the largest sum of the unit
                 coordinates u.  Element order in a transition cell: the
                 pyramid, then two tetrahedra per face in face order, the
                 face's two other corners taken in lexicographic order of
                 (x, y, z).
  kind "hex_prism_pyr_tet" : all four types (nz >= 3): "hex_pyr_tet" where
                 the cell centre has y >= 0; where y < 0, hexahedra in the
                 layers k < nz // 2 and prism cells above (their z faces are
                 full quadrilaterals and their y faces are cut like the Kuhn
                 cells', so they meet hexahedra, transition cells and
                 tetrahedra conformingly).
  kinds "hex_warp", "prism_warp", "mixed_warp" : the curved (non-affine)
                 forms of "hex", "prism" and "mixed": every grid vertex x is
                 moved to x + warp h (sin y cos z, sin z cos x, sin x cos y)
                 (h the cell size per axis, warp = 0.2 by default; the field
                 is periodic, so the mesh stays periodic and conforming) and
                 each element is the map of its moved vertices with the
                 element's vertex shape functions -- trilinear for a
                 hexahedron (8 vertices), a triangle's barycentric functions
                 times the line's for a prism (6 vertices) -- so quadrilateral
                 faces are bilinear (curved) surfaces and the metrics vary
                 from point to point.  The cofactor metric terms
                 det J J^-1 of a trilinear map are exact (no discrete metric
                 is formed); their normal components are bilinear on every
                 face, so the GL(n)^2 flux points interpolate them exactly,
                 and the volume integrand is integrated exactly by GL(m)^3:
                 free-stream preservation is exact at every order.
Metrics: affine meshes keep one J per element (Jinv, detJ of shape (E, 3, 3)
and (E,)); curved meshes give them per point through metrics(t, ref_pts).
surf_aa=True builds the reference elements with surface-flux
anti-aliasing (flux points at the face quadrature points).
Element numbering: cells in index order; a prism cell yields A then B, a
pyramid cell its six pyramids in face order, a transition cell its pyramid
then its ten tetrahedra.  The
position in that sequence is the global element id; each element type keeps
its own elements in order of appearance.

Pairing (section 2.1: paired flux points coincide in physical space) is done
by physical coordinates modulo the period.  Which side of a pair is "L" is
not fixed by the paper (the common solution is asymmetric, so each pair must
be visited once); the reading used: L is the element with the lower global
id; for an element paired with itself across the periodic boundary, L is the
face whose centroid is lexicographically smaller in (x, y, z).
"""

import numpy as np

from .elements import RefElement


# reference vertices of the curved element types, in shape-function order
_REF_VERTS = {
    "hex": np.array([[2 * a - 1, 2 * b - 1, 2 * c - 1] for c in range(2) for b in range(2) for a in range(2)], float),
    "prism": np.array([[x, y, z] for z in (-1.0, 1.0) for (x, y) in ((-1.0, -1.0), (1.0, -1.0), (-1.0, 1.0))]),
}


# reference vertices of the affine element types, in the order in which a
# general mesh lists an element's vertices (hexahedra and prisms as above;
# tetrahedra V0..V3; pyramids the base corners a + 2b at (2a-1, 2b-1, -1),
# then the apex)
REF_VERTS = {
    "hex": _REF_VERTS["hex"],
    "prism": _REF_VERTS["prism"],
    "tet": np.array([[-1.0, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]),
    "pyr": np.array([[-1.0, -1, -1], [1, -1, -1], [-1, 1, -1], [1, 1, -1], [0, 0, 1]]),
}


def elements_mesh(p, verts, lattice=None, surf_aa=False):
    """A conforming mesh of affine elements from their vertices (section 2.1:
    each element is the image of its reference element under its own
    mapping, eqs. transall / govqtrans; here an affine one per element).

    verts: dict type -> (E_t, nv, 3) vertex coordinates in the order of
    REF_VERTS; element order (and so the global id that decides L/R) is
    hexahedra, prisms, tetrahedra, pyramids, each in the given order.
    lattice: (3, 3) period vectors (rows) of a periodic mesh, or None.  A
    vertex set that is not the affine image of the reference element raises
    ValueError, as does a face that pairs with no other."""
    types = [t for t in ("hex", "prism", "tet", "pyr") if t in verts and len(verts[t])]
    m = Mesh.__new__(Mesh)
    m.p, m.kind, m.curved = p, "elements", False
    allv = np.concatenate([np.asarray(verts[t], float).reshape(-1, 3) for t in types])
    m.lo = allv.min(axis=0)
    m.hi = allv.max(axis=0)
    if lattice is None:
        # no period: a lattice far larger than the mesh never wraps a face
        lattice = np.diag(4.0 * (m.hi - m.lo) + 1.0)
    m.lattice = np.asarray(lattice, float)
    m.period = None
    m.refs = {t: RefElement(t, p, None, surf_aa=surf_aa) for t in types}
    m.types = types
    m.org, m.J, m.gid, m.nelem = {}, {}, {}, {}
    g = 0
    hmin = np.inf
    for t in types:
        X = np.asarray(verts[t], float)
        ref = REF_VERTS[t]
        A = np.concatenate([np.ones((len(ref), 1)), ref], axis=1)  # [1, xi]
        coef = np.einsum("ij,ejk->eik", np.linalg.pinv(A), X)  # (E, 4, 3): org, then J^T rows
        org, J = coef[:, 0, :], np.transpose(coef[:, 1:, :], (0, 2, 1))
        fit = org[:, None, :] + np.einsum("eij,vj->evi", J, ref)
        size = np.linalg.norm(X.max(axis=1) - X.min(axis=1), axis=1)
        if np.any(np.abs(fit - X).max(axis=(1, 2)) > 1e-10 * size):
            raise ValueError("elements must be affine images of the reference element")
        m.org[t], m.J[t] = org, J
        m.gid[t] = g + np.arange(len(X))
        g += len(X)
        m.nelem[t] = len(X)
        hmin = min(hmin, float(np.linalg.norm(J, axis=1).min()))
    m.h = np.full(3, hmin)
    m.detJ = {t: np.linalg.det(m.J[t]) for t in types}
    m.Jinv = {t: np.linalg.inv(m.J[t]) for t in types}
    if any(np.any(m.detJ[t] <= 0) for t in types):
        raise ValueError("non-positive Jacobian")
    m._pair()
    return m


def _kuhn_tets(x0, h):
    """Vertices (4, 3) of the six tetrahedra of the cell at x0 (see the
    module header), each with a positive orientation."""
    from itertools import permutations
    out = []
    for order in permutations(range(3)):
        u = [np.zeros(3)]
        for ax in order:
            nxt = u[-1].copy()
            nxt[ax] = 1.0
            u.append(nxt)
        P = [x0 + h * np.array([1.0 - q[0], q[1], q[2]]) for q in u]
        if np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)) < 0:
            P[1], P[2] = P[2], P[1]
        out.append(P)
    return out


def _pyramid_on_face(x0, h, ax, sg):
    """Jacobian and origin of the pyramid on the face (ax, sg) of the cell at
    x0 with its apex at the cell centre (the map of kind "pyr")."""
    C = x0 + 0.5 * h
    t1, t2 = [a for a in range(3) if a != ax]
    if (sg < 0) != (ax != 1):
        t1, t2 = t2, t1
    e1, e2 = np.zeros(3), np.zeros(3)
    e1[t1], e2[t2] = 0.5 * h[t1], 0.5 * h[t2]
    B = C.copy()
    B[ax] += sg * 0.5 * h[ax]
    return np.stack([e1, e2, 0.5 * (C - B)], axis=1), B + 0.5 * (C - B)


def _transition_tets(x0, h, base):
    """Vertices (4, 3) of the ten tetrahedra of a transition cell whose
    pyramid sits on the face base = (axis, sign): for each other face, its
    corners D0, D1 with the smallest and largest sum of the Kuhn unit
    coordinates u = ((x0+h-x)/h, (y-y0)/h, (z-z0)/h) and the cell centre C,
    with each of the two remaining corners; positive orientation."""
    C = x0 + 0.5 * h
    out = []
    for ax in range(3):
        for sg in (-1.0, 1.0):
            if (ax, sg) == base:
                continue
            corners = []
            for a in (0.0, 1.0):
                for b in (0.0, 1.0):
                    u = np.zeros(3)
                    u[ax] = 0.0 if sg < 0 else 1.0
                    o = [d for d in range(3) if d != ax]
                    u[o[0]], u[o[1]] = a, b
                    # the face is sg along axis ax in x; u_x runs against x
                    if ax == 0:
                        u[0] = 1.0 - u[0]
                    corners.append(u)
            corners.sort(key=lambda u: u.sum())
            X = [x0 + h * np.array([1.0 - u[0], u[1], u[2]]) for u in corners]
            D0, D1 = X[0], X[3]
            # the two other corners in lexicographic order of (x, y, z)
            for O in sorted((X[1], X[2]), key=lambda x: tuple(x)):
                P = [D0, D1, O, C]
                if np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)) < 0:
                    P[1], P[2] = P[2], P[1]
                out.append(P)
    return out


class Mesh:
    def __init__(self, nx, ny, nz, p, kind="hex", lo=-np.pi, hi=np.pi, m=None, tri_nodes=None, surf_aa=False,
                 warp=0.2):
        self.nx, self.ny, self.nz, self.p, self.kind = nx, ny, nz, p, kind
        self.lo, self.hi = lo, hi
        L = hi - lo
        self.period = np.array([L, L, L])
        self.lattice = np.diag(self.period)  # period vectors (rows)
        h = np.array([L / nx, L / ny, L / nz])
        self.h = h
        self.curved = kind.endswith("_warp")
        if self.curved:
            kind = kind[:-len("_warp")]
            if kind not in ("hex", "prism", "mixed"):
                raise ValueError("warped meshes: hex, prism or mixed")
        types = {"hex": ["hex"], "prism": ["prism"], "mixed": ["hex", "prism"], "tet": ["tet"],
                 "prism_tet": ["prism", "tet"], "pyr": ["pyr"], "hex_pyr": ["hex", "pyr"],
                 "hex_pyr_tet": ["hex", "tet", "pyr"], "hex_prism_pyr_tet": ["hex", "prism", "tet", "pyr"]}[kind]
        if kind in ("hex_pyr_tet", "hex_prism_pyr_tet") and nz < 3:
            raise ValueError(kind + " needs nz >= 3")
        self.refs = {}
        for t in types:
            self.refs[t] = RefElement(t, p, m, tri_nodes=tri_nodes, surf_aa=surf_aa)
        org = {t: [] for t in types}
        A = {t: [] for t in types}
        gid = {t: [] for t in types}
        g = 0
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    x0 = lo + np.array([i, j, k]) * h
                    zc = x0[2] + 0.5 * h[2]
                    yc = x0[1] + 0.5 * h[1]
                    if kind == "mixed":
                        ctype = "hex" if zc < 0.0 else "prism"
                    elif kind == "prism_tet":
                        ctype = "prism" if yc < 0.0 else "tet"
                    elif kind == "hex_pyr":
                        ctype = "hex" if zc < 0.0 else "pyr"
                    elif kind in ("hex_pyr_tet", "hex_prism_pyr_tet"):
                        kh = nz // 2
                        ctype = "hex" if k < kh else ("trans_down" if k == kh else
                                                      ("trans_up" if k == nz - 1 else "tet"))
                        if kind == "hex_prism_pyr_tet" and yc < 0.0 and k >= kh:
                            ctype = "prism"
                    else:
                        ctype = kind
                    if ctype in ("trans_down", "trans_up"):
                        base = (2, -1.0) if ctype == "trans_down" else (2, 1.0)
                        Jp, op = _pyramid_on_face(x0, h, *base)
                        org["pyr"].append(op)
                        A["pyr"].append(Jp)
                        gid["pyr"].append(g)
                        g += 1
                        for P in _transition_tets(x0, h, base):
                            Jt = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1) / 2.0
                            org["tet"].append(P[0] + Jt @ np.ones(3))
                            A["tet"].append(Jt)
                            gid["tet"].append(g)
                            g += 1
                    elif ctype == "pyr":
                        C = x0 + 0.5 * h
                        for ax in range(3):
                            for sg in (-1.0, 1.0):
                                t1, t2 = [a for a in range(3) if a != ax]
                                # e1 x e2 must point into the cell, along -sg
                                if (sg < 0) != (ax != 1):
                                    t1, t2 = t2, t1
                                e1, e2 = np.zeros(3), np.zeros(3)
                                e1[t1], e2[t2] = 0.5 * h[t1], 0.5 * h[t2]
                                B = C.copy()
                                B[ax] += sg * 0.5 * h[ax]
                                Jp = np.stack([e1, e2, 0.5 * (C - B)], axis=1)
                                org["pyr"].append(B + 0.5 * (C - B))
                                A["pyr"].append(Jp)
                                gid["pyr"].append(g)
                                g += 1
                    elif ctype == "tet":
                        for P in _kuhn_tets(x0, h):
                            Jt = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1) / 2.0
                            org["tet"].append(P[0] + Jt @ np.ones(3))
                            A["tet"].append(Jt)
                            gid["tet"].append(g)
                            g += 1
                    elif ctype == "hex":
                        org["hex"].append(x0 + 0.5 * h)
                        A["hex"].append(np.diag(0.5 * h))
                        gid["hex"].append(g)
                        g += 1
                    else:
                        hx, hy, hz = 0.5 * h
                        # columns: d x / d(xi, eta, zeta)
                        org["prism"].append(x0 + 0.5 * h)
                        A["prism"].append(np.array([[0.0, hx, 0.0], [0.0, 0.0, hy], [hz, 0.0, 0.0]]))
                        gid["prism"].append(g)
                        g += 1
                        org["prism"].append(x0 + 0.5 * h)
                        A["prism"].append(np.array([[0.0, -hx, 0.0], [0.0, 0.0, hy], [-hz, 0.0, 0.0]]))
                        gid["prism"].append(g)
                        g += 1
        self.types = [t for t in types if len(org[t])]
        self.org = {t: np.array(org[t]) for t in self.types}
        self.J = {t: np.array(A[t]) for t in self.types}
        self.gid = {t: np.array(gid[t]) for t in self.types}
        self.nelem = {t: len(self.org[t]) for t in self.types}
        if self.curved:
            # vertices: the affine images of the reference vertices (cell
            # corners), moved by the warp field
            self.verts = {}
            for t in self.types:
                V = self.org[t][:, None, :] + np.einsum("eij,vj->evi", self.J[t], _REF_VERTS[t])
                self.verts[t] = V + warp * h * np.stack([np.sin(V[..., 1]) * np.cos(V[..., 2]),
                                                         np.sin(V[..., 2]) * np.cos(V[..., 0]),
                                                         np.sin(V[..., 0]) * np.cos(V[..., 1])], axis=-1)
            self.detJ, self.Jinv, self.detJq, self.Jinvq = {}, {}, {}, {}
            for t in self.types:
                r = self.refs[t]
                self.detJ[t], self.Jinv[t] = self.metrics(t, r.upts)  # at the solution points
                self.detJq[t], self.Jinvq[t] = self.metrics(t, r.qpts)  # at the quadrature points
                if np.any(self.metrics(t, r.fpts)[0] <= 0) or np.any(self.detJq[t] <= 0):
                    raise ValueError("non-positive Jacobian")
        else:
            self.detJ = {t: np.linalg.det(self.J[t]) for t in self.types}
            self.Jinv = {t: np.linalg.inv(self.J[t]) for t in self.types}
        if any(np.any(self.detJ[t] <= 0) for t in self.types):
            raise ValueError("non-positive Jacobian")
        self._pair()

    @staticmethod
    def _shape(t, ref_pts):
        """Vertex shape functions N_v (npts, nv) and their gradients
        (npts, nv, 3).  hex: trilinear, vertex v = a + 2b + 4c at reference
        corner (2a-1, 2b-1, 2c-1).  prism: lambda_t(xi, eta) (1 -+ zeta)/2,
        vertex v = t + 3c with lambda_0 = -(xi+eta)/2, lambda_1 = (1+xi)/2,
        lambda_2 = (1+eta)/2 (triangle vertices (-1,-1), (1,-1), (-1,1)),
        c = 0 at zeta = -1."""
        x = np.asarray(ref_pts, float)
        if t == "hex":
            s = np.array([[2 * a - 1, 2 * b - 1, 2 * c - 1] for c in range(2) for b in range(2) for a in range(2)],
                         float)
            f = 0.5 * (1.0 + x[:, None, :] * s[None, :, :])  # (npts, 8, 3)
            N = f.prod(axis=2)
            dN = np.empty(f.shape)
            for d in range(3):
                o = [k for k in range(3) if k != d]
                dN[:, :, d] = 0.5 * s[None, :, d] * f[:, :, o[0]] * f[:, :, o[1]]
            return N, dN
        lam = np.stack([-(x[:, 0] + x[:, 1]) / 2, (1 + x[:, 0]) / 2, (1 + x[:, 1]) / 2], axis=1)
        dlam = np.array([[-0.5, -0.5], [0.5, 0.0], [0.0, 0.5]])
        zf = np.stack([(1 - x[:, 2]) / 2, (1 + x[:, 2]) / 2], axis=1)
        zs = np.array([-0.5, 0.5])
        N = np.empty((len(x), 6))
        dN = np.empty((len(x), 6, 3))
        for c in range(2):
            for tv in range(3):
                v = tv + 3 * c
                N[:, v] = lam[:, tv] * zf[:, c]
                dN[:, v, 0] = dlam[tv, 0] * zf[:, c]
                dN[:, v, 1] = dlam[tv, 1] * zf[:, c]
                dN[:, v, 2] = lam[:, tv] * zs[c]
        return N, dN

    def metrics(self, t, ref_pts, elems=None):
        """det J (E, npts) and J^-1 (E, npts, 3, 3) at reference points
        (curved meshes; J[i][j] = d x_i / d xi_j)."""
        X = self.verts[t] if elems is None else self.verts[t][elems]
        _, dN = self._shape(t, ref_pts)
        J = np.einsum("evi,pvj->epij", X, dN)
        return np.linalg.det(J), np.linalg.inv(J)

    # physical coordinates of reference points for every element of type t
    def phys(self, t, ref_pts, elems=None):
        if self.curved:
            X = self.verts[t] if elems is None else self.verts[t][elems]
            N, _ = self._shape(t, ref_pts)
            return np.einsum("pv,evi->epi", N, X)
        org = self.org[t] if elems is None else self.org[t][elems]
        J = self.J[t] if elems is None else self.J[t][elems]
        return org[:, None, :] + np.einsum("eij,pj->epi", J, ref_pts)

    def upts_coords(self, t):
        return self.phys(t, self.refs[t].upts)

    def _pair(self):
        # flat flux-point numbering: types in order, then element, then point
        self.foff, off = {}, 0
        for t in self.types:
            self.foff[t] = off
            off += self.nelem[t] * self.refs[t].nf
        self.nfpts = off
        # per flat flux point: element type index and element
        self.ftype = np.concatenate([np.full(self.nelem[t] * self.refs[t].nf, i) for i, t in enumerate(self.types)])
        self.felem = np.concatenate([np.repeat(np.arange(self.nelem[t]), self.refs[t].nf) for t in self.types])
        # faces: match by centroid modulo the period lattice (rows of
        # self.lattice; coordinates taken in lattice units), then points
        # within a face pair
        fkeys, finfo, fcent = [], [], []
        Qk = 1 << 24
        Binv = np.linalg.inv(self.lattice.T)  # physical -> lattice coordinates
        for ti, t in enumerate(self.types):
            r = self.refs[t]
            E = self.nelem[t]
            c = np.stack([self.phys(t, r.fpts[r.fface == f]).mean(axis=1) for f in range(r.nfaces)],
                         axis=1).reshape(-1, 3)
            fcent.append(c)
            fkeys.append(np.mod(np.rint(((c - self.lo) @ Binv.T) * Qk).astype(np.int64), Qk))
            finfo.append(np.stack([np.full(E * r.nfaces, ti), np.repeat(np.arange(E), r.nfaces),
                                   np.tile(np.arange(r.nfaces), E), np.repeat(self.gid[t], r.nfaces)], axis=1))
        key, info, cent = np.concatenate(fkeys), np.concatenate(finfo), np.concatenate(fcent)
        order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
        ks = key[order]
        eq = np.all(ks[1:] == ks[:-1], axis=1)
        if len(ks) % 2 or not np.all(eq[0::2]) or np.any(eq[1::2]):
            raise ValueError("faces do not pair up (non-conforming mesh?)")
        fa, fb = order[0::2], order[1::2]
        ga, gb = info[fa, 3], info[fb, 3]
        ca, cb = cent[fa], cent[fb]
        lex = np.where(ca[:, 0] != cb[:, 0], ca[:, 0] < cb[:, 0],
                       np.where(ca[:, 1] != cb[:, 1], ca[:, 1] < cb[:, 1], ca[:, 2] < cb[:, 2]))
        a_first = np.where(ga == gb, lex, ga < gb)
        fL, fR = np.where(a_first, fa, fb), np.where(a_first, fb, fa)
        iL, iR = [], []
        # group face pairs by (type, local face) on both sides; match points in batch
        cls = np.stack([info[fL, 0], info[fL, 2], info[fR, 0], info[fR, 2]], axis=1)
        ucls, inv = np.unique(cls, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        for ci, (tl, ffl, tr, ffr) in enumerate(ucls):
            allsel = np.nonzero(inv == ci)[0]
            tL, tR = self.types[tl], self.types[tr]
            rL, rR = self.refs[tL], self.refs[tR]
            pl = np.nonzero(rL.fface == ffl)[0]
            pr = np.nonzero(rR.fface == ffr)[0]
            for c0 in range(0, len(allsel), 65536):
                sel = allsel[c0:c0 + 65536]
                eL, eR = info[fL[sel], 1], info[fR[sel], 1]
                XL = self.phys(tL, rL.fpts[pl], eL)
                XR = self.phys(tR, rR.fpts[pr], eR)
                if len(pl) != len(pr):
                    raise ValueError("paired faces have different point counts")
                # coordinates relative to each face's centroid coincide for the
                # two sides (the centroids differ by a period at most): match the
                # points by the rank of their quantised relative coordinates
                G, npt = XL.shape[0], XL.shape[1]
                q = 1e-7 * self.h.min()
                kL = np.rint((XL - XL.mean(axis=1, keepdims=True)) / q).astype(np.int64).reshape(-1, 3)
                kR = np.rint((XR - XR.mean(axis=1, keepdims=True)) / q).astype(np.int64).reshape(-1, 3)
                rows = np.repeat(np.arange(G), npt)
                oL = np.lexsort((kL[:, 2], kL[:, 1], kL[:, 0], rows)).reshape(G, npt) - (np.arange(G) * npt)[:, None]
                oR = np.lexsort((kR[:, 2], kR[:, 1], kR[:, 0], rows)).reshape(G, npt) - (np.arange(G) * npt)[:, None]
                j = np.empty_like(oL)
                np.put_along_axis(j, oL, oR, axis=1)
                d = XL - np.take_along_axis(XR, j[:, :, None], axis=1)
                dl = d @ Binv.T
                d = (dl - np.rint(dl)) @ self.lattice
                if np.abs(d).max() > 1e-9 * self.h.min():
                    raise ValueError("flux points of paired faces do not coincide")
                iL.append((self.foff[tL] + eL[:, None] * rL.nf + pl[None, :]).reshape(-1))
                iR.append((self.foff[tR] + eR[:, None] * rR.nf + pr[j]).reshape(-1))
        self.iL, self.iR = np.concatenate(iL), np.concatenate(iR)
        if len(self.iL) * 2 != self.nfpts:
            raise ValueError("flux points left unpaired")
        self.partner = np.full(self.nfpts, -1, dtype=np.int64)
        self.partner[self.iL] = self.iR
        self.partner[self.iR] = self.iL
        if np.any(self.partner < 0):
            raise ValueError("flux points left unpaired")
        # physical unit normals and area factors (Nanson): n = det J J^-T nhat / mag
        nrm, mag = [], []
        for t in self.types:
            r = self.refs[t]
            if self.curved:
                dj, ji = self.metrics(t, r.fpts)  # at every flux point
                v = dj[:, :, None] * np.einsum("efdc,fd->efc", ji, r.fnorm)
            else:
                v = self.detJ[t][:, None, None] * np.einsum("edc,fd->efc", self.Jinv[t], r.fnorm)
            mg = np.linalg.norm(v, axis=2)
            nrm.append((v / mg[:, :, None]).reshape(-1, 3))
            mag.append(mg.reshape(-1))
        self.fnrm, self.fmag = np.concatenate(nrm), np.concatenate(mag)
