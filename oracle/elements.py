"""Reference elements and the dense operator matrices of the paper.
Test infrastructure only.

Reference elements
  hex   [-1,1]^3.  Solution points GL(n)^3 (n = p+1), index i + n(j + n k).
        Faces 0..5 = xi-, xi+, eta-, eta+, zeta-, zeta+; each carries GL(n)^2
        flux points, index a + n b over the two tangential coordinates in
        increasing axis order.
  prism triangle {xi, eta >= -1, xi + eta <= 0} x zeta in [-1,1].  Solution
        points = triangle nodes (N_t) x GL(n), index t + N_t k (section 4.1).
        Faces 0,1 = zeta -1/+1 (flux points at the triangle nodes); faces
        2,3,4 = the quadrilaterals eta = -1, xi + eta = 0, xi = -1 with GL(n)
        points along the edge (parameter s, edges run counter-clockwise) times
        GL(n) in zeta, index a + n b.
  tet   {xi, eta, zeta >= -1, xi + eta + zeta <= -1}, vertices V0..V3 =
        (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).  Solution points: the
        tetrahedron node set of quadrature.tetrahedron_nodes (a reading).
        Faces 0..3 = zeta = -1, eta = -1, xi = -1 and the slanted face
        opposite V0; each a triangle carrying the triangle nodes (mapped from
        the reference triangle with vertices (-1,-1), (1,-1), (-1,1) to the
        face's vertices in the order listed in _build_tet).
  pyr   square base [-1,1]^2 at zeta = -1, apex (0, 0, 1); vertices V0..V4 =
        (-1,-1,-1), (1,-1,-1), (1,1,-1), (-1,1,-1), (0,0,1).  Solution points:
        quadrature.pyramid_nodes (a reading).  Face 0 = the base (GL(n)^2
        flux points, index a + n b over (xi, eta)); faces 1..4 = the
        triangles (V0,V1,V4), (V1,V2,V4), (V2,V3,V4), (V3,V0,V4) (outward
        normals (0,-2,1), (2,0,1), (0,2,1), (-2,0,1) over sqrt 5), carrying
        the triangle nodes mapped like the tetrahedron's faces.
All operators are computed in extended precision (numpy longdouble) and kept
there; callers cast them to their working precision (rounding once).
Anti-aliasing quadrature (section 2.1.1): hex GL(m)^3; prism conical triangle
rule with (p+1)^2 points (degree 2p+1) x GL(m); m = p + 3 by default;
tet and pyr conical-product rules with (p+1)^3 points (degree 2p+1).

Surface-flux anti-aliasing (surf_aa=True, section 2.1.1 and table
"operatorms"): the flux points are replaced by quadrature points on the
faces -- GL(m)^2 on every quadrilateral face (index a + m b), the conical
triangle rule with (p+1)^2 points on the prism triangles -- and every
operator acting on flux points (M0, M3, M6) is rebuilt for that point set.
The lifting integral is then taken with the face rule itself,
E[u, f] = l_u(x^f) w_f; on quadrilaterals this is the exact DG lifting of
the GL(m) Lagrange basis (the rule integrates degree p + m - 1 exactly); on
triangles a (p+1)^2-point set defines no nodal basis, so the quadrature form
is the definition used there (a reading).

Operators (section 2.2; shapes as implied by the products):
  M0[f, u]     = l_u(x^f)                               disu
  Dg[d, s, u]  = d l_u / d xi_d (x^u_s)                 M4 (gradient) and M1
  M3[u, f]     = (div g_f)(x^u); DG correction functions, i.e. the lifting
                 Mass^-1 int_face l l^face_f dS_ref     tdivtconf
  M6[d, u, f]  = n_d(f) M3[u, f]                        tgradcoru
  M7[q, u]     = l_u(x^q)                               uqpts / gradcoru_qpts
  M8[u, q]     = L2 projection, Mass^-1 L_q^T W_q       (eq. FR-tdivtpcorfq)
  wu[u]        = int l_u  (integration weights for conservation checks)
The correction-function family is not fixed by the paper (it defers to
Vincent et al. 2011); the DG choice is taken (a reading).
"""

import numpy as np

from . import basis, quadrature


class RefElement:
    def __init__(self, etype, p, m=None, tri_nodes=None, surf_aa=False):
        if m is None:
            m = p + 3
        self.etype, self.p, self.n, self.m = etype, p, p + 1, m
        self.surf_aa = surf_aa
        self.fwts = None  # face quadrature weights per flux point (surf_aa)
        n = self.n
        gl, glw = quadrature.gauss_legendre(n)
        self.gl, self.glw = gl, glw
        if etype == "hex":
            self._build_hex(gl)
        elif etype == "prism":
            self._build_prism(gl, tri_nodes)
        elif etype == "tet":
            self._build_tet(tri_nodes)
        elif etype == "pyr":
            self._build_pyr(tri_nodes)
        else:
            raise ValueError(etype)
        self.nu, self.nf, self.nq = len(self.upts), len(self.fpts), len(self.qpts)
        self._build_operators()

    # ------------------------------------------------------------------ hex
    def _build_hex(self, gl):
        n, m = self.n, self.m
        self.upts = np.array([(gl[i], gl[j], gl[k]) for k in range(n) for j in range(n) for i in range(n)])
        self.nfaces = 6
        faces = []
        for axis in range(3):
            for sgn in (-1.0, 1.0):
                tang = [a for a in range(3) if a != axis]

                def fmap(s, t, axis=axis, sgn=sgn, tang=tang):
                    x = np.zeros((len(s), 3))
                    x[:, axis] = sgn
                    x[:, tang[0]] = s
                    x[:, tang[1]] = t
                    return x

                nrm = np.zeros(3)
                nrm[axis] = sgn
                faces.append(dict(kind="quad", map=fmap, normal=nrm, jac=1.0))
        self.faces = faces
        qx, qw = quadrature.gauss_legendre(m)
        if self.surf_aa:
            self._quad_face_points(qx, qw)
        else:
            self._quad_face_points(gl)
        self.qpts = np.array([(qx[i], qx[j], qx[k]) for k in range(m) for j in range(m) for i in range(m)])
        self.qwts = np.array([qw[i] * qw[j] * qw[k] for k in range(m) for j in range(m) for i in range(m)])

    # ---------------------------------------------------------------- prism
    def _build_prism(self, gl, tri_nodes):
        p, n, m = self.p, self.n, self.m
        tn = quadrature.triangle_nodes(p) if tri_nodes is None else np.asarray(tri_nodes, float)
        self.tri_nodes = tn
        self.nt = len(tn)
        self.upts = np.array([(tn[t, 0], tn[t, 1], gl[k]) for k in range(n) for t in range(self.nt)])
        self.nfaces = 5
        faces = []
        for sgn in (-1.0, 1.0):
            def tmap(xi, eta, sgn=sgn):
                return np.stack([xi, eta, np.full_like(xi, sgn)], axis=1)
            faces.append(dict(kind="tri", map=tmap, normal=np.array([0.0, 0.0, sgn]), jac=1.0))
        # edges run counter-clockwise: v0=(-1,-1) -> v1=(1,-1) -> v2=(-1,1) -> v0
        edges = [
            (lambda s: (s, -np.ones_like(s)), np.array([0.0, -1.0, 0.0]), 1.0),
            (lambda s: (-s, s), np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0), np.sqrt(2.0)),
            (lambda s: (-np.ones_like(s), -s), np.array([-1.0, 0.0, 0.0]), 1.0),
        ]
        for emap, nrm, jac in edges:
            def qmap(s, t, emap=emap):
                xi, eta = emap(s)
                return np.stack([xi, eta, t], axis=1)
            faces.append(dict(kind="quad", map=qmap, normal=nrm, jac=jac))
        self.faces = faces
        tq, tw = quadrature.triangle_conical(p + 1)
        fp, fid, fw = [], [], []
        for f, fc in enumerate(faces):
            if fc["kind"] == "tri":
                if self.surf_aa:
                    x = fc["map"](tq[:, 0], tq[:, 1])
                    fw.append(tw * fc["jac"])
                else:
                    x = fc["map"](tn[:, 0], tn[:, 1])
            else:
                if self.surf_aa:
                    g1, w1 = quadrature.gauss_legendre(m)
                else:
                    g1, w1 = gl, None
                k = len(g1)
                s = np.array([g1[a] for b in range(k) for a in range(k)])
                t = np.array([g1[b] for b in range(k) for a in range(k)])
                x = fc["map"](s, t)
                if self.surf_aa:
                    fw.append(np.array([w1[a] * w1[b] for b in range(k) for a in range(k)]) * fc["jac"])
            fp.append(x)
            fid += [f] * len(x)
        self.fpts = np.concatenate(fp)
        self.fface = np.array(fid)
        self.fnorm = np.array([faces[f]["normal"] for f in self.fface])
        if self.surf_aa:
            self.fwts = np.concatenate(fw)
        lq, lw = quadrature.gauss_legendre(m)
        self.qpts = np.array([(tq[t, 0], tq[t, 1], lq[k]) for k in range(m) for t in range(len(tq))])
        self.qwts = np.array([tw[t] * lw[k] for k in range(m) for t in range(len(tq))])

    # ------------------------------------------------------------------ tet
    def _build_tet(self, tri_nodes):
        p = self.p
        tn = quadrature.triangle_nodes(p) if tri_nodes is None else np.asarray(tri_nodes, float)
        self.tri_nodes = tn
        self.nt = len(tn)
        self.upts = quadrature.tetrahedron_nodes(p)
        V = quadrature.TET_VERTS
        self.nfaces = 4
        # (vertices the reference triangle's (-1,-1), (1,-1), (-1,1) map to, normal)
        spec = [((0, 1, 2), (0.0, 0.0, -1.0)), ((0, 1, 3), (0.0, -1.0, 0.0)), ((0, 2, 3), (-1.0, 0.0, 0.0)),
                ((1, 2, 3), tuple(np.ones(3) / np.sqrt(3.0)))]
        faces = []
        for (a, b, c), nrm in spec:
            A, B, C = V[a], V[b], V[c]

            def tmap(s, t, A=A, B=B, C=C):
                s, t = np.asarray(s, float), np.asarray(t, float)
                la, lb, lc = -(s + t) / 2.0, (1.0 + s) / 2.0, (1.0 + t) / 2.0
                return la[:, None] * A + lb[:, None] * B + lc[:, None] * C
            jac = np.linalg.norm(np.cross(B - A, C - A)) / 2.0 / 2.0  # face area / reference triangle area
            faces.append(dict(kind="tri", map=tmap, normal=np.array(nrm), jac=jac))
        self.faces = faces
        tq, tw = quadrature.triangle_conical(p + 1)
        fp, fid, fw = [], [], []
        for f, fc in enumerate(faces):
            if self.surf_aa:
                fp.append(fc["map"](tq[:, 0], tq[:, 1]))
                fw.append(tw * fc["jac"])
            else:
                fp.append(fc["map"](tn[:, 0], tn[:, 1]))
            fid += [f] * len(fp[-1])
        self.fpts = np.concatenate(fp)
        self.fface = np.array(fid)
        self.fnorm = np.array([faces[f]["normal"] for f in self.fface])
        if self.surf_aa:
            self.fwts = np.concatenate(fw)
        self.qpts, self.qwts = quadrature.tetrahedron_conical(p + 1)

    # -------------------------------------------------------------- pyramid
    def _build_pyr(self, tri_nodes):
        p, n = self.p, self.n
        if self.surf_aa:
            raise ValueError("pyramids: no surface-flux anti-aliasing")
        tn = quadrature.triangle_nodes(p) if tri_nodes is None else np.asarray(tri_nodes, float)
        self.tri_nodes = tn
        self.nt = len(tn)
        self.upts = quadrature.pyramid_nodes(p)
        V = quadrature.PYR_VERTS
        self.nfaces = 5

        def bmap(s, t):
            s, t = np.asarray(s, float), np.asarray(t, float)
            return np.stack([s, t, -np.ones_like(s)], axis=1)
        faces = [dict(kind="quad", map=bmap, normal=np.array([0.0, 0.0, -1.0]), jac=1.0)]
        for (a, b, c), nrm in [((0, 1, 4), (0.0, -2.0, 1.0)), ((1, 2, 4), (2.0, 0.0, 1.0)),
                               ((2, 3, 4), (0.0, 2.0, 1.0)), ((3, 0, 4), (-2.0, 0.0, 1.0))]:
            A, B, C = V[a], V[b], V[c]

            def tmap(s, t, A=A, B=B, C=C):
                s, t = np.asarray(s, float), np.asarray(t, float)
                la, lb, lc = -(s + t) / 2.0, (1.0 + s) / 2.0, (1.0 + t) / 2.0
                return la[:, None] * A + lb[:, None] * B + lc[:, None] * C
            jac = np.linalg.norm(np.cross(B - A, C - A)) / 2.0 / 2.0
            faces.append(dict(kind="tri", map=tmap, normal=np.array(nrm) / np.sqrt(5.0), jac=jac))
        self.faces = faces
        gl = self.gl
        s = np.array([gl[a] for b in range(n) for a in range(n)])
        t = np.array([gl[b] for b in range(n) for a in range(n)])
        fp = [bmap(s, t)] + [fc["map"](tn[:, 0], tn[:, 1]) for fc in faces[1:]]
        self.fpts = np.concatenate(fp)
        self.fface = np.concatenate([np.full(len(x), f) for f, x in enumerate(fp)])
        self.fnorm = np.array([faces[f]["normal"] for f in self.fface])
        self.qpts, self.qwts = quadrature.pyramid_conical(p + 1)

    def _quad_face_points(self, g1, w1=None):
        """Tensor points g1 x g1 on every (quadrilateral) face; with weights
        w1 the points are a face quadrature rule (surface-flux AA)."""
        k = len(g1)
        s = np.array([g1[a] for b in range(k) for a in range(k)])
        t = np.array([g1[b] for b in range(k) for a in range(k)])
        fp, fid, fw = [], [], []
        for f, fc in enumerate(self.faces):
            fp.append(fc["map"](s, t))
            fid += [f] * (k * k)
            if w1 is not None:
                fw.append(np.array([w1[a] * w1[b] for b in range(k) for a in range(k)]) * fc["jac"])
        self.fpts = np.concatenate(fp)
        self.fface = np.array(fid)
        self.fnorm = np.array([self.faces[f]["normal"] for f in self.fface])
        if w1 is not None:
            self.fwts = np.concatenate(fw)

    # ------------------------------------------------------------ operators
    def _build_operators(self):
        et, p, n = self.etype, self.p, self.n
        up = self.upts
        self.M0, _ = basis.nodal(et, p, up, self.fpts)
        _, Dg = basis.nodal(et, p, up, up)
        self.Dg = Dg
        Lq, _ = basis.nodal(et, p, up, self.qpts)
        self.M7 = Lq
        W = np.diag(self.qwts)
        mass = Lq.T @ W @ Lq
        self.mass = mass
        massinv = basis.inv(mass)
        self.M8 = massinv @ (Lq.T @ W)
        self.wu = Lq.T @ self.qwts

        if et == "pyr":
            # the pyramid space is not closed under differentiation, so the
            # strong form (M1 - M3 M2) M9 differs from its weak form there;
            # the weak form is kept (see rhs.py, step 10):
            #   Kq[d] = -Mass^-1 Dq_d^T W_q (nu x nq), Ku[d] = Kq[d] M7
            _, Dq = basis.nodal(et, p, up, self.qpts)
            self.Kq = np.stack([-massinv @ (Dq[d].T * np.asarray(self.qwts, dtype=basis.EXT)[None, :])
                                for d in range(3)])
            self.Ku = np.einsum("dsq,qu->dsu", self.Kq, Lq)
        if self.surf_aa:
            # flux points are face quadrature points: the lifting integral
            # taken with the face rule, E[u, f] = l_u(x^f) w_f
            E = self.M0.T * np.asarray(self.fwts, dtype=basis.EXT)[None, :]
            self.M3 = massinv @ E
            self.M6 = self.fnorm.T[:, None, :] * self.M3[None, :, :]
            return
        # DG lifting: E[u, f] = int_face(f) l_u l^face_f dS_ref
        E = np.zeros((self.nu, self.nf), dtype=basis.EXT)
        gl = self.gl
        for fidx, fc in enumerate(self.faces):
            cols = np.nonzero(self.fface == fidx)[0]
            if fc["kind"] == "quad":
                g, gw = quadrature.gauss_legendre(n + 1)
                s = np.array([g[a] for b in range(n + 1) for a in range(n + 1)])
                t = np.array([g[b] for b in range(n + 1) for a in range(n + 1)])
                w = np.array([gw[a] * gw[b] for b in range(n + 1) for a in range(n + 1)]) * fc["jac"]
                xs = fc["map"](s, t)
                Ls = basis.line_nodal(gl, s)
                Lt = basis.line_nodal(gl, t)
                lface = np.stack([Ls[:, a] * Lt[:, b] for b in range(n) for a in range(n)], axis=1)
            else:
                tq, tw = quadrature.triangle_conical(p + 1)
                xs = fc["map"](tq[:, 0], tq[:, 1])
                w = tw * fc["jac"]
                lface = basis.tri_nodal(p, self.tri_nodes, tq)
            Lv, _ = basis.nodal(et, p, up, xs)
            E[:, cols] = Lv.T @ (w[:, None] * lface)
        self.M3 = massinv @ E
        self.M6 = self.fnorm.T[:, None, :] * self.M3[None, :, :]
