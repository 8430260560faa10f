// Host-side data structures of the flux-reconstruction library: reference
// elements with their factorised operators, and the periodic box mesh with
// its face connectivity.  No device code here.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fr {

// 1-D operators on Gauss-Legendre solution points (n = p+1) and m GL
// quadrature points.  These are the factors of the hex operators
// (section 4: M7 and M9 factor into per-direction sparse sweeps).
struct Line1D {
  int n = 0, m = 0;
  std::vector<double> x, w;    // GL(n) nodes and weights
  std::vector<double> xq, wq;  // GL(m)
  std::vector<double> D;       // n x n  D[i][j] = l_j'(x_i)
  std::vector<double> I;       // m x n  I[a][i] = l_i(xq_a)
  std::vector<double> Dq;      // m x n  l_i'(xq_a)
  std::vector<double> P;       // n x m  L2 projection  I^T W_q / w_i
  std::vector<double> AP;      // n x m  -(Dq^T W_q)/w_i : projection followed by the
                               //        SBP form of (M1 - M3 M2) along the line
  std::vector<double> APu;     // n x n  -(D^T W)/w_i : the same at the solution points
                               //        (no anti-aliasing: flux collocated at GL(n))
  std::vector<double> lb, rb;  // l_i(-1), l_i(+1)
  std::vector<double> liftL, liftR;  // l_i(-1)/w_i, l_i(+1)/w_i  (DG correction)
};

// Triangle factors of the prism operators (section 4.1: block structured
// triangle-plane operator times a sparse line operator).
struct Tri {
  int p = 0, nt = 0, ntq = 0;
  std::vector<double> nodes;        // nt x 2
  std::vector<double> qp, qw;       // ntq x 2, ntq  (conical rule, degree 2p+1)
  std::vector<double> Tq;           // ntq x nt  l_t(q)
  std::vector<double> Dxi, Deta;    // nt x nt   derivatives of l_t at the nodes
  std::vector<double> DxiQ, DetaQ;  // ntq x nt  derivatives of l_t at q
  std::vector<double> mass, massInv;  // nt x nt
  std::vector<double> PT;           // nt x ntq  M_T^-1 Tq^T W
  std::vector<double> APxi, APeta;  // nt x ntq  -M_T^-1 DQ^T W
  std::vector<double> Tedge;        // 3 x n x nt   l_t at the GL points of each edge
  std::vector<double> LiftEdge;     // 3 x nt x n   M_T^-1 Tedge^T diag(w) |edge jac|
  double edgeJac[3] = {1, 1, 1};
  double edgeNormal[3][2] = {{0, -1}, {0, 0}, {-1, 0}};
};

// Geometry of a reference element (hex, prism, tet or pyramid) and its dense
// operators.  etype: 0 hex, 1 prism, 2 tet, 3 pyramid.
struct RefElem {
  int etype = 0, p = 0, n = 0, m = 0;
  int nu = 0, nf = 0, nq = 0, nfaces = 0, nfp_max = 0;
  Line1D line;
  Tri tri;  // prisms only
  std::vector<double> upts, fpts, qpts, qwts;  // N x 3 / N
  std::vector<int> face_start, face_npts;      // per face
  std::vector<double> face_normal;             // nfaces x 3, unit reference normals
  std::vector<double> face_jac;                // tets, pyramids: face area / reference face area
  std::vector<double> wu;                      // integrals of the nodal basis
  // dense operators of section 2.2 (row-major), built from the factors
  std::vector<double> M0, M3, M7, M8, Dg;  // Dg: 3 x nu x nu
  // tetrahedra and pyramids (no factorisation): projection-divergence per
  // reference direction, AP_d = -Mass^-1 Dq_d^T W_q (3 x nu x nq), and the
  // mass matrix; pyramids also Ku_d = AP_d M7 (3 x nu x nu), the divergence
  // of a flux held at the solution points (no anti-aliasing)
  std::vector<double> APd, mass, Ku;
};

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x, std::vector<double>& w);
void triangle_nodes(int p, std::vector<double>& xy);
void build_ref(int etype, int p, RefElem& r);

// element types of a mesh: 0 hexahedra, 1 prisms, 2 tetrahedra, 3 pyramids
constexpr int NTYPES = 4;
constexpr int kFacesOf[NTYPES] = {6, 5, 4, 5};
// flux points of face f of type t at order p: n^2 on a quadrilateral
// (hexahedron faces, prism faces 2..4, the pyramid base), n(n+1)/2 on a
// triangle (prism faces 0, 1, tetrahedron faces, pyramid faces 1..4)
inline int face_npts(int t, int f, int p) {
  const int n = p + 1;
  const bool quad = t == 0 || (t == 1 && f >= 2) || (t == 3 && f == 0);
  return quad ? n * n : n * (n + 1) / 2;
}
// box mesh kinds: 0 hex, 1 prism, 2 hex (z < 0) + prism, 3 tet,
// 4 prism (y < 0) + tet; 5, 6, 7: kinds 0, 1, 2 on the warped grid (curved);
// 8 pyramid (six per cell), 9 hex (z < 0) + pyramid, 10 hex + pyramid +
// tetrahedron (transition cells, nz >= 3), 11 kind 10 with prisms where y < 0
constexpr int kNumKinds = 12;
inline bool kind_curved(int kind) { return kind >= 5 && kind <= 7; }
// kinds with tetrahedra or pyramids (dense-operator element types)
inline bool kind_dense(int kind) { return kind == 3 || kind == 4 || kind >= 8; }
// vertex displacement of the warped grid, in cell sizes
constexpr double kWarp = 0.2;

// Periodic box mesh with face connectivity.
struct Mesh {
  int nx = 0, ny = 0, nz = 0, p = 0, kind = 0;  // kind -1: a mesh from element vertices
  double lo = 0, hi = 0;
  int64_t nel[NTYPES] = {};
  std::vector<double> org[NTYPES];    // element origin (x at reference 0)
  std::vector<double> jac[NTYPES];    // J (3x3 row-major, rows x,y,z cols xi,eta,zeta)
  std::vector<double> jinv[NTYPES];   // J^-1
  std::vector<double> detj[NTYPES];
  std::vector<int64_t> gid[NTYPES];   // mesh-order index
  // face slots: type t, element e, face f at slot_base[t] + e * kFacesOf[t] + f
  int64_t slot_base[NTYPES] = {};
  int64_t nslots = 0;
  std::vector<int64_t> nbr_slot;  // paired slot
  // face data (states, viscous fluxes) are stored per slot with the slot's
  // own number of points: slot s starts at point slot_po[s]; npts in all
  std::vector<int64_t> slot_po;
  int64_t npts = 0;
  std::vector<int32_t> perm_id;   // own point r -> neighbour point perms[perm_id][r]
  std::vector<uint8_t> is_left;
  // curved meshes: the vertices of every element, [E][nv][3] per type
  // (hexahedra: 8, vertex a + 2b + 4c at reference corner (2a-1, 2b-1, 2c-1),
  // trilinear map; prisms: 6, vertex t + 3c at triangle vertex t of
  // (-1,-1), (1,-1), (-1,1) and zeta = 2c-1, map lambda_t(xi, eta)(1 -+ zeta)/2);
  // jac/jinv/detj then hold the undeformed element's
  bool curved = false;
  std::vector<double> verts[NTYPES];
  std::vector<double> nrm;        // per slot: L-side physical unit normal (3)
  std::vector<double> mag;        // per slot: the slot's own area factor |det J J^-T n|
  std::vector<std::vector<int>> perms;
};

// physical point and Jacobian J[i][j] = d x_i / d xi_j of element e of type t
// at reference point xi (affine, or the trilinear map of a curved mesh)
void map_point(const Mesh& m, int t, int64_t e, const double* xi, double* x);
void jac_point(const Mesh& m, int t, int64_t e, const double* xi, double J[9]);

// element counts per type of a box mesh (same cell typing as build_box_mesh)
void box_counts(int nx, int ny, int nz, double lo, double hi, int kind, int64_t nel[NTYPES]);

// True if every prism triangle face sees its neighbour's triangle nodes in
// the same order (identity point permutation), as surface-flux
// anti-aliasing on the (unsymmetric) triangle quadrature rule requires.
bool prism_tri_faces_aligned(const Mesh& m);

// Build the box mesh and its connectivity; returns an error string or "".
std::string build_box_mesh(int nx, int ny, int nz, double lo, double hi, int p, int kind,
                           const RefElem* refs[NTYPES], Mesh& m);

// Build a conforming mesh of affine elements from their vertices (n_elem[t]
// elements of type t, verts[t] of n_elem[t] x nv x 3 doubles, the vertex
// orders of fr_mesh_elements) with an optional period lattice (9 doubles, the
// rows the period vectors; null: no period); returns an error string or "".
std::string build_element_mesh(int p, const int64_t n_elem[NTYPES], const double* const verts[NTYPES],
                               const double* period, const RefElem* refs[NTYPES], Mesh& m);

}  // namespace fr
