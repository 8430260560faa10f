// Periodic box meshes and face connectivity (host).
//
// Cells c = i + nx (j + ny k).  Hexahedra are axis aligned.  A prism cell is
// split by the diagonal of its x-z face from (x0+h, z0) to (x0, z0+h) and
// extruded along y; the two prisms map the reference prism (triangle in
// (xi, eta), line in zeta) with positive Jacobian:
//   first : x = x0 + (eta+1) hx/2,      y = y0 + (zeta+1) hy/2, z = z0 + (xi+1) hz/2
//   second: x = x0 + hx - (eta+1) hx/2, y = y0 + (zeta+1) hy/2, z = z0 + hz - (xi+1) hz/2
// so every z = const cell face is a full prism quadrilateral and a mixed mesh
// (hexahedra below z = 0) is conforming.  A tetrahedron cell holds six
// tetrahedra: the Kuhn subdivision of the cube mirrored in x (unit
// coordinates u = ((x0+h-x)/h, (y-y0)/h, (z-z0)/h); for each order (a, b, c)
// of the axes the tetrahedron u_a >= u_b >= u_c with vertices 0, e_a,
// e_a + e_b, (1,1,1) mapped to the reference vertices V0..V3, V1 and V2
// swapped where that gives a negative Jacobian).  Opposite cell faces are cut
// along parallel diagonals (conforming across cells and the period), and the
// y faces along the prisms' diagonal (prism triangles meet tetrahedra in the
// prism/tet mesh, prisms below y = 0).  A pyramid cell holds six pyramids,
// one on each cell face f (x-, x+, y-, y+, z-, z+), apex at the cell centre C:
// reference (xi, eta, zeta) maps to B + xi e1 + eta e2 + (1+zeta)/2 (C - B),
// B the face centre, e1, e2 the face's half edges ordered so that e1 x e2
// points into the cell (x-: y, z; x+: z, y; y-: z, x; y+: x, z; z-: x, y;
// z+: y, x).  Bases meet hexahedron faces or other bases; the triangles meet
// the neighbouring pyramids of the same cell (hexahedra below z = 0 in the
// hex/pyramid mesh).  The hexahedron/pyramid/tetrahedron mesh (nz >= 3) has
// hexahedra in layers k < nz/2, Kuhn tetrahedron cells in the layers between
// nz/2 and nz-1, and transition cells in layer nz/2 and the last layer: a
// pyramid on the face towards the hexahedra (z-, or z+ in the last layer,
// which meets the first layer across the period) and the pyramids of the
// five other faces cut into two tetrahedra each along the face diagonal the
// Kuhn cells use (joining the corners with the smallest and the largest sum
// of the unit coordinates u); element order: the pyramid, then two
// tetrahedra per face in face order (the face's two other corners in
// lexicographic order of (x, y, z)).  The four-type mesh is that one where
// the cell centre has y >= 0; where y < 0 it has hexahedra in the layers
// k < nz/2 and prism cells above (their z faces are full quadrilaterals, their
// y faces cut like the Kuhn cells').
//
// Connectivity: faces are paired by their centroids modulo the period, then
// the points of each face pair are matched by coordinates (section 2.1: paired
// flux points coincide in physical space).  Of each pair, "L" is the element
// with the lower mesh-order index; for an element paired with itself, the
// face with the lexicographically smaller centroid.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <thread>

#include "fr_host.h"

namespace fr {

// run body(lo, hi, chunk) over [0, n) in contiguous chunks on up to 16 host
// threads (one chunk when n is small); returns the number of chunks
static int64_t chunk_len(int64_t n) {
  int nth = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 40000) nth = 1;
  return std::max<int64_t>(1, (n + nth - 1) / nth);
}

template <typename F>
static int parallel_chunks(int64_t n, F body) {
  const int64_t per = chunk_len(n);
  const bool serial = per >= n;
  std::vector<std::thread> th;
  int c = 0;
  for (int64_t lo = 0; lo < n; lo += per, ++c) {
    const int64_t hi = std::min(n, lo + per);
    if (serial) {
      body(lo, hi, c);
    } else {
      th.emplace_back(body, lo, hi, c);
    }
  }
  for (auto& t : th) t.join();
  return c;
}

// element type of cell (j, k): kind 2 has hexahedra where the cell centre
// has z < 0 and prisms elsewhere; kind 4 prisms where y < 0, tetrahedra
// elsewhere; kind 9 hexahedra where z < 0, pyramids elsewhere
// Cell codes: 0..3 one element type per cell; 4, 5 transition cells with the
// pyramid on the z- / z+ face.
constexpr int kTransDown = 4, kTransUp = 5;
static int cell_type(int j, int k, int ny, int nz, double lo, double hi, int kind) {
  if (kind == 10) return k < nz / 2 ? 0 : (k == nz / 2 ? kTransDown : (k == nz - 1 ? kTransUp : 2));
  if (kind == 11) {
    const double hy = (hi - lo) / ny;
    if ((lo + j * hy) + 0.5 * hy < 0.0) return k < nz / 2 ? 0 : 1;
    return cell_type(j, k, ny, nz, lo, hi, 10);
  }
  if (kind == 8) return 3;
  if (kind == 9) return cell_type(j, k, ny, nz, lo, hi, 2) == 0 ? 0 : 3;
  if (kind == 2) {
    const double hz = (hi - lo) / nz;
    return (lo + k * hz) + 0.5 * hz < 0.0 ? 0 : 1;
  }
  if (kind == 4) {
    const double hy = (hi - lo) / ny;
    return (lo + j * hy) + 0.5 * hy < 0.0 ? 1 : 2;
  }
  if (kind == 7) return cell_type(j, k, ny, nz, lo, hi, 2);
  return kind == 3 ? 2 : (kind >= 5 ? kind - 5 : kind);
}

static constexpr int kPerCell[NTYPES] = {1, 2, 6, 6};

void box_counts(int nx, int ny, int nz, double lo, double hi, int kind, int64_t nel[NTYPES]) {
  for (int t = 0; t < NTYPES; ++t) nel[t] = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      const int t = cell_type(j, k, ny, nz, lo, hi, kind);
      if (t >= kTransDown) {
        nel[3] += nx;
        nel[2] += (int64_t)nx * 10;
      } else {
        nel[t] += (int64_t)nx * kPerCell[t];
      }
    }
}

// vertices of the six tetrahedra of the cell at x0 (module header)
static void kuhn_tets(const double x0[3], const double h[3], double P[6][4][3]) {
  static const int order[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int o = 0; o < 6; ++o) {
    double u[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
    u[1][order[o][0]] = 1;
    u[2][order[o][0]] = 1;
    u[2][order[o][1]] = 1;
    for (int v = 0; v < 4; ++v) {
      P[o][v][0] = x0[0] + h[0] * (1.0 - u[v][0]);
      P[o][v][1] = x0[1] + h[1] * u[v][1];
      P[o][v][2] = x0[2] + h[2] * u[v][2];
    }
    double a[3], b[3], c[3];
    for (int d = 0; d < 3; ++d) {
      a[d] = P[o][1][d] - P[o][0][d];
      b[d] = P[o][2][d] - P[o][0][d];
      c[d] = P[o][3][d] - P[o][0][d];
    }
    const double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                       a[2] * (b[0] * c[1] - b[1] * c[0]);
    if (det < 0)
      for (int d = 0; d < 3; ++d) std::swap(P[o][1][d], P[o][2][d]);
  }
}

// vertex shape functions and their gradients (see Mesh::verts)
static int vertex_shape(int t, const double* xi, double* N, double (*dN)[3]) {
  if (t == 0) {
    for (int v = 0; v < 8; ++v) {
      const double s[3] = {v & 1 ? 1.0 : -1.0, v & 2 ? 1.0 : -1.0, v & 4 ? 1.0 : -1.0};
      const double f[3] = {0.5 * (1 + s[0] * xi[0]), 0.5 * (1 + s[1] * xi[1]), 0.5 * (1 + s[2] * xi[2])};
      N[v] = f[0] * f[1] * f[2];
      dN[v][0] = 0.5 * s[0] * f[1] * f[2];
      dN[v][1] = 0.5 * f[0] * s[1] * f[2];
      dN[v][2] = 0.5 * f[0] * f[1] * s[2];
    }
    return 8;
  }
  const double lam[3] = {-(xi[0] + xi[1]) / 2, (1 + xi[0]) / 2, (1 + xi[1]) / 2};
  const double dl[3][2] = {{-0.5, -0.5}, {0.5, 0.0}, {0.0, 0.5}};
  for (int c = 0; c < 2; ++c)
    for (int tv = 0; tv < 3; ++tv) {
      const int v = tv + 3 * c;
      const double zf = c ? 0.5 * (1 + xi[2]) : 0.5 * (1 - xi[2]);
      N[v] = lam[tv] * zf;
      dN[v][0] = dl[tv][0] * zf;
      dN[v][1] = dl[tv][1] * zf;
      dN[v][2] = lam[tv] * (c ? 0.5 : -0.5);
    }
  return 6;
}

void map_point(const Mesh& m, int t, int64_t e, const double* xi, double* x) {
  if (m.curved && t < 2) {
    double N[8], dN[8][3];
    const int nv = vertex_shape(t, xi, N, dN);
    const double* X = &m.verts[t][3 * nv * e];
    for (int d = 0; d < 3; ++d) x[d] = 0;
    for (int v = 0; v < nv; ++v)
      for (int d = 0; d < 3; ++d) x[d] += N[v] * X[3 * v + d];
    return;
  }
  const double* A = &m.jac[t][9 * e];
  const double* o = &m.org[t][3 * e];
  for (int d = 0; d < 3; ++d) x[d] = o[d] + A[3 * d] * xi[0] + A[3 * d + 1] * xi[1] + A[3 * d + 2] * xi[2];
}

void jac_point(const Mesh& m, int t, int64_t e, const double* xi, double J[9]) {
  if (m.curved && t < 2) {
    double N[8], dN[8][3];
    const int nv = vertex_shape(t, xi, N, dN);
    const double* X = &m.verts[t][3 * nv * e];
    for (int k = 0; k < 9; ++k) J[k] = 0;
    for (int v = 0; v < nv; ++v)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[3 * i + j] += dN[v][j] * X[3 * v + i];
    return;
  }
  for (int k = 0; k < 9; ++k) J[k] = m.jac[t][9 * e + k];
}

static std::string finish_mesh(Mesh& M, const RefElem* refs[NTYPES], const double lat[9], const double lo3[3],
                               double hmin);

std::string build_box_mesh(int nx, int ny, int nz, double lo, double hi, int p, int kind,
                           const RefElem* refs[NTYPES], Mesh& M) {
  M = Mesh();
  M.nx = nx;
  M.ny = ny;
  M.nz = nz;
  M.p = p;
  M.kind = kind;
  M.lo = lo;
  M.hi = hi;
  const double Lx = hi - lo;
  const double h[3] = {Lx / nx, Lx / ny, Lx / nz};
  int64_t g = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double x0[3] = {lo + i * h[0], lo + j * h[1], lo + k * h[2]};
        int t = cell_type(j, k, ny, nz, lo, hi, kind);
        double c[3] = {x0[0] + 0.5 * h[0], x0[1] + 0.5 * h[1], x0[2] + 0.5 * h[2]};
        // the pyramid on cell face (ax, sg) (sg = 0: minus side), apex at c
        auto pyramid = [&](int ax, int sg) {
          int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
          // e1 x e2 along the inward normal -(2 sg - 1) e_ax
          if ((sg == 0) != (ax != 1)) std::swap(t1, t2);
          double J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
          J[3 * t1 + 0] = 0.5 * h[t1];
          J[3 * t2 + 1] = 0.5 * h[t2];
          J[3 * ax + 2] = (sg ? -0.25 : 0.25) * h[ax];  // (C - B)/2
          for (int d = 0; d < 3; ++d) M.org[3].push_back(c[d] + (d == ax ? (sg ? 0.25 : -0.25) * h[ax] : 0.0));
          M.jac[3].insert(M.jac[3].end(), J, J + 9);
          M.gid[3].push_back(g++);
        };
        // a tetrahedron of vertices P (positive orientation enforced)
        auto tetra = [&](double P[4][3]) {
          double a[3], b[3], cc[3];
          for (int d = 0; d < 3; ++d) {
            a[d] = P[1][d] - P[0][d];
            b[d] = P[2][d] - P[0][d];
            cc[d] = P[3][d] - P[0][d];
          }
          const double det = a[0] * (b[1] * cc[2] - b[2] * cc[1]) - a[1] * (b[0] * cc[2] - b[2] * cc[0]) +
                             a[2] * (b[0] * cc[1] - b[1] * cc[0]);
          if (det < 0)
            for (int d = 0; d < 3; ++d) std::swap(P[1][d], P[2][d]);
          // x = P0 + J (xi + 1): columns (P_v - P0)/2; origin at xi = 0
          double J[9];
          for (int d = 0; d < 3; ++d)
            for (int v = 0; v < 3; ++v) J[3 * d + v] = 0.5 * (P[v + 1][d] - P[0][d]);
          for (int d = 0; d < 3; ++d) M.org[2].push_back(P[0][d] + J[3 * d] + J[3 * d + 1] + J[3 * d + 2]);
          M.jac[2].insert(M.jac[2].end(), J, J + 9);
          M.gid[2].push_back(g++);
        };
        if (t == 3) {
          for (int ax = 0; ax < 3; ++ax)
            for (int sg = 0; sg < 2; ++sg) pyramid(ax, sg);
        } else if (t >= kTransDown) {
          const int bsg = t == kTransUp ? 1 : 0;
          pyramid(2, bsg);
          for (int ax = 0; ax < 3; ++ax)
            for (int sg = 0; sg < 2; ++sg) {
              if (ax == 2 && sg == bsg) continue;
              // the face's corners in Kuhn unit coordinates u (u_x = (x0 + h - x)/h),
              // ordered by the sum of u: the diagonal joins the first and last
              double u[4][3];
              for (int q = 0; q < 4; ++q) {
                int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;
                double w[3];
                w[ax] = sg ? 1.0 : 0.0;
                w[o0] = q & 1;
                w[o1] = (q >> 1) & 1;
                u[q][0] = 1.0 - w[0];  // w: unit coordinates along +x, +y, +z
                u[q][1] = w[1];
                u[q][2] = w[2];
              }
              int ord[4] = {0, 1, 2, 3};
              std::sort(ord, ord + 4, [&](int a, int b) {
                return u[a][0] + u[a][1] + u[a][2] < u[b][0] + u[b][1] + u[b][2];
              });
              auto X = [&](int q, double* x) {
                x[0] = x0[0] + h[0] * (1.0 - u[q][0]);
                x[1] = x0[1] + h[1] * u[q][1];
                x[2] = x0[2] + h[2] * u[q][2];
              };
              // the two other corners in lexicographic order of (x, y, z)
              double m1[3], m2[3];
              X(ord[1], m1);
              X(ord[2], m2);
              if (std::lexicographical_compare(m2, m2 + 3, m1, m1 + 3)) std::swap(ord[1], ord[2]);
              for (int other = 1; other <= 2; ++other) {
                double P[4][3];
                X(ord[0], P[0]);
                X(ord[3], P[1]);
                X(ord[other], P[2]);
                for (int d = 0; d < 3; ++d) P[3][d] = c[d];
                tetra(P);
              }
            }
        } else if (t == 2) {
          double P[6][4][3];
          kuhn_tets(x0, h, P);
          for (int o = 0; o < 6; ++o) {
            // x = P0 + J (xi + 1): columns (P_v - P0)/2; origin at xi = 0
            double J[9];
            for (int d = 0; d < 3; ++d)
              for (int v = 0; v < 3; ++v) J[3 * d + v] = 0.5 * (P[o][v + 1][d] - P[o][0][d]);
            for (int d = 0; d < 3; ++d) M.org[2].push_back(P[o][0][d] + J[3 * d] + J[3 * d + 1] + J[3 * d + 2]);
            M.jac[2].insert(M.jac[2].end(), J, J + 9);
            M.gid[2].push_back(g++);
          }
        } else if (t == 0) {
          for (int d = 0; d < 3; ++d) M.org[0].push_back(c[d]);
          double J[9] = {0.5 * h[0], 0, 0, 0, 0.5 * h[1], 0, 0, 0, 0.5 * h[2]};
          M.jac[0].insert(M.jac[0].end(), J, J + 9);
          M.gid[0].push_back(g++);
        } else {
          for (int s = 0; s < 2; ++s) {
            double sg = s ? -1.0 : 1.0;
            for (int d = 0; d < 3; ++d) M.org[1].push_back(c[d]);
            double J[9] = {0, sg * 0.5 * h[0], 0, 0, 0, 0.5 * h[1], sg * 0.5 * h[2], 0, 0};
            M.jac[1].insert(M.jac[1].end(), J, J + 9);
            M.gid[1].push_back(g++);
          }
        }
      }
  M.curved = kind_curved(kind);
  if (M.curved) {
    // vertices: the affine images of the reference vertices (cell corners),
    // moved by the warp field x + w h (sin y cos z, sin z cos x, sin x cos y)
    static const double kRefV[2][8][3] = {
        {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}, {1, 1, 1}},
        {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}, {0, 0, 0}, {0, 0, 0}}};
    for (int t = 0; t < 2; ++t) {
      const int nv = t == 0 ? 8 : 6;
      const int64_t E = (int64_t)M.gid[t].size();
      M.verts[t].resize(3 * nv * E);
      for (int64_t e = 0; e < E; ++e)
        for (int v = 0; v < nv; ++v) {
          const double* A = &M.jac[t][9 * e];
          const double* o = &M.org[t][3 * e];
          const double* xi = kRefV[t][v];
          double x[3];
          for (int d = 0; d < 3; ++d) x[d] = o[d] + A[3 * d] * xi[0] + A[3 * d + 1] * xi[1] + A[3 * d + 2] * xi[2];
          double* X = &M.verts[t][3 * (nv * e + v)];
          X[0] = x[0] + kWarp * h[0] * std::sin(x[1]) * std::cos(x[2]);
          X[1] = x[1] + kWarp * h[1] * std::sin(x[2]) * std::cos(x[0]);
          X[2] = x[2] + kWarp * h[2] * std::sin(x[0]) * std::cos(x[1]);
        }
      // the maps must keep a positive Jacobian at the vertices and centre
      for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k <= nv; ++k) {
          const double c0[3] = {0, 0, 0}, cp[3] = {-1.0 / 3.0, -1.0 / 3.0, 0};
          const double* xi = k < nv ? kRefV[t][k] : (t == 0 ? c0 : cp);
          double J[9];
          jac_point(M, t, e, xi, J);
          const double d = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                           J[2] * (J[3] * J[7] - J[4] * J[6]);
          if (!(d > 0)) return "non-positive Jacobian";
        }
    }
  }
  const double lat[9] = {Lx, 0, 0, 0, Lx, 0, 0, 0, Lx};
  const double lo3[3] = {lo, lo, lo};
  return finish_mesh(M, refs, lat, lo3, std::min(h[0], std::min(h[1], h[2])));
}

// Metrics, face slots, face pairing by centroid modulo the period lattice
// (lattice coordinates quantised to 2^-24 of a period), L/R, point
// permutations and normals of a mesh whose elements are set (org, jac, gid,
// verts).  lat: period vectors (rows); lo3: an origin of the quantisation;
// hmin: the smallest element size (tolerances).
static std::string finish_mesh(Mesh& M, const RefElem* refs[NTYPES], const double lat[9], const double lo3[3],
                               double hmin) {
  for (int t = 0; t < NTYPES; ++t) {
    M.nel[t] = (int64_t)M.gid[t].size();
    M.jinv[t].resize(9 * M.nel[t]);
    M.detj[t].resize(M.nel[t]);
    for (int64_t e = 0; e < M.nel[t]; ++e) {
      const double* A = &M.jac[t][9 * e];
      double d = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
      if (!(d > 0)) return "non-positive Jacobian";
      M.detj[t][e] = d;
      double* B = &M.jinv[t][9 * e];
      B[0] = (A[4] * A[8] - A[5] * A[7]) / d;
      B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
      B[2] = (A[1] * A[5] - A[2] * A[4]) / d;
      B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
      B[4] = (A[0] * A[8] - A[2] * A[6]) / d;
      B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
      B[6] = (A[3] * A[7] - A[4] * A[6]) / d;
      B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
      B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
    }
  }
  M.slot_base[0] = 0;
  for (int t = 1; t < NTYPES; ++t) M.slot_base[t] = M.slot_base[t - 1] + M.nel[t - 1] * kFacesOf[t - 1];
  M.nslots = M.slot_base[NTYPES - 1] + M.nel[NTYPES - 1] * kFacesOf[NTYPES - 1];
  const int64_t S = M.nslots;
  M.slot_po.resize(S);
  {
    int64_t po = 0, s = 0;
    for (int t = 0; t < NTYPES; ++t)
      for (int64_t e = 0; e < M.nel[t]; ++e)
        for (int f = 0; f < kFacesOf[t]; ++f) {
          M.slot_po[s++] = po;
          po += face_npts(t, f, M.p);
        }
    M.npts = po;
  }

  // lattice coordinates: c_lat = B (c - lo), B the inverse of the matrix
  // whose columns are the period vectors
  double B[9];
  {
    const double* L = lat;  // rows: period vectors; the matrix A = L^T
    const double a0 = L[0], a1 = L[3], a2 = L[6], b0 = L[1], b1 = L[4], b2 = L[7], c0 = L[2], c1 = L[5], c2 = L[8];
    // A = [[a0 a1 a2], [b0 b1 b2], [c0 c1 c2]] (columns = period vectors)
    const double det = a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
    if (!(std::fabs(det) > 0)) return "degenerate period lattice";
    B[0] = (b1 * c2 - b2 * c1) / det;
    B[1] = (a2 * c1 - a1 * c2) / det;
    B[2] = (a1 * b2 - a2 * b1) / det;
    B[3] = (b2 * c0 - b0 * c2) / det;
    B[4] = (a0 * c2 - a2 * c0) / det;
    B[5] = (a2 * b0 - a0 * b2) / det;
    B[6] = (b0 * c1 - b1 * c0) / det;
    B[7] = (a1 * c0 - a0 * c1) / det;
    B[8] = (a0 * b1 - a1 * b0) / det;
  }
  // physical face points and centroids
  auto phys = [&](int t, int64_t e, const double* xi, double* x) { map_point(M, t, e, xi, x); };
  std::vector<double> cent(3 * S);
  std::vector<std::array<int64_t, 4>> keys(S);  // quantised centroid mod period, slot
  const double Q = double(1 << 24);
  auto slot_info = [&](int64_t s, int& t, int64_t& e, int& f) {
    t = 0;
    for (int u = 1; u < NTYPES; ++u)
      if (M.nel[u] > 0 && s >= M.slot_base[u]) t = u;
    int64_t r = s - M.slot_base[t];
    e = r / kFacesOf[t];
    f = int(r % kFacesOf[t]);
  };
  parallel_chunks(S, [&](int64_t s0, int64_t s1, int) {
  for (int64_t s = s0; s < s1; ++s) {
    int t, f;
    int64_t e;
    slot_info(s, t, e, f);
    const RefElem& R = *refs[t];
    double c[3] = {0, 0, 0};
    for (int q = 0; q < R.face_npts[f]; ++q) {
      double x[3];
      phys(t, e, &R.fpts[3 * (R.face_start[f] + q)], x);
      for (int d = 0; d < 3; ++d) c[d] += x[d] / R.face_npts[f];
    }
    std::array<int64_t, 4> k;
    for (int d = 0; d < 3; ++d) cent[3 * s + d] = c[d];
    for (int d = 0; d < 3; ++d) {
      const double cl = B[3 * d] * (c[0] - lo3[0]) + B[3 * d + 1] * (c[1] - lo3[1]) + B[3 * d + 2] * (c[2] - lo3[2]);
      int64_t v = (int64_t)std::llround(cl * Q);
      v %= (int64_t)Q;
      if (v < 0) v += (int64_t)Q;
      k[d] = v;
    }
    k[3] = s;
    keys[s] = k;
  }
  });
  {
    // chunks sorted on host threads, then merged pairwise
    parallel_chunks(S, [&](int64_t s0, int64_t s1, int) { std::sort(keys.begin() + s0, keys.begin() + s1); });
    for (int64_t w = chunk_len(S); w < S; w *= 2) {
      std::vector<std::thread> th;
      for (int64_t lo = 0; lo + w < S; lo += 2 * w) {
        const int64_t mid = lo + w, hi = std::min(S, lo + 2 * w);
        th.emplace_back([&keys, lo, mid, hi] {
          std::inplace_merge(keys.begin() + lo, keys.begin() + mid, keys.begin() + hi);
        });
      }
      for (auto& t : th) t.join();
    }
  }
  if (S % 2) return "odd number of faces";
  M.nbr_slot.assign(S, -1);
  M.perm_id.assign(S, 0);
  M.is_left.assign(S, 0);
  M.nrm.assign(3 * S, 0);
  M.mag.assign(S, 0);
  for (int64_t i = 0; i < S; i += 2) {
    const auto& a = keys[i];
    const auto& b = keys[i + 1];
    if (a[0] != b[0] || a[1] != b[1] || a[2] != b[2]) return "faces do not pair up (non-conforming mesh)";
    if (i + 2 < S && keys[i + 2][0] == a[0] && keys[i + 2][1] == a[1] && keys[i + 2][2] == a[2])
      return "more than two faces share a centroid";
    int64_t sa = a[3], sb = b[3];
    M.nbr_slot[sa] = sb;
    M.nbr_slot[sb] = sa;
  }
  // per pair: L/R and point permutation.  Chunks of slots run on host
  // threads, each with its own permutation table; the tables are merged in
  // slot order, so permutation ids are numbered by first appearance.
  struct Local {
    std::vector<std::vector<int>> perms;
    std::vector<int> pid;  // per slot of the chunk: index into perms
    std::string err;
  };
  std::vector<Local> loc(16);
  const int nchunk = parallel_chunks(S, [&](int64_t s0, int64_t s1, int chunk) {
    Local& L = loc[chunk];
    L.pid.assign(s1 - s0, -1);
    std::vector<int> last;  // face class -> local permutation id
    for (int64_t s = s0; s < s1; ++s) {
      int64_t o = M.nbr_slot[s];
      int t, f, to, fo;
      int64_t e, eo;
      slot_info(s, t, e, f);
      slot_info(o, to, eo, fo);
      const RefElem& R = *refs[t];
      const RefElem& RO = *refs[to];
      const int np = R.face_npts[f];
      if (RO.face_npts[fo] != np) {
        L.err = "paired faces have different point counts";
        return;
      }
      bool left;
      if (M.gid[t][e] != M.gid[to][eo]) {
        left = M.gid[t][e] < M.gid[to][eo];
      } else {
        const double* ca = &cent[3 * s];
        const double* cb = &cent[3 * o];
        left = std::lexicographical_compare(ca, ca + 3, cb, cb + 3);
      }
      M.is_left[s] = left ? 1 : 0;
      // try the permutation found last for this (type, face, type, face)
      // class first; search by brute force only when it does not match
      auto dist2 = [&](int q, int r) {
        double x[3], y[3];
        phys(t, e, &R.fpts[3 * (R.face_start[f] + q)], x);
        phys(to, eo, &RO.fpts[3 * (RO.face_start[fo] + r)], y);
        // minimum image in lattice coordinates
        double dl[3];
        for (int d = 0; d < 3; ++d) {
          dl[d] = B[3 * d] * (x[0] - y[0]) + B[3 * d + 1] * (x[1] - y[1]) + B[3 * d + 2] * (x[2] - y[2]);
          dl[d] -= std::nearbyint(dl[d]);
        }
        double d2 = 0;
        for (int d = 0; d < 3; ++d) {
          const double dd = lat[d] * dl[0] + lat[3 + d] * dl[1] + lat[6 + d] * dl[2];
          d2 += dd * dd;
        }
        return d2;
      };
      const double tol = 1e-9 * hmin, tol2 = tol * tol;
      const int cls = ((t * 8 + f) * NTYPES + to) * 8 + fo;
      int pid = cls < (int)last.size() ? last[cls] : -1;
      if (pid >= 0) {
        const std::vector<int>& pm = L.perms[pid];
        for (int q = 0; q < np && pid >= 0; ++q)
          if (dist2(q, pm[q]) > tol2) pid = -1;
      }
      if (pid < 0) {
        std::vector<int> perm(np, -1);
        for (int q = 0; q < np; ++q) {
          double best = 1e300;
          int bi = -1;
          for (int r = 0; r < np; ++r) {
            const double d = dist2(q, r);
            if (d < best) {
              best = d;
              bi = r;
            }
          }
          if (best > tol2) {
            L.err = "paired flux points do not coincide";
            return;
          }
          perm[q] = bi;
        }
        std::vector<int> chk(perm);
        std::sort(chk.begin(), chk.end());
        for (int q = 0; q < np; ++q)
          if (chk[q] != q) {
            L.err = "flux-point matching is not one-to-one";
            return;
          }
        pid = (int)(std::find(L.perms.begin(), L.perms.end(), perm) - L.perms.begin());
        if (pid == (int)L.perms.size()) L.perms.push_back(perm);
        if (cls >= (int)last.size()) last.resize(cls + 1, -1);
        last[cls] = pid;
      }
      L.pid[s - s0] = pid;
    }
  });
  {
    std::map<std::vector<int>, int> permidx;
    int64_t s = 0;
    for (int c = 0; c < nchunk; ++c) {
      const Local& L = loc[c];
      if (!L.err.empty()) return L.err;
      std::vector<int> l2g(L.perms.size(), -1);
      for (int lid : L.pid) {
        if (l2g[lid] < 0) {
          auto it = permidx.find(L.perms[lid]);
          if (it == permidx.end()) {
            it = permidx.emplace(L.perms[lid], (int)M.perms.size()).first;
            M.perms.push_back(L.perms[lid]);
          }
          l2g[lid] = it->second;
        }
        M.perm_id[s++] = l2g[lid];
      }
    }
  }
  // normals: n = det J J^-T nhat / mag (Nanson).  The unit normal is the L
  // side's for both slots of a pair (both evaluate the common flux with the
  // same inputs); the area factor is each slot's own (the two differ where
  // the reference faces differ in size, e.g. a tetrahedron's slanted face
  // against an axis-aligned one)
  auto nanson = [&](int64_t s, double v[3]) {
    int t, f;
    int64_t e;
    slot_info(s, t, e, f);
    const double* B = &M.jinv[t][9 * e];
    const double* nh = &refs[t]->face_normal[3 * f];
    for (int c = 0; c < 3; ++c) v[c] = M.detj[t][e] * (B[0 * 3 + c] * nh[0] + B[1 * 3 + c] * nh[1] + B[2 * 3 + c] * nh[2]);
    return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  };
  parallel_chunks(S, [&](int64_t s0, int64_t s1, int) {
  for (int64_t s = s0; s < s1; ++s) {
    double v[3];
    M.mag[s] = nanson(s, v);
    if (!M.is_left[s]) nanson(M.nbr_slot[s], v);
    const double mg = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int c = 0; c < 3; ++c) M.nrm[3 * s + c] = v[c] / mg;
  }
  });
  return "";
}

// reference vertices of the affine element types, in the order in which
// fr_mesh_elements lists an element's vertices
static const double kElemRefV[NTYPES][8][3] = {
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}, {1, 1, 1}},
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}},
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}},
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}, {0, 0, 1}}};
static constexpr int kElemNV[NTYPES] = {8, 6, 4, 5};

std::string build_element_mesh(int p, const int64_t n_elem[NTYPES], const double* const verts[NTYPES],
                               const double* period, const RefElem* refs[NTYPES], Mesh& M) {
  M = Mesh();
  M.p = p;
  M.kind = -1;
  double lo3[3] = {1e300, 1e300, 1e300}, hi3[3] = {-1e300, -1e300, -1e300};
  double hmin = 1e300;
  int64_t g = 0;
  for (int t = 0; t < NTYPES; ++t) {
    const int nv = kElemNV[t];
    const double(*rv)[3] = kElemRefV[t];
    // the affine fit x = org + J xi: least squares over the vertices (the
    // normal equations of [1, xi] are exact here), then every vertex checked
    double G[4][4] = {}, Gi[4][4];
    for (int v = 0; v < nv; ++v) {
      const double a[4] = {1, rv[v][0], rv[v][1], rv[v][2]};
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) G[i][j] += a[i] * a[j];
    }
    // Gauss-Jordan inverse of the 4x4 Gram matrix
    double W[4][8];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 8; ++j) W[i][j] = j < 4 ? G[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int c = 0; c < 4; ++c) {
      int piv = c;
      for (int r = c + 1; r < 4; ++r)
        if (std::fabs(W[r][c]) > std::fabs(W[piv][c])) piv = r;
      for (int j = 0; j < 8; ++j) std::swap(W[c][j], W[piv][j]);
      const double d = W[c][c];
      for (int j = 0; j < 8; ++j) W[c][j] /= d;
      for (int r = 0; r < 4; ++r)
        if (r != c) {
          const double f = W[r][c];
          for (int j = 0; j < 8; ++j) W[r][j] -= f * W[c][j];
        }
    }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) Gi[i][j] = W[i][4 + j];
    const int64_t E = n_elem[t];
    for (int64_t e = 0; e < E; ++e) {
      const double* X = verts[t] + (size_t)e * nv * 3;
      double c[4][3] = {};  // rows: org, then the columns of J
      for (int v = 0; v < nv; ++v) {
        const double a[4] = {1, rv[v][0], rv[v][1], rv[v][2]};
        for (int i = 0; i < 4; ++i) {
          double w = 0;
          for (int j = 0; j < 4; ++j) w += Gi[i][j] * a[j];
          for (int d = 0; d < 3; ++d) c[i][d] += w * X[3 * v + d];
        }
      }
      double size = 0, mis = 0;
      for (int v = 0; v < nv; ++v)
        for (int u = 0; u < nv; ++u) {
          double d2 = 0;
          for (int d = 0; d < 3; ++d) d2 += (X[3 * v + d] - X[3 * u + d]) * (X[3 * v + d] - X[3 * u + d]);
          size = std::max(size, std::sqrt(d2));
        }
      for (int v = 0; v < nv; ++v)
        for (int d = 0; d < 3; ++d) {
          const double x = c[0][d] + c[1][d] * rv[v][0] + c[2][d] * rv[v][1] + c[3][d] * rv[v][2];
          mis = std::max(mis, std::fabs(x - X[3 * v + d]));
          lo3[d] = std::min(lo3[d], X[3 * v + d]);
          hi3[d] = std::max(hi3[d], X[3 * v + d]);
        }
      if (!(size > 0) || !std::isfinite(mis)) return "degenerate element";
      if (mis > 1e-10 * size) return "element is not the affine image of the reference element";
      for (int d = 0; d < 3; ++d) M.org[t].push_back(c[0][d]);
      double J[9];
      for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) J[3 * d + k] = c[1 + k][d];
      M.jac[t].insert(M.jac[t].end(), J, J + 9);
      M.gid[t].push_back(g++);
      for (int k = 0; k < 3; ++k)
        hmin = std::min(hmin, std::sqrt(J[k] * J[k] + J[3 + k] * J[3 + k] + J[6 + k] * J[6 + k]));
    }
  }
  if (g == 0) return "no elements";
  double lat[9];
  if (period) {
    for (int k = 0; k < 9; ++k) lat[k] = period[k];
  } else {
    // no period: a lattice far larger than the mesh never wraps a face
    for (int k = 0; k < 9; ++k) lat[k] = 0;
    for (int d = 0; d < 3; ++d) lat[4 * d] = 4.0 * (hi3[d] - lo3[d]) + 1.0;
  }
  return finish_mesh(M, refs, lat, lo3, hmin);
}

bool prism_tri_faces_aligned(const Mesh& m) {
  std::vector<char> checked(m.perms.size(), 0), ok(m.perms.size(), 1);
  for (int64_t e = 0; e < m.nel[1]; ++e)
    for (int f = 0; f < 2; ++f) {
      const int id = m.perm_id[m.slot_base[1] + e * 5 + f];
      if (!checked[id]) {
        checked[id] = 1;
        const std::vector<int>& pm = m.perms[id];
        for (size_t r = 0; r < pm.size(); ++r)
          if (pm[r] != (int)r) ok[id] = 0;
      }
      if (!ok[id]) return false;
    }
  return true;
}

}  // namespace fr
