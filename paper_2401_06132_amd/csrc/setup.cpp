// Reference elements and their operators (host).
//
// Points: Gauss-Legendre roots by bracketing + Newton on the three-term
// recurrence; Gauss-Jacobi(1,0) likewise with the closed-form weights.
// Lines: Lagrange polynomials evaluated by their product formula.
// Triangles: the Proriol-Koornwinder-Dubiner basis (Jacobi polynomials in
// collapsed coordinates) for the nodal Vandermonde.
// Operators follow section 2.2 (M0, M3, M7, M8, gradients) with the DG
// correction functions; the factored forms follow section 4 (hex: three 1-D
// sweeps) and section 4.1 (prism: triangle-plane block times line).
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "fr_host.h"

namespace fr {

namespace {

// P_n^{(a,b)}(x) and its derivative by the standard recurrence.
void jacobi(int n, double a, double b, double x, double& pn, double& dpn) {
  auto val = [&](int k, double aa, double bb) {
    if (k == 0) return 1.0;
    double p0 = 1.0, p1 = 0.5 * ((aa + bb + 2.0) * x + (aa - bb));
    for (int j = 2; j <= k; ++j) {
      double c = 2.0 * j + aa + bb;
      double a1 = 2.0 * j * (j + aa + bb) * (c - 2.0);
      double a2 = (c - 1.0) * (aa * aa - bb * bb);
      double a3 = (c - 2.0) * (c - 1.0) * c;
      double a4 = 2.0 * (j + aa - 1.0) * (j + bb - 1.0) * c;
      double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
      p0 = p1;
      p1 = p2;
    }
    return p1;
  };
  pn = val(n, a, b);
  dpn = n == 0 ? 0.0 : 0.5 * (n + a + b + 1.0) * val(n - 1, a + 1.0, b + 1.0);
}

void roots(int n, double a, double b, std::vector<double>& x) {
  x.clear();
  const int ns = 4000;
  double pa, d;
  jacobi(n, a, b, -1.0, pa, d);
  double xa = -1.0;
  for (int s = 1; s <= ns; ++s) {
    double xb = -1.0 + 2.0 * s / ns, pb;
    jacobi(n, a, b, xb, pb, d);
    if (pb == 0.0) {
      x.push_back(xb);  // exact root on a sample point (e.g. x = 0 for odd n)
    } else if (pa != 0.0 && (pa < 0) != (pb < 0)) {
      double lo = xa, hi = xb, flo = pa;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi), fm;
        jacobi(n, a, b, mid, fm, d);
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      double r = 0.5 * (lo + hi);
      for (int it = 0; it < 3; ++it) {
        double f, df;
        jacobi(n, a, b, r, f, df);
        if (df != 0) r -= f / df;
      }
      x.push_back(r);
    }
    xa = xb;
    pa = pb;
  }
  if ((int)x.size() != n) throw std::runtime_error("root finding failed");
}

double lagrange(const std::vector<double>& x, int j, double y) {
  double v = 1.0;
  for (size_t k = 0; k < x.size(); ++k)
    if ((int)k != j) v *= (y - x[k]) / (x[j] - x[k]);
  return v;
}

double dlagrange(const std::vector<double>& x, int j, double y) {
  double s = 0.0;
  for (size_t mm = 0; mm < x.size(); ++mm) {
    if ((int)mm == j) continue;
    double t = 1.0 / (x[j] - x[mm]);
    for (size_t k = 0; k < x.size(); ++k)
      if ((int)k != j && k != mm) t *= (y - x[k]) / (x[j] - x[k]);
    s += t;
  }
  return s;
}

// Dense inverse by Gauss-Jordan with partial pivoting (small matrices).
std::vector<double> inverse(std::vector<double> A, int n) {
  std::vector<double> B(n * n, 0.0);
  for (int i = 0; i < n; ++i) B[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) throw std::runtime_error("singular matrix");
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(B[c * n + k], B[piv * n + k]);
    }
    double d = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= d;
      B[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        B[r * n + k] -= f * B[c * n + k];
      }
    }
  }
  return B;
}

// PKD basis on the triangle {xi,eta >= -1, xi+eta <= 0}: mode (i,j), i+j <= p,
// psi = P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i with a = 2(1+xi)/(1-eta) - 1, b = eta.
// Points with eta = 1 (the top vertex) are never evaluated.
void pkd(int p, double xi, double eta, double* v, double* dxi, double* deta) {
  double b = eta, omb = 1.0 - b;
  double a = 2.0 * (1.0 + xi) / omb - 1.0;
  int k = 0;
  for (int j0 = 0; j0 <= p; ++j0) {
    for (int i = 0; i + j0 <= p; ++i) {
      int j = j0;
      double pa, dpa, pb, dpb;
      jacobi(i, 0.0, 0.0, a, pa, dpa);
      jacobi(j, 2.0 * i + 1.0, 0.0, b, pb, dpb);
      double w = std::pow(omb, i), wm1 = i > 0 ? std::pow(omb, i - 1) : 0.0;
      v[k] = pa * pb * w;
      dxi[k] = i > 0 ? 2.0 * dpa * pb * wm1 : 0.0;
      deta[k] = (i > 0 ? dpa * (1.0 + a) * pb * wm1 : 0.0) + pa * (dpb * w - (i > 0 ? i * pb * wm1 : 0.0));
      ++k;
    }
  }
}

}  // namespace

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) { gauss_jacobi(n, 0.0, 0.0, x, w); }

void gauss_jacobi(int n, double a, double b, std::vector<double>& x, std::vector<double>& w) {
  roots(n, a, b, x);
  w.resize(n);
  double c = std::pow(2.0, a + b + 1.0) * std::exp(std::lgamma(n + a + 1.0) + std::lgamma(n + b + 1.0) -
                                                    std::lgamma(n + a + b + 1.0) - std::lgamma(n + 1.0));
  for (int i = 0; i < n; ++i) {
    double f, df;
    jacobi(n, a, b, x[i], f, df);
    w[i] = c / ((1.0 - x[i] * x[i]) * df * df);
  }
}

void triangle_nodes(int p, std::vector<double>& xy) {
  // Blyth-Pozrikidis points from the Gauss-Legendre master grid
  std::vector<double> g, gw;
  gauss_legendre(p + 1, g, gw);
  std::vector<double> v(p + 1);
  for (int i = 0; i <= p; ++i) v[i] = 0.5 * (1.0 + g[i]);
  xy.clear();
  for (int j = 0; j <= p; ++j)
    for (int i = 0; i + j <= p; ++i) {
      int k = p - i - j;
      double X = (1.0 + 2.0 * v[i] - v[j] - v[k]) / 3.0;
      double Y = (1.0 + 2.0 * v[j] - v[i] - v[k]) / 3.0;
      xy.push_back(2.0 * X - 1.0);
      xy.push_back(2.0 * Y - 1.0);
    }
}

static void build_line(int p, int m, Line1D& L) {
  int n = p + 1;
  L.n = n;
  L.m = m;
  gauss_legendre(n, L.x, L.w);
  gauss_legendre(m, L.xq, L.wq);
  L.D.assign(n * n, 0);
  L.I.assign(m * n, 0);
  L.Dq.assign(m * n, 0);
  L.P.assign(n * m, 0);
  L.AP.assign(n * m, 0);
  L.APu.assign(n * n, 0);
  L.lb.resize(n);
  L.rb.resize(n);
  L.liftL.resize(n);
  L.liftR.resize(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) L.D[i * n + j] = dlagrange(L.x, j, L.x[i]);
  for (int a = 0; a < m; ++a)
    for (int i = 0; i < n; ++i) {
      L.I[a * n + i] = lagrange(L.x, i, L.xq[a]);
      L.Dq[a * n + i] = dlagrange(L.x, i, L.xq[a]);
    }
  for (int i = 0; i < n; ++i) {
    for (int a = 0; a < m; ++a) {
      L.P[i * m + a] = L.I[a * n + i] * L.wq[a] / L.w[i];
      L.AP[i * m + a] = -L.Dq[a * n + i] * L.wq[a] / L.w[i];
    }
    L.lb[i] = lagrange(L.x, i, -1.0);
    L.rb[i] = lagrange(L.x, i, 1.0);
    for (int j = 0; j < n; ++j) L.APu[i * n + j] = -L.D[j * n + i] * L.w[j] / L.w[i];
    L.liftL[i] = L.lb[i] / L.w[i];
    L.liftR[i] = L.rb[i] / L.w[i];
  }
}

static void build_tri(int p, const Line1D& L, Tri& T) {
  T.p = p;
  triangle_nodes(p, T.nodes);
  int nt = (p + 1) * (p + 2) / 2, n = p + 1;
  T.nt = nt;
  // conical rule with (p+1)^2 points: GL in a, Gauss-Jacobi(1,0) in b
  std::vector<double> ga, gwa, gb, gwb;
  gauss_legendre(p + 1, ga, gwa);
  gauss_jacobi(p + 1, 1.0, 0.0, gb, gwb);
  T.ntq = (p + 1) * (p + 1);
  for (int j = 0; j <= p; ++j)
    for (int i = 0; i <= p; ++i) {
      T.qp.push_back(0.5 * (1.0 + ga[i]) * (1.0 - gb[j]) - 1.0);
      T.qp.push_back(gb[j]);
      T.qw.push_back(0.5 * gwa[i] * gwb[j]);
    }
  int ntq = T.ntq;
  std::vector<double> V(nt * nt), v(nt), dx(nt), dy(nt);
  for (int t = 0; t < nt; ++t) {
    pkd(p, T.nodes[2 * t], T.nodes[2 * t + 1], v.data(), dx.data(), dy.data());
    for (int k = 0; k < nt; ++k) V[t * nt + k] = v[k];
  }
  std::vector<double> Vi = inverse(V, nt);
  // nodal basis at a point: l_t(y) = sum_k psi_k(y) Vi[k][t]
  auto nodal = [&](double xi, double eta, double* l, double* lx, double* ly) {
    pkd(p, xi, eta, v.data(), dx.data(), dy.data());
    for (int t = 0; t < nt; ++t) {
      double s = 0, sx = 0, sy = 0;
      for (int k = 0; k < nt; ++k) {
        s += v[k] * Vi[k * nt + t];
        sx += dx[k] * Vi[k * nt + t];
        sy += dy[k] * Vi[k * nt + t];
      }
      l[t] = s;
      if (lx) lx[t] = sx;
      if (ly) ly[t] = sy;
    }
  };
  T.Tq.assign(ntq * nt, 0);
  T.DxiQ.assign(ntq * nt, 0);
  T.DetaQ.assign(ntq * nt, 0);
  for (int q = 0; q < ntq; ++q)
    nodal(T.qp[2 * q], T.qp[2 * q + 1], &T.Tq[q * nt], &T.DxiQ[q * nt], &T.DetaQ[q * nt]);
  T.Dxi.assign(nt * nt, 0);
  T.Deta.assign(nt * nt, 0);
  std::vector<double> tmp(nt);
  for (int t = 0; t < nt; ++t) nodal(T.nodes[2 * t], T.nodes[2 * t + 1], tmp.data(), &T.Dxi[t * nt], &T.Deta[t * nt]);
  T.mass.assign(nt * nt, 0);
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b) {
      double s = 0;
      for (int q = 0; q < ntq; ++q) s += T.Tq[q * nt + a] * T.qw[q] * T.Tq[q * nt + b];
      T.mass[a * nt + b] = s;
    }
  T.massInv = inverse(T.mass, nt);
  T.PT.assign(nt * ntq, 0);
  T.APxi.assign(nt * ntq, 0);
  T.APeta.assign(nt * ntq, 0);
  for (int t = 0; t < nt; ++t)
    for (int q = 0; q < ntq; ++q) {
      double s = 0, sx = 0, sy = 0;
      for (int k = 0; k < nt; ++k) {
        s += T.massInv[t * nt + k] * T.Tq[q * nt + k];
        sx += T.massInv[t * nt + k] * T.DxiQ[q * nt + k];
        sy += T.massInv[t * nt + k] * T.DetaQ[q * nt + k];
      }
      T.PT[t * ntq + q] = s * T.qw[q];
      T.APxi[t * ntq + q] = -sx * T.qw[q];
      T.APeta[t * ntq + q] = -sy * T.qw[q];
    }
  // edges (counter-clockwise): e0 eta=-1 (xi=s); e1 hypotenuse (-s, s); e2 xi=-1 (-1, -s)
  T.edgeJac[0] = 1.0;
  T.edgeJac[1] = std::sqrt(2.0);
  T.edgeJac[2] = 1.0;
  T.edgeNormal[0][0] = 0.0;
  T.edgeNormal[0][1] = -1.0;
  T.edgeNormal[1][0] = 1.0 / std::sqrt(2.0);
  T.edgeNormal[1][1] = 1.0 / std::sqrt(2.0);
  T.edgeNormal[2][0] = -1.0;
  T.edgeNormal[2][1] = 0.0;
  T.Tedge.assign(3 * n * nt, 0);
  T.LiftEdge.assign(3 * nt * n, 0);
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < n; ++i) {
      double s = L.x[i];
      double xi = e == 0 ? s : (e == 1 ? -s : -1.0);
      double eta = e == 0 ? -1.0 : (e == 1 ? s : -s);
      nodal(xi, eta, &T.Tedge[(e * n + i) * nt], nullptr, nullptr);
    }
  for (int e = 0; e < 3; ++e)
    for (int t = 0; t < nt; ++t)
      for (int i = 0; i < n; ++i) {
        double s = 0;
        for (int k = 0; k < nt; ++k) s += T.massInv[t * nt + k] * T.Tedge[(e * n + i) * nt + k];
        T.LiftEdge[(e * nt + t) * n + i] = s * L.w[i] * T.edgeJac[e];
      }
}

// Tetrahedron {xi, eta, zeta >= -1, xi + eta + zeta <= -1} with vertices
// V0..V3 = (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).
static const double kTetV[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
// faces: the vertices the reference triangle's (-1,-1), (1,-1), (-1,1) map to
static const int kTetFace[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

// Pyramid: square base [-1,1]^2 at zeta = -1 (face 0), apex (0,0,1); the
// triangles (faces 1..4) run round the base counter-clockwise seen from above
static const double kPyrV[5][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1}, {0, 0, 1}};
static const int kPyrFace[4][3] = {{0, 1, 4}, {1, 2, 4}, {2, 3, 4}, {3, 0, 4}};

// solution points: barycentric Blyth-Pozrikidis-type construction on the GL
// master grid v = (1 + GL(p+1))/2: for i + j + k + l = p,
// lambda_a = (1 + 4 v_a - (v_i + v_j + v_k + v_l))/4 (l for V0, i, j, k for V1..V3)
static void tet_nodes(int p, std::vector<double>& x) {
  x.clear();
  if (p == 0) {
    x = {-0.5, -0.5, -0.5};
    return;
  }
  std::vector<double> g, gw;
  gauss_legendre(p + 1, g, gw);
  std::vector<double> v(p + 1);
  for (int i = 0; i <= p; ++i) v[i] = 0.5 * (1.0 + g[i]);
  for (int k = 0; k <= p; ++k)
    for (int j = 0; j + k <= p; ++j)
      for (int i = 0; i + j + k <= p; ++i) {
        const int idx[4] = {p - i - j - k, i, j, k};
        const double sum = v[idx[0]] + v[idx[1]] + v[idx[2]] + v[idx[3]];
        double c[3] = {0, 0, 0};
        for (int a = 0; a < 4; ++a) {
          const double lam = (1.0 + 4.0 * v[idx[a]] - sum) / 4.0;
          for (int d = 0; d < 3; ++d) c[d] += lam * kTetV[a][d];
        }
        x.insert(x.end(), c, c + 3);
      }
}

// The tetrahedron has no tensor structure, so its operators come from a
// Vandermonde inverse of the full P_p basis; that and the mass-matrix inverse
// run in long double (the Vandermonde's condition number reaches ~5e3 at
// p = 4) and the results are rounded once.
typedef long double xreal;

static std::vector<xreal> inverse_x(std::vector<xreal> A, int n) {
  std::vector<xreal> B(n * n, 0.0L);
  for (int i = 0; i < n; ++i) B[i * n + i] = 1.0L;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0L) throw std::runtime_error("singular matrix");
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(B[c * n + k], B[piv * n + k]);
    }
    const xreal d = 1.0L / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= d;
      B[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const xreal f = A[r * n + c];
      if (f == 0.0L) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        B[r * n + k] -= f * B[c * n + k];
      }
    }
  }
  return B;
}

// Legendre P_0..P_p and derivatives at x (three-term recurrence)
static void legendre_x(int p, xreal x, xreal* P, xreal* dP) {
  P[0] = 1.0L;
  dP[0] = 0.0L;
  if (p >= 1) {
    P[1] = x;
    dP[1] = 1.0L;
  }
  for (int k = 1; k < p; ++k) {
    P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
  }
}

// basis of P_p on the tetrahedron: Legendre products P_a(xi) P_b(eta) P_c(zeta),
// a + b + c <= p, with gradients
static void tet_basis(int p, const xreal* y, xreal* v, xreal* g0, xreal* g1, xreal* g2) {
  xreal P[3][8], dP[3][8];
  for (int d = 0; d < 3; ++d) legendre_x(p, y[d], P[d], dP[d]);
  int k = 0;
  for (int c = 0; c <= p; ++c)
    for (int b = 0; b + c <= p; ++b)
      for (int a = 0; a + b + c <= p; ++a) {
        v[k] = P[0][a] * P[1][b] * P[2][c];
        g0[k] = dP[0][a] * P[1][b] * P[2][c];
        g1[k] = P[0][a] * dP[1][b] * P[2][c];
        g2[k] = P[0][a] * P[1][b] * dP[2][c];
        ++k;
      }
}

// pyramid solution points (a reading; the paper prints none): p+1 layers at
// the Gauss-Legendre(p+1) heights zeta_l in increasing order, layer l holding
// the tensor Gauss-Legendre(p+1-l) grid of the collapsed coordinates
// (a, b) = (2 xi, 2 eta)/(1 - zeta); every layer is unisolvent for Q_{p-l} in
// (a, b), which makes the set unisolvent for the pyramid space
static void pyr_nodes(int p, std::vector<double>& x) {
  x.clear();
  std::vector<double> t, tw;
  gauss_legendre(p + 1, t, tw);
  for (int l = 0; l <= p; ++l) {
    std::vector<double> g, gw;
    gauss_legendre(p + 1 - l, g, gw);
    const double s = 0.5 * (1.0 - t[l]);
    for (int j = 0; j <= p - l; ++j)
      for (int i = 0; i <= p - l; ++i) {
        x.push_back(g[i] * s);
        x.push_back(g[j] * s);
        x.push_back(t[l]);
      }
  }
}

// basis of the pyramid space (rational; Bergot, Cohen and Durufle 2010): in
// the collapsed coordinates a = 2 xi/(1-zeta), b = 2 eta/(1-zeta), c = zeta,
// P_i(a) P_j(b) (1-c)^max(i,j) P_k(c) for i, j <= p, k <= p - max(i,j).  It
// contains P_p, its trace is Q_p on the base and P_p on each triangle.  Its
// gradient by the chain rule: d a/d xi = 2/(1-c), d a/d zeta = a/(1-c), and
// likewise for b.  Never evaluated at the apex.
static void pyr_basis(int p, const xreal* y, xreal* v, xreal* g0, xreal* g1, xreal* g2) {
  const xreal om = 1.0L - y[2], a = 2.0L * y[0] / om, b = 2.0L * y[1] / om;
  xreal Pa[8], dPa[8], Pb[8], dPb[8], Pc[8], dPc[8];
  legendre_x(p, a, Pa, dPa);
  legendre_x(p, b, Pb, dPb);
  legendre_x(p, y[2], Pc, dPc);
  int k = 0;
  for (int j = 0; j <= p; ++j)
    for (int i = 0; i <= p; ++i) {
      const int mu = std::max(i, j);
      xreal omu = 1.0L;
      for (int e = 0; e < mu; ++e) omu *= om;
      for (int l = 0; l + mu <= p; ++l) {
        const xreal C = omu * Pc[l];
        const xreal dC = omu * dPc[l] - (mu > 0 ? mu * (omu / om) * Pc[l] : 0.0L);
        v[k] = Pa[i] * Pb[j] * C;
        g0[k] = dPa[i] * Pb[j] * C * 2.0L / om;
        g1[k] = Pa[i] * dPb[j] * C * 2.0L / om;
        g2[k] = (dPa[i] * a * Pb[j] + Pa[i] * dPb[j] * b) * C / om + Pa[i] * Pb[j] * dC;
        ++k;
      }
    }
}

// Lagrange polynomial j through the nodes x, at y (extended precision)
static xreal lagrange_x(const std::vector<double>& x, int j, xreal y) {
  xreal v = 1.0L;
  for (size_t k = 0; k < x.size(); ++k)
    if ((int)k != j) v *= (y - (xreal)x[k]) / ((xreal)x[j] - (xreal)x[k]);
  return v;
}

// Tetrahedra (etype 2) and pyramids (etype 3): no tensor structure, so the
// operators are dense, from the Vandermonde inverse of the element's basis.
// Pyramid faces: the base (GL(n)^2 flux points, index a + n b over
// (xi, eta)) and four triangles; tetrahedron faces: four triangles; each
// triangle carries the triangle nodes mapped from the reference triangle's
// (-1,-1), (1,-1), (-1,1) to the face's listed vertices.  AP_d is the weak
// form -Mass^-1 Dq_d^T W_q; for tetrahedra it equals (M1 - M3 M2) M9, for
// pyramids (whose space is not closed under differentiation) it is the
// divergence by definition, and Ku_d = AP_d M7 is its form without
// anti-aliasing.
static void build_dense(int etype, int p, RefElem& r) {
  build_tri(p, r.line, r.tri);
  const Tri& T = r.tri;
  const Line1D& L = r.line;
  const bool pyr = etype == 3;
  const int n = p + 1, nt = T.nt;
  const int nu = pyr ? n * (n + 1) * (2 * n + 1) / 6 : n * (n + 1) * (n + 2) / 6;
  const int ntri = 4;
  r.nu = nu;
  r.nfaces = pyr ? 5 : 4;
  r.nfp_max = pyr ? n * n : nt;
  if (pyr)
    pyr_nodes(p, r.upts);
  else
    tet_nodes(p, r.upts);
  const double cen[3] = {pyr ? 0.0 : -0.5, pyr ? 0.0 : -0.5, -0.5};  // reference centroid
  if (pyr) {
    r.face_start.push_back(0);
    r.face_npts.push_back(n * n);
    r.face_normal.insert(r.face_normal.end(), {0.0, 0.0, -1.0});
    r.face_jac.push_back(1.0);
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a) r.fpts.insert(r.fpts.end(), {L.x[a], L.x[b], -1.0});
  }
  for (int f = 0; f < ntri; ++f) {
    const double* A = pyr ? kPyrV[kPyrFace[f][0]] : kTetV[kTetFace[f][0]];
    const double* B = pyr ? kPyrV[kPyrFace[f][1]] : kTetV[kTetFace[f][1]];
    const double* C = pyr ? kPyrV[kPyrFace[f][2]] : kTetV[kTetFace[f][2]];
    r.face_start.push_back((int)r.fpts.size() / 3);
    r.face_npts.push_back(nt);
    // outward unit normal: (B - A) x (C - A), oriented away from the centroid
    double e1[3], e2[3], nr[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = B[d] - A[d];
      e2[d] = C[d] - A[d];
    }
    nr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    nr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    nr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double len = std::sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
    double side = 0;
    for (int d = 0; d < 3; ++d) side += nr[d] * (cen[d] - A[d]);
    const double sgn = side > 0 ? -1.0 : 1.0;
    for (int d = 0; d < 3; ++d) r.face_normal.push_back(sgn * nr[d] / len);
    r.face_jac.push_back(0.25 * len);  // face area / reference triangle area (2)
    for (int t = 0; t < nt; ++t) {
      const double s = T.nodes[2 * t], u = T.nodes[2 * t + 1];
      const double la = -(s + u) / 2.0, lb = (1.0 + s) / 2.0, lc = (1.0 + u) / 2.0;
      for (int d = 0; d < 3; ++d) r.fpts.push_back(la * A[d] + lb * B[d] + lc * C[d]);
    }
  }
  // conical-product rules with (p+1)^3 points (degree 2p+1)
  {
    const int k = p + 1;
    std::vector<double> a, wa, b, wb, c, wc;
    gauss_legendre(k, a, wa);
    gauss_jacobi(k, 1.0, 0.0, b, wb);
    gauss_jacobi(k, 2.0, 0.0, c, wc);
    for (int l = 0; l < k; ++l)
      for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i) {
          if (pyr) {
            // xi = a (1-c)/2, eta = b (1-c)/2, zeta = c; dV = (1-c)^2/4
            const double s = 0.5 * (1 - c[l]);
            r.qpts.insert(r.qpts.end(), {a[i] * s, a[j] * s, c[l]});
            r.qwts.push_back(wa[i] * wa[j] * wc[l] / 4.0);
          } else {
            r.qpts.push_back(0.25 * (1 + a[i]) * (1 - b[j]) * (1 - c[l]) - 1.0);
            r.qpts.push_back(0.5 * (1 + b[j]) * (1 - c[l]) - 1.0);
            r.qpts.push_back(c[l]);
            r.qwts.push_back(wa[i] * wb[j] * wc[l] / 8.0);
          }
        }
  }
  r.nf = (int)r.fpts.size() / 3;
  r.nq = (int)r.qwts.size();
  const int nf = r.nf, nq = r.nq;
  auto basis = [&](const xreal* y, xreal* v, xreal* g0, xreal* g1, xreal* g2) {
    if (pyr)
      pyr_basis(p, y, v, g0, g1, g2);
    else
      tet_basis(p, y, v, g0, g1, g2);
  };
  // nodal basis l_u(y) = sum_k psi_k(y) Vi[k][u]
  std::vector<xreal> V(nu * nu), v(nu), g0(nu), g1(nu), g2(nu);
  for (int u = 0; u < nu; ++u) {
    const xreal y[3] = {r.upts[3 * u], r.upts[3 * u + 1], r.upts[3 * u + 2]};
    basis(y, v.data(), g0.data(), g1.data(), g2.data());
    for (int k = 0; k < nu; ++k) V[u * nu + k] = v[k];
  }
  const std::vector<xreal> Vi = inverse_x(V, nu);
  auto nodal = [&](const double* yd, xreal* l, xreal* d0, xreal* d1, xreal* d2) {
    const xreal y[3] = {yd[0], yd[1], yd[2]};
    basis(y, v.data(), g0.data(), g1.data(), g2.data());
    for (int u = 0; u < nu; ++u) {
      xreal s = 0, s0 = 0, s1 = 0, s2 = 0;
      for (int k = 0; k < nu; ++k) {
        const xreal w = Vi[k * nu + u];
        s += v[k] * w;
        s0 += g0[k] * w;
        s1 += g1[k] * w;
        s2 += g2[k] * w;
      }
      if (l) l[u] = s;
      if (d0) {
        d0[u] = s0;
        d1[u] = s1;
        d2[u] = s2;
      }
    }
  };
  auto rounded = [](const std::vector<xreal>& a) { return std::vector<double>(a.begin(), a.end()); };
  std::vector<xreal> M0(nf * nu), Dg(3 * nu * nu), M7(nq * nu), Dq(3 * nq * nu);
  for (int f = 0; f < nf; ++f) nodal(&r.fpts[3 * f], &M0[f * nu], nullptr, nullptr, nullptr);
  for (int s = 0; s < nu; ++s)
    nodal(&r.upts[3 * s], nullptr, &Dg[(0 * nu + s) * nu], &Dg[(1 * nu + s) * nu], &Dg[(2 * nu + s) * nu]);
  for (int q = 0; q < nq; ++q)
    nodal(&r.qpts[3 * q], &M7[q * nu], &Dq[(0 * nq + q) * nu], &Dq[(1 * nq + q) * nu], &Dq[(2 * nq + q) * nu]);
  r.M0 = rounded(M0);
  r.Dg = rounded(Dg);
  r.M7 = rounded(M7);
  std::vector<xreal> mass(nu * nu);
  for (int a = 0; a < nu; ++a)
    for (int b = 0; b < nu; ++b) {
      xreal s = 0;
      for (int q = 0; q < nq; ++q) s += M7[q * nu + a] * (xreal)r.qwts[q] * M7[q * nu + b];
      mass[a * nu + b] = s;
    }
  r.mass = rounded(mass);
  const std::vector<xreal> Mi = inverse_x(mass, nu);
  r.M8.assign(nu * nq, 0);
  std::vector<xreal> AP(3 * nu * nq);
  std::vector<xreal> wu(nu, 0.0L);
  for (int u = 0; u < nu; ++u) {
    for (int q = 0; q < nq; ++q) {
      xreal s = 0, s0 = 0, s1 = 0, s2 = 0;
      for (int k = 0; k < nu; ++k) {
        const xreal w = Mi[u * nu + k];
        s += w * M7[q * nu + k];
        s0 += w * Dq[(0 * nq + q) * nu + k];
        s1 += w * Dq[(1 * nq + q) * nu + k];
        s2 += w * Dq[(2 * nq + q) * nu + k];
      }
      const xreal wq = r.qwts[q];
      r.M8[u * nq + q] = (double)(s * wq);
      AP[(0 * nu + u) * nq + q] = -s0 * wq;
      AP[(1 * nu + u) * nq + q] = -s1 * wq;
      AP[(2 * nu + u) * nq + q] = -s2 * wq;
      wu[u] += M7[q * nu + u] * wq;
    }
  }
  r.APd = rounded(AP);
  r.wu = rounded(wu);
  if (pyr) {
    r.Ku.assign(3 * nu * nu, 0);
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < nu; ++s)
        for (int u = 0; u < nu; ++u) {
          xreal acc = 0;
          for (int q = 0; q < nq; ++q) acc += AP[(d * nu + s) * nq + q] * M7[q * nu + u];
          r.Ku[(d * nu + s) * nu + u] = (double)acc;
        }
  }
  // DG lifting: E[u, f] = int_face l_u l^face_f dS_ref, with the triangle
  // rule mapped onto each triangle and GL(n+1)^2 on the base; M3 = Mass^-1 E
  std::vector<xreal> Ef(nu * nf, 0.0L), lf(nu);
  const int f0 = pyr ? 1 : 0;
  for (int f = 0; f < ntri; ++f) {
    const double* A = pyr ? kPyrV[kPyrFace[f][0]] : kTetV[kTetFace[f][0]];
    const double* B = pyr ? kPyrV[kPyrFace[f][1]] : kTetV[kTetFace[f][1]];
    const double* C = pyr ? kPyrV[kPyrFace[f][2]] : kTetV[kTetFace[f][2]];
    for (int q = 0; q < T.ntq; ++q) {
      const double s = T.qp[2 * q], u = T.qp[2 * q + 1];
      const double la = -(s + u) / 2.0, lb = (1.0 + s) / 2.0, lc = (1.0 + u) / 2.0;
      double y[3];
      for (int d = 0; d < 3; ++d) y[d] = la * A[d] + lb * B[d] + lc * C[d];
      nodal(y, lf.data(), nullptr, nullptr, nullptr);
      const xreal w = (xreal)T.qw[q] * (xreal)r.face_jac[f0 + f];
      for (int t = 0; t < nt; ++t) {
        const xreal wt = w * (xreal)T.Tq[q * nt + t];
        for (int uu = 0; uu < nu; ++uu) Ef[uu * nf + r.face_start[f0 + f] + t] += lf[uu] * wt;
      }
    }
  }
  if (pyr) {
    std::vector<double> g, gw;
    gauss_legendre(n + 1, g, gw);
    for (int qb = 0; qb <= n; ++qb)
      for (int qa = 0; qa <= n; ++qa) {
        const double y[3] = {g[qa], g[qb], -1.0};
        nodal(y, lf.data(), nullptr, nullptr, nullptr);
        const xreal w = (xreal)gw[qa] * (xreal)gw[qb];
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            const xreal wt = w * lagrange_x(L.x, a, g[qa]) * lagrange_x(L.x, b, g[qb]);
            for (int uu = 0; uu < nu; ++uu) Ef[uu * nf + a + n * b] += lf[uu] * wt;
          }
      }
  }
  r.M3.assign(nu * nf, 0);
  for (int u = 0; u < nu; ++u)
    for (int f = 0; f < nf; ++f) {
      xreal s = 0;
      for (int k = 0; k < nu; ++k) s += Mi[u * nu + k] * Ef[k * nf + f];
      r.M3[u * nf + f] = (double)s;
    }
}

void build_ref(int etype, int p, RefElem& r) {
  int n = p + 1, m = p + 3;
  r.etype = etype;
  r.p = p;
  r.n = n;
  r.m = m;
  build_line(p, m, r.line);
  const Line1D& L = r.line;
  auto push3 = [](std::vector<double>& v, double a, double b, double c) {
    v.push_back(a);
    v.push_back(b);
    v.push_back(c);
  };
  r.upts.clear();
  r.fpts.clear();
  r.qpts.clear();
  r.qwts.clear();
  r.face_start.clear();
  r.face_npts.clear();
  r.face_normal.clear();
  r.face_jac.clear();
  if (etype >= 2) {
    build_dense(etype, p, r);
    return;
  }
  if (etype == 0) {
    r.nu = n * n * n;
    r.nfaces = 6;
    r.nfp_max = n * n;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) push3(r.upts, L.x[i], L.x[j], L.x[k]);
    for (int ax = 0; ax < 3; ++ax)
      for (int sg = 0; sg < 2; ++sg) {
        double s = sg ? 1.0 : -1.0;
        r.face_start.push_back((int)r.fpts.size() / 3);
        r.face_npts.push_back(n * n);
        double nr[3] = {0, 0, 0};
        nr[ax] = s;
        push3(r.face_normal, nr[0], nr[1], nr[2]);
        int t0 = ax == 0 ? 1 : 0, t1 = ax == 2 ? 1 : 2;
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            double c[3];
            c[ax] = s;
            c[t0] = L.x[a];
            c[t1] = L.x[b];
            push3(r.fpts, c[0], c[1], c[2]);
          }
      }
    for (int k = 0; k < m; ++k)
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
          push3(r.qpts, L.xq[i], L.xq[j], L.xq[k]);
          r.qwts.push_back(L.wq[i] * L.wq[j] * L.wq[k]);
        }
  } else {
    build_tri(p, L, r.tri);
    const Tri& T = r.tri;
    int nt = T.nt;
    r.nu = nt * n;
    r.nfaces = 5;
    r.nfp_max = n * n;
    for (int k = 0; k < n; ++k)
      for (int t = 0; t < nt; ++t) push3(r.upts, T.nodes[2 * t], T.nodes[2 * t + 1], L.x[k]);
    for (int sg = 0; sg < 2; ++sg) {
      r.face_start.push_back((int)r.fpts.size() / 3);
      r.face_npts.push_back(nt);
      push3(r.face_normal, 0, 0, sg ? 1.0 : -1.0);
      for (int t = 0; t < nt; ++t) push3(r.fpts, T.nodes[2 * t], T.nodes[2 * t + 1], sg ? 1.0 : -1.0);
    }
    for (int e = 0; e < 3; ++e) {
      r.face_start.push_back((int)r.fpts.size() / 3);
      r.face_npts.push_back(n * n);
      push3(r.face_normal, T.edgeNormal[e][0], T.edgeNormal[e][1], 0.0);
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          double s = L.x[a];
          double xi = e == 0 ? s : (e == 1 ? -s : -1.0);
          double eta = e == 0 ? -1.0 : (e == 1 ? s : -s);
          push3(r.fpts, xi, eta, L.x[b]);
        }
    }
    for (int k = 0; k < m; ++k)
      for (int q = 0; q < T.ntq; ++q) {
        push3(r.qpts, T.qp[2 * q], T.qp[2 * q + 1], L.xq[k]);
        r.qwts.push_back(T.qw[q] * L.wq[k]);
      }
  }
  r.nf = (int)r.fpts.size() / 3;
  r.nq = (int)r.qwts.size();
  int nu = r.nu, nf = r.nf, nq = r.nq;

  // dense operators from the factors
  r.M0.assign(nf * nu, 0);
  r.M3.assign(nu * nf, 0);
  r.M7.assign(nq * nu, 0);
  r.M8.assign(nu * nq, 0);
  r.Dg.assign(3 * nu * nu, 0);
  r.wu.assign(nu, 0);
  if (etype == 0) {
    auto uidx = [n](int i, int j, int k) { return i + n * (j + n * k); };
    for (int ax = 0; ax < 3; ++ax)
      for (int sg = 0; sg < 2; ++sg) {
        int f = 2 * ax + sg;
        const std::vector<double>& bv = sg ? L.rb : L.lb;
        const std::vector<double>& lv = sg ? L.liftR : L.liftL;
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            int fp = r.face_start[f] + a + n * b;
            for (int i = 0; i < n; ++i) {
              int c[3];
              c[ax] = i;
              c[ax == 0 ? 1 : 0] = a;
              c[ax == 2 ? 1 : 2] = b;
              int u = uidx(c[0], c[1], c[2]);
              r.M0[fp * nu + u] = bv[i];
              r.M3[u * nf + fp] = lv[i];
            }
          }
      }
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          int s = uidx(i, j, k);
          r.wu[s] = L.w[i] * L.w[j] * L.w[k];
          for (int a = 0; a < n; ++a) {
            r.Dg[(0 * nu + s) * nu + uidx(a, j, k)] = L.D[i * n + a];
            r.Dg[(1 * nu + s) * nu + uidx(i, a, k)] = L.D[j * n + a];
            r.Dg[(2 * nu + s) * nu + uidx(i, j, a)] = L.D[k * n + a];
          }
        }
    for (int c = 0; c < m; ++c)
      for (int b = 0; b < m; ++b)
        for (int a = 0; a < m; ++a) {
          int q = a + m * (b + m * c);
          for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
              for (int i = 0; i < n; ++i) {
                int u = uidx(i, j, k);
                r.M7[q * nu + u] = L.I[a * n + i] * L.I[b * n + j] * L.I[c * n + k];
                r.M8[u * nq + q] = L.P[i * m + a] * L.P[j * m + b] * L.P[k * m + c];
              }
        }
  } else {
    const Tri& T = r.tri;
    int nt = T.nt, ntq = T.ntq;
    for (int sg = 0; sg < 2; ++sg) {
      const std::vector<double>& bv = sg ? L.rb : L.lb;
      const std::vector<double>& lv = sg ? L.liftR : L.liftL;
      for (int t = 0; t < nt; ++t) {
        int fp = r.face_start[sg] + t;
        for (int k = 0; k < n; ++k) {
          r.M0[fp * nu + t + nt * k] = bv[k];
          r.M3[(t + nt * k) * nf + fp] = lv[k];
        }
      }
    }
    for (int e = 0; e < 3; ++e)
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          int fp = r.face_start[2 + e] + a + n * b;
          for (int t = 0; t < nt; ++t) {
            r.M0[fp * nu + t + nt * b] = T.Tedge[(e * n + a) * nt + t];
            r.M3[(t + nt * b) * nf + fp] = T.LiftEdge[(e * nt + t) * n + a];
          }
        }
    for (int k = 0; k < n; ++k)
      for (int t = 0; t < nt; ++t) {
        int s = t + nt * k;
        for (int t2 = 0; t2 < nt; ++t2) {
          r.Dg[(0 * nu + s) * nu + t2 + nt * k] = T.Dxi[t * nt + t2];
          r.Dg[(1 * nu + s) * nu + t2 + nt * k] = T.Deta[t * nt + t2];
        }
        for (int a = 0; a < n; ++a) r.Dg[(2 * nu + s) * nu + t + nt * a] = L.D[k * n + a];
      }
    for (int c = 0; c < m; ++c)
      for (int q = 0; q < ntq; ++q) {
        int qq = q + ntq * c;
        for (int k = 0; k < n; ++k)
          for (int t = 0; t < nt; ++t) {
            int u = t + nt * k;
            r.M7[qq * nu + u] = T.Tq[q * nt + t] * L.I[c * n + k];
            r.M8[u * nq + qq] = T.PT[t * ntq + q] * L.P[k * m + c];
          }
      }
    for (int k = 0; k < n; ++k)
      for (int t = 0; t < nt; ++t) {
        double s = 0;
        for (int q = 0; q < ntq; ++q) s += T.Tq[q * nt + t] * T.qw[q];
        r.wu[t + nt * k] = s * L.w[k];
      }
  }
}

}  // namespace fr
