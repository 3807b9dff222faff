// Host FP64 setup: nodes, orthonormal-basis operators, geometry, face matching.
//
// The paper's own scheme expands the solution on each element in an
// orthonormal basis (Appendix A, Eq. 11: the mass matrix is then a multiple
// of the identity).  The nodal operators here are built from the same kind
// of basis -- the collapsed-coordinate (Dubiner) orthonormal polynomials on
// the tetrahedron and triangle -- evaluated at warp-and-blend nodes
// (Warburton, J. Eng. Math. 2006):
//   V[i][m] = psi_m(node i),  Dr = Vr V^-1,  M^-1 = V V^T,
//   face mass E_f = (V2 V2^T)^-1 on the face nodes,  LIFT_f = V V^T E_f.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace dg {
namespace {

constexpr int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
constexpr int kPerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// ---- small dense linear algebra -------------------------------------------

// In-place inverse of a row-major n x n matrix, Gauss-Jordan with partial
// pivoting.  Returns false when singular.
bool invert(std::vector<double>& a, int n) {
  std::vector<double> inv(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[size_t(r) * n + c]) > std::fabs(a[size_t(p) * n + c])) p = r;
    if (std::fabs(a[size_t(p) * n + c]) < 1e-300) return false;
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[size_t(p) * n + j], a[size_t(c) * n + j]);
        std::swap(inv[size_t(p) * n + j], inv[size_t(c) * n + j]);
      }
    const double d = 1.0 / a[size_t(c) * n + c];
    for (int j = 0; j < n; ++j) {
      a[size_t(c) * n + j] *= d;
      inv[size_t(c) * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[size_t(r) * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[size_t(r) * n + j] -= f * a[size_t(c) * n + j];
        inv[size_t(r) * n + j] -= f * inv[size_t(c) * n + j];
      }
    }
  }
  a.swap(inv);
  return true;
}

// C[m x n] = A[m x k] * B[k x n], row-major.
std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int m,
                           int k, int n) {
  std::vector<double> C(size_t(m) * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < k; ++l) {
      const double a = A[size_t(i) * k + l];
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[size_t(i) * n + j] += a * B[size_t(l) * n + j];
    }
  return C;
}

std::vector<double> transpose(const std::vector<double>& A, int m, int n) {
  std::vector<double> T(size_t(m) * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) T[size_t(j) * m + i] = A[size_t(i) * n + j];
  return T;
}

// ---- Jacobi polynomials ----------------------------------------------------

// Jacobi polynomial P_n^(al,be)(x) normalized to unit L2 norm on [-1,1] with
// weight (1-x)^al (1+x)^be.  Standard three-term recurrence for the
// classical polynomials, then division by the square root of the norm
//   h_n = 2^(al+be+1)/(2n+al+be+1) G(n+al+1)G(n+be+1)/(G(n+al+be+1) n!).
double jacobi_norm(double x, int n, double al, double be) {
  double p0 = 1.0, p1 = 0.0;
  if (n > 0) p1 = 0.5 * (al - be + (al + be + 2.0) * x);
  double pn = (n == 0) ? p0 : p1;
  for (int k = 2; k <= n; ++k) {
    const double s = 2.0 * k + al + be;
    const double a1 = 2.0 * k * (k + al + be) * (s - 2.0);
    const double a2 = (s - 1.0) * (al * al - be * be);
    const double a3 = (s - 2.0) * (s - 1.0) * s;
    const double a4 = 2.0 * (k + al - 1.0) * (k + be - 1.0) * s;
    pn = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = pn;
  }
  const double lh = (al + be + 1.0) * std::log(2.0) - std::log(2.0 * n + al + be + 1.0) +
                    std::lgamma(n + al + 1.0) + std::lgamma(n + be + 1.0) -
                    std::lgamma(n + al + be + 1.0) - std::lgamma(n + 1.0);
  return pn / std::exp(0.5 * lh);
}

// d/dx of the normalized P_n^(al,be): sqrt(n(n+al+be+1)) P_{n-1}^(al+1,be+1).
double jacobi_norm_deriv(double x, int n, double al, double be) {
  if (n == 0) return 0.0;
  return std::sqrt(double(n) * (n + al + be + 1.0)) * jacobi_norm(x, n - 1, al + 1.0, be + 1.0);
}

// Gauss-Lobatto-Legendre points on [-1,1], ascending: the endpoints and the
// zeros of P_N' (equivalently of P_{N-1}^(1,1)), by Newton's method from the
// Chebyshev-Gauss-Lobatto points.
std::vector<double> lgl(int N) {
  std::vector<double> x(N + 1);
  x[0] = -1.0;
  x[N] = 1.0;
  for (int j = 1; j < N; ++j) {
    double z = -std::cos(M_PI * j / N);
    for (int it = 0; it < 100; ++it) {
      const double f = jacobi_norm(z, N - 1, 1.0, 1.0);
      const double df = jacobi_norm_deriv(z, N - 1, 1.0, 1.0);
      const double dz = f / df;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[j] = z;
  }
  std::sort(x.begin(), x.end());
  return x;
}

// ---- warp-and-blend nodes --------------------------------------------------

// Scaled 1D warp: the Lagrange interpolant (on N+1 equispaced points) of the
// displacement from equispaced to LGL points, divided by (1 - x^2).  Both
// end displacements vanish, so the division is done term by term on the
// interior Lagrange polynomials, each of which carries (x+1)(x-1).
double edge_warp(int N, const std::vector<double>& xgl, double x) {
  double w = 0.0;
  for (int i = 1; i < N; ++i) {
    const double xi = -1.0 + 2.0 * i / N;
    double term = (xgl[i] - xi) / (1.0 - xi * xi);
    for (int j = 1; j < N; ++j) {
      if (j == i) continue;
      const double xj = -1.0 + 2.0 * j / N;
      term *= (x - xj) / (xi - xj);
    }
    w += term;
  }
  return w;
}

double blend_alpha(int N) {
  static const double a[15] = {0.0,    0.0,    0.0,    0.1002, 1.1332, 1.5608, 1.3413, 1.2577,
                               1.1603, 1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655};
  return N <= 15 ? a[N - 1] : 1.0;
}

// Reference coordinates of the order-N nodes, [Np][3].
std::vector<double> warp_blend(int N) {
  const double alpha = blend_alpha(N);
  const std::vector<double> xgl = lgl(N);
  const double s3 = std::sqrt(3.0), s6 = std::sqrt(6.0);
  // equilateral tetrahedron, vertex v <-> barycentric lambda_v
  const double E[4][3] = {{-1.0, -1.0 / s3, -1.0 / s6},
                          {1.0, -1.0 / s3, -1.0 / s6},
                          {0.0, 2.0 / s3, -1.0 / s6},
                          {0.0, 0.0, 3.0 / s6}};
  std::vector<std::array<double, 4>> lam;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k) {
        const int l = N - i - j - k;
        lam.push_back({double(l) / N, double(i) / N, double(j) / N, double(k) / N});
      }
  const int Np = int(lam.size());
  std::vector<double> out(size_t(Np) * 3);
  const double tol = 1e-10;
  const double c120 = std::cos(2.0 * M_PI / 3.0), s120 = std::sin(2.0 * M_PI / 3.0);
  const double c240 = std::cos(4.0 * M_PI / 3.0), s240 = std::sin(4.0 * M_PI / 3.0);
  for (int n = 0; n < Np; ++n) {
    const auto& L = lam[n];
    double X[3] = {0, 0, 0};
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) X[d] += L[v] * E[v][d];
    double shift[3] = {0, 0, 0};
    for (int f = 0; f < 4; ++f) {
      // face with base edge P->Q and apex R; vertex A is opposite
      const int P = kFaceVerts[f][0], Q = kFaceVerts[f][1], R = kFaceVerts[f][2];
      const int A = 6 - P - Q - R;
      const double la = L[A], l1 = L[R], l2 = L[P], l3 = L[Q];
      double t1[3], t2[3], n1 = 0, n2 = 0;
      for (int d = 0; d < 3; ++d) {
        t1[d] = E[Q][d] - E[P][d];
        t2[d] = E[R][d] - 0.5 * (E[P][d] + E[Q][d]);
        n1 += t1[d] * t1[d];
        n2 += t2[d] * t2[d];
      }
      n1 = std::sqrt(n1);
      n2 = std::sqrt(n2);
      // 2D warp of the face's equilateral triangle: one term per edge,
      // each along that edge's direction (0, 120, 240 degrees)
      const double w1 = 4.0 * l2 * l3 * edge_warp(N, xgl, l3 - l2) * (1.0 + (alpha * l1) * (alpha * l1));
      const double w2 = 4.0 * l1 * l3 * edge_warp(N, xgl, l1 - l3) * (1.0 + (alpha * l2) * (alpha * l2));
      const double w3 = 4.0 * l1 * l2 * edge_warp(N, xgl, l2 - l1) * (1.0 + (alpha * l3) * (alpha * l3));
      const double dx = w1 + c120 * w2 + c240 * w3;
      const double dy = s120 * w2 + s240 * w3;
      double blend = l1 * l2 * l3;
      const double denom = (l1 + 0.5 * la) * (l2 + 0.5 * la) * (l3 + 0.5 * la);
      if (denom > tol) blend = (1.0 + (alpha * la) * (alpha * la)) * blend / denom;
      const int positive = (l1 > tol) + (l2 > tol) + (l3 > tol);
      if (la < tol && positive < 3) {
        // on an edge of this face: the pure edge warp replaces everything
        for (int d = 0; d < 3; ++d) shift[d] = dx * t1[d] / n1 + dy * t2[d] / n2;
      } else {
        for (int d = 0; d < 3; ++d) shift[d] += blend * (dx * t1[d] / n1 + dy * t2[d] / n2);
      }
    }
    // back to (r,s,t):  X = (E1+E2+E3-E0)/2 + [E1-E0 | E2-E0 | E3-E0]/2 * (r,s,t)
    std::vector<double> M(9);
    double b[3];
    for (int d = 0; d < 3; ++d) {
      M[d * 3 + 0] = 0.5 * (E[1][d] - E[0][d]);
      M[d * 3 + 1] = 0.5 * (E[2][d] - E[0][d]);
      M[d * 3 + 2] = 0.5 * (E[3][d] - E[0][d]);
      b[d] = X[d] + shift[d] - 0.5 * (E[1][d] + E[2][d] + E[3][d] - E[0][d]);
    }
    invert(M, 3);
    for (int d = 0; d < 3; ++d)
      out[size_t(n) * 3 + d] = M[d * 3 + 0] * b[0] + M[d * 3 + 1] * b[1] + M[d * 3 + 2] * b[2];
  }
  return out;
}

// ---- orthonormal bases -----------------------------------------------------

// Collapsed coordinates of the tetrahedron: a = 2(1+r)/(-s-t) - 1,
// b = 2(1+s)/(1-t) - 1, c = t (a = -1 on the edge s+t = 0, b = -1 at t = 1).
void collapse3(double r, double s, double t, double& a, double& b, double& c) {
  a = (std::fabs(s + t) > 1e-14) ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
  b = (std::fabs(t - 1.0) > 1e-14) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
  c = t;
}

double ipow(double x, int n) {
  double y = 1.0;
  for (int i = 0; i < n; ++i) y *= x;
  return y;
}

// psi_ijk = 2^(2i+j+3/2) f(a) A^i g(b) B^(i+j) h(c), A = (1-b)/2, B = (1-c)/2,
// f = P_i^(0,0), g = P_j^(2i+1,0), h = P_k^(2i+2j+2,0) (normalized), which
// is orthonormal on the reference tetrahedron (dr ds dt = A B^2 da db dc).
// Gradient by the chain rule with
//   da/dr = 1/(AB), da/ds = da/dt = (1+a)/(2AB), db/ds = 1/B,
//   db/dt = (1+b)/(2B), dc/dt = 1,
// the negative powers of A and B cancelled analytically.
void basis3(int i, int j, int k, double r, double s, double t, double& v, double& vr,
            double& vs, double& vt) {
  double a, b, c;
  collapse3(r, s, t, a, b, c);
  const double A = 0.5 * (1.0 - b), B = 0.5 * (1.0 - c);
  const double f = jacobi_norm(a, i, 0, 0), df = jacobi_norm_deriv(a, i, 0, 0);
  const double g = jacobi_norm(b, j, 2 * i + 1, 0), dg = jacobi_norm_deriv(b, j, 2 * i + 1, 0);
  const double h = jacobi_norm(c, k, 2 * i + 2 * j + 2, 0);
  const double dh = jacobi_norm_deriv(c, k, 2 * i + 2 * j + 2, 0);
  const double scale = std::pow(2.0, 2 * i + j + 1.5);
  v = scale * f * ipow(A, i) * g * ipow(B, i + j) * h;
  // d/dr: f' A^(i-1) g B^(i+j-1) h   (zero when i = 0 since f' = 0)
  double dr = 0.0;
  if (i > 0) dr = df * ipow(A, i - 1) * g * ipow(B, i + j - 1) * h;
  // d/db (A^i g) = A^i g' - (i/2) A^(i-1) g
  double gb = ipow(A, i) * dg;
  if (i > 0) gb -= 0.5 * i * ipow(A, i - 1) * g;
  // f * d/db(A^i g) * db/ds * B^(i+j) h = f gb B^(i+j-1) h; zero when i+j = 0
  double sb = 0.0;
  if (i + j > 0) sb = f * gb * ipow(B, i + j - 1) * h;
  const double ds = 0.5 * (1.0 + a) * dr + sb;
  // d/dc (B^(i+j) h) = B^(i+j) h' - ((i+j)/2) B^(i+j-1) h
  double hc = ipow(B, i + j) * dh;
  if (i + j > 0) hc -= 0.5 * (i + j) * ipow(B, i + j - 1) * h;
  const double dt = 0.5 * (1.0 + a) * dr + 0.5 * (1.0 + b) * sb + f * ipow(A, i) * g * hc;
  vr = scale * dr;
  vs = scale * ds;
  vt = scale * dt;
}

// psi_ij = 2^(i+1/2) P_i(a) A^i P_j^(2i+1,0)(b) on the triangle
// {u,v >= -1, u+v <= 0}, a = 2(1+u)/(1-v) - 1, b = v, A = (1-b)/2.
double basis2(int i, int j, double u, double v) {
  const double a = (std::fabs(v - 1.0) > 1e-14) ? 2.0 * (1.0 + u) / (1.0 - v) - 1.0 : -1.0;
  const double A = 0.5 * (1.0 - v);
  return std::pow(2.0, i + 0.5) * jacobi_norm(a, i, 0, 0) * ipow(A, i) *
         jacobi_norm(v, j, 2 * i + 1, 0);
}

}  // namespace

std::string build_reference(int N, RefOps& ops) {
  if (N < 1 || N > 8) return "N must be in 1..8";
  ops.N = N;
  ops.Np = (N + 1) * (N + 2) * (N + 3) / 6;
  ops.Nfp = (N + 1) * (N + 2) / 2;
  const int Np = ops.Np, Nfp = ops.Nfp;
  ops.rst = warp_blend(N);

  std::vector<double> V(size_t(Np) * Np), Vr(V.size()), Vs(V.size()), Vt(V.size());
  for (int n = 0; n < Np; ++n) {
    int m = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j)
        for (int k = 0; k <= N - i - j; ++k, ++m) {
          double v, vr, vs, vt;
          basis3(i, j, k, ops.rst[n * 3], ops.rst[n * 3 + 1], ops.rst[n * 3 + 2], v, vr, vs, vt);
          V[size_t(n) * Np + m] = v;
          Vr[size_t(n) * Np + m] = vr;
          Vs[size_t(n) * Np + m] = vs;
          Vt[size_t(n) * Np + m] = vt;
        }
  }
  std::vector<double> Vinv = V;
  if (!invert(Vinv, Np)) return "singular Vandermonde matrix";
  ops.Vinv = Vinv;
  ops.Dr = matmul(Vr, Vinv, Np, Np, Np);
  ops.Ds = matmul(Vs, Vinv, Np, Np, Np);
  ops.Dt = matmul(Vt, Vinv, Np, Np, Np);
  const std::vector<double> Minv = matmul(V, transpose(V, Np, Np), Np, Np, Np);

  // face node lists, ascending node index
  ops.Fmask.assign(size_t(4) * Nfp, -1);
  for (int f = 0; f < 4; ++f) {
    int cnt = 0;
    for (int n = 0; n < Np; ++n) {
      const double r = ops.rst[n * 3], s = ops.rst[n * 3 + 1], t = ops.rst[n * 3 + 2];
      const double d = (f == 0) ? 1 + t : (f == 1) ? 1 + s : (f == 2) ? 1 + r + s + t : 1 + r;
      if (std::fabs(d) < 1e-10) {
        if (cnt >= Nfp) return "too many face nodes";
        ops.Fmask[size_t(f) * Nfp + cnt++] = n;
      }
    }
    if (cnt != Nfp) return "wrong number of face nodes";
  }

  // face mass in the face's own two reference coordinates (area 2)
  static const int kParam[4][2] = {{0, 1}, {0, 2}, {1, 2}, {1, 2}};
  ops.LIFT.assign(size_t(Np) * 4 * Nfp, 0.0);
  for (int f = 0; f < 4; ++f) {
    std::vector<double> V2(size_t(Nfp) * Nfp);
    for (int q = 0; q < Nfp; ++q) {
      const int n = ops.Fmask[size_t(f) * Nfp + q];
      const double u = ops.rst[n * 3 + kParam[f][0]], v = ops.rst[n * 3 + kParam[f][1]];
      int m = 0;
      for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j, ++m) V2[size_t(q) * Nfp + m] = basis2(i, j, u, v);
    }
    std::vector<double> M2 = matmul(V2, transpose(V2, Nfp, Nfp), Nfp, Nfp, Nfp);
    if (!invert(M2, Nfp)) return "singular face Vandermonde matrix";
    // LIFT_f[:, q] = Minv[:, Fmask_f] * M2[:, q]
    for (int row = 0; row < Np; ++row)
      for (int q = 0; q < Nfp; ++q) {
        double acc = 0.0;
        for (int p = 0; p < Nfp; ++p)
          acc += Minv[size_t(row) * Np + ops.Fmask[size_t(f) * Nfp + p]] * M2[size_t(p) * Nfp + q];
        ops.LIFT[size_t(row) * 4 * Nfp + f * Nfp + q] = acc;
      }
  }

  // neighbour node tables: node i of face f has barycentric coordinates
  // (b0,b1,b2) on the face's local vertices; with orientation o the shared
  // vertex j of my face is vertex kPerms[o][j] of the neighbour's face f2.
  ops.nbr_node.assign(size_t(4) * 4 * 6 * Nfp, 0);
  auto bary = [&](int n, int v) {
    const double r = ops.rst[n * 3], s = ops.rst[n * 3 + 1], t = ops.rst[n * 3 + 2];
    switch (v) {
      case 0: return -0.5 * (1 + r + s + t);
      case 1: return 0.5 * (1 + r);
      case 2: return 0.5 * (1 + s);
      default: return 0.5 * (1 + t);
    }
  };
  for (int f = 0; f < 4; ++f)
    for (int f2 = 0; f2 < 4; ++f2)
      for (int o = 0; o < 6; ++o)
        for (int i = 0; i < Nfp; ++i) {
          const int n = ops.Fmask[size_t(f) * Nfp + i];
          int found = -1;
          for (int q = 0; q < Nfp && found < 0; ++q) {
            const int n2 = ops.Fmask[size_t(f2) * Nfp + q];
            bool same = true;
            for (int j = 0; j < 3; ++j) {
              const double mine = bary(n, kFaceVerts[f][j]);
              const double theirs = bary(n2, kFaceVerts[f2][kPerms[o][j]]);
              if (std::fabs(mine - theirs) > 1e-9) same = false;
            }
            if (same) found = n2;
          }
          if (found < 0) return "face node tables incomplete";
          ops.nbr_node[((size_t(f) * 4 + f2) * 6 + o) * Nfp + i] = uint8_t(found);
        }
  return "";
}

std::string build_mesh(const RefOps& ops, int64_t K, const double* xyz, const int64_t* EToV,
                       const int8_t* bc, HostMesh& m) {
  (void)ops;
  m.K = K;
  m.xyz.assign(xyz, xyz + K * 12);
  m.EToV.assign(EToV, EToV + K * 4);
  m.bc.assign(bc, bc + K * 4);
  m.drst_dx.assign(size_t(K) * 9, 0.0);
  m.J.assign(size_t(K), 0.0);
  m.nrm.assign(size_t(K) * 12, 0.0);
  m.Fscale.assign(size_t(K) * 4, 0.0);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f)
      if (m.bc[k * 4 + f] < 0 || m.bc[k * 4 + f] > 5) return "unknown boundary tag";

  for (int64_t k = 0; k < K; ++k) {
    double* X = &m.xyz[size_t(k) * 12];
    // Jacobian matrix of x(r,s,t): columns (v1-v0)/2, (v2-v0)/2, (v3-v0)/2
    auto jac = [&](double Jm[3][3]) {
      for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) Jm[d][c] = 0.5 * (X[(c + 1) * 3 + d] - X[d]);
    };
    double Jm[3][3];
    jac(Jm);
    double det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                 Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                 Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
    double scale = 0.0;
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) scale = std::max(scale, std::fabs(Jm[d][c]));
    if (std::fabs(det) <= 1e-12 * scale * scale * scale) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "degenerate element %lld", (long long)k);
      return buf;
    }
    if (det < 0) {  // swap local vertices 1 and 2: faces 1 and 3 trade places
      for (int d = 0; d < 3; ++d) std::swap(X[3 + d], X[6 + d]);
      std::swap(m.EToV[k * 4 + 1], m.EToV[k * 4 + 2]);
      std::swap(m.bc[k * 4 + 1], m.bc[k * 4 + 3]);
      jac(Jm);
      det = -det;
    }
    m.J[k] = det;
    // inverse by cofactors: drst_dx[a][d] = d(r_a)/d(x_d)
    double* G = &m.drst_dx[size_t(k) * 9];
    G[0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) / det;
    G[1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
    G[2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
    G[3] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) / det;
    G[4] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
    G[5] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
    G[6] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) / det;
    G[7] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
    G[8] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
    // outward normals from the reference-coordinate gradients:
    // f0 (t=-1): -grad t, f1 (s=-1): -grad s, f2 (r+s+t=-1): grad(r+s+t),
    // f3 (r=-1): -grad r.  |n| is sJ/J = Fscale.
    for (int f = 0; f < 4; ++f) {
      double n[3];
      for (int d = 0; d < 3; ++d) {
        const double gr = G[d], gs = G[3 + d], gt = G[6 + d];
        n[d] = (f == 0) ? -gt : (f == 1) ? -gs : (f == 2) ? gr + gs + gt : -gr;
      }
      const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int d = 0; d < 3; ++d) m.nrm[size_t(k) * 12 + f * 3 + d] = n[d] / len;
      m.Fscale[size_t(k) * 4 + f] = len;
    }
  }

  // face matching by sorted vertex-id triples
  struct FaceRec {
    std::array<int64_t, 3> key;
    int64_t k;
    int f;
  };
  std::vector<FaceRec> recs(size_t(K) * 4);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      std::array<int64_t, 3> key;
      for (int j = 0; j < 3; ++j) key[j] = m.EToV[k * 4 + kFaceVerts[f][j]];
      std::sort(key.begin(), key.end());
      if (key[0] == key[1] || key[1] == key[2]) return "element with repeated vertex ids";
      recs[size_t(k) * 4 + f] = {key, k, f};
    }
  std::sort(recs.begin(), recs.end(), [](const FaceRec& a, const FaceRec& b) {
    return a.key != b.key ? a.key < b.key : (a.k != b.k ? a.k < b.k : a.f < b.f);
  });
  m.EToE.assign(size_t(K) * 4, -1);
  m.EToF.assign(size_t(K) * 4, 0);
  m.orient.assign(size_t(K) * 4, 0);
  if (K > INT32_MAX) return "too many elements";
  size_t i = 0;
  while (i < recs.size()) {
    size_t j = i + 1;
    while (j < recs.size() && recs[j].key == recs[i].key) ++j;
    const size_t cnt = j - i;
    if (cnt > 2) return "face shared by more than two elements";
    if (cnt == 1) {
      if (m.bc[recs[i].k * 4 + recs[i].f] == 0) return "unmatched face tagged interior";
    } else {
      const FaceRec& a = recs[i];
      const FaceRec& b = recs[i + 1];
      const int ta = m.bc[a.k * 4 + a.f], tb = m.bc[b.k * 4 + b.f];
      if ((ta == 0) != (tb == 0)) return "shared face tagged interior on one side only";
      if (ta == 0) {
        for (int side = 0; side < 2; ++side) {
          const FaceRec& me = side ? b : a;
          const FaceRec& nb = side ? a : b;
          int pos[3];
          for (int q = 0; q < 3; ++q) {
            const int64_t g = m.EToV[me.k * 4 + kFaceVerts[me.f][q]];
            pos[q] = -1;
            for (int r = 0; r < 3; ++r)
              if (m.EToV[nb.k * 4 + kFaceVerts[nb.f][r]] == g) pos[q] = r;
          }
          int code = -1;
          for (int o = 0; o < 6; ++o)
            if (kPerms[o][0] == pos[0] && kPerms[o][1] == pos[1] && kPerms[o][2] == pos[2]) code = o;
          if (code < 0) return "face vertex permutation not found";
          m.EToE[me.k * 4 + me.f] = int32_t(nb.k);
          m.EToF[me.k * 4 + me.f] = uint8_t(nb.f);
          m.orient[me.k * 4 + me.f] = uint8_t(code);
        }
      }
    }
    i = j;
  }
  return "";
}

void node_coordinates(const RefOps& ops, const HostMesh& m, double* out) {
  for (int64_t k = 0; k < m.K; ++k) {
    const double* X = &m.xyz[size_t(k) * 12];
    for (int n = 0; n < ops.Np; ++n) {
      const double r = ops.rst[n * 3], s = ops.rst[n * 3 + 1], t = ops.rst[n * 3 + 2];
      const double l[4] = {-0.5 * (1 + r + s + t), 0.5 * (1 + r), 0.5 * (1 + s), 0.5 * (1 + t)};
      for (int d = 0; d < 3; ++d) {
        double x = 0.0;
        for (int v = 0; v < 4; ++v) x += l[v] * X[v * 3 + d];
        out[(size_t(k) * ops.Np + n) * 3 + d] = x;
      }
    }
  }
}

void neighbour_map(const RefOps& ops, const HostMesh& m, int64_t* out) {
  const int Nfp = ops.Nfp;
  for (int64_t k = 0; k < m.K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int32_t k2 = m.EToE[k * 4 + f];
      for (int i = 0; i < Nfp; ++i) {
        int64_t v = -1;
        if (k2 >= 0) {
          const int f2 = m.EToF[k * 4 + f], o = m.orient[k * 4 + f];
          v = int64_t(k2) * ops.Np + ops.nbr_node[((size_t(f) * 4 + f2) * 6 + o) * Nfp + i];
        }
        out[(size_t(k) * 4 + f) * Nfp + i] = v;
      }
    }
}

std::string curved_geometry(const RefOps& ops, const HostMesh& m, const double* x, double tol,
                            std::vector<int64_t>& elems, std::vector<float>& vg,
                            std::vector<float>& sg) {
  const int Np = ops.Np, Nfp = ops.Nfp;
  elems.clear();
  vg.clear();
  sg.clear();
  std::vector<double> straight(size_t(m.K) * Np * 3);
  node_coordinates(ops, m, straight.data());
  std::vector<double> edge(m.K);
  for (int64_t k = 0; k < m.K; ++k) {
    const double* X = &m.xyz[size_t(k) * 12];
    double e2 = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) d2 += (X[a * 3 + d] - X[b * 3 + d]) * (X[a * 3 + d] - X[b * 3 + d]);
        e2 = std::max(e2, d2);
      }
    edge[k] = std::sqrt(e2);
    double dev = 0.0;
    for (int n = 0; n < Np * 3; ++n) {
      const double v = x[size_t(k) * Np * 3 + n];
      if (!std::isfinite(v)) return "non-finite node position";
      dev = std::max(dev, std::fabs(v - straight[size_t(k) * Np * 3 + n]));
    }
    if (dev > tol * edge[k]) elems.push_back(k);
  }
  // shared face nodes must coincide
  for (int64_t k = 0; k < m.K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int32_t k2 = m.EToE[k * 4 + f];
      if (k2 < 0) continue;
      const int f2 = m.EToF[k * 4 + f], o = m.orient[k * 4 + f];
      for (int i = 0; i < Nfp; ++i) {
        const int n1 = ops.Fmask[f * Nfp + i];
        const int n2 = ops.nbr_node[((size_t(f) * 4 + f2) * 6 + o) * Nfp + i];
        for (int d = 0; d < 3; ++d)
          if (std::fabs(x[(size_t(k) * Np + n1) * 3 + d] - x[(size_t(k2) * Np + n2) * 3 + d]) >
              tol * std::max(edge[k], edge[k2]))
            return "curved node positions do not coincide on a shared face";
      }
    }
  static const double kGrad[4][3] = {{0, 0, -1}, {0, -1, 0}, {1, 1, 1}, {-1, 0, 0}};
  const size_t nc = elems.size();
  vg.resize(nc * Np * 9);
  sg.resize(nc * 4 * Nfp * 4);
  std::vector<double> G(size_t(Np) * 9);
  for (size_t c = 0; c < nc; ++c) {
    const double* X = x + size_t(elems[c]) * Np * 3;
    for (int n = 0; n < Np; ++n) {
      double Jm[3][3];  // Jm[d][a] = d x_d / d r_a
      const double* D[3] = {&ops.Dr[size_t(n) * Np], &ops.Ds[size_t(n) * Np], &ops.Dt[size_t(n) * Np]};
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
          double v = 0.0;
          for (int j = 0; j < Np; ++j) v += D[a][j] * X[j * 3 + d];
          Jm[d][a] = v;
        }
      // inverse by cofactors: G[a][d] = cof(Jm)[d][a] / det
      const double c00 = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
      const double c01 = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
      const double c02 = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
      const double det = Jm[0][0] * c00 + Jm[0][1] * c01 + Jm[0][2] * c02;
      if (!(det > 0.0)) return "curved element with a non-positive Jacobian at a node";
      double* g = &G[size_t(n) * 9];
      g[0 * 3 + 0] = c00 / det;
      g[1 * 3 + 0] = c01 / det;
      g[2 * 3 + 0] = c02 / det;
      g[0 * 3 + 1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
      g[1 * 3 + 1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
      g[2 * 3 + 1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
      g[0 * 3 + 2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
      g[1 * 3 + 2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
      g[2 * 3 + 2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
      for (int i = 0; i < 9; ++i) vg[(c * Np + n) * 9 + i] = float(g[i]);
    }
    for (int f = 0; f < 4; ++f)
      for (int i = 0; i < Nfp; ++i) {
        const double* g = &G[size_t(ops.Fmask[f * Nfp + i]) * 9];
        double nv[3];
        for (int d = 0; d < 3; ++d)
          nv[d] = kGrad[f][0] * g[0 * 3 + d] + kGrad[f][1] * g[1 * 3 + d] + kGrad[f][2] * g[2 * 3 + d];
        const double len = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        float* o = &sg[((c * 4 + f) * Nfp + i) * 4];
        for (int d = 0; d < 3; ++d) o[d] = float(nv[d] / len);
        o[3] = float(len);
      }
  }
  return "";
}

namespace {

// Smallest barycentric coordinate of x in element k's straight-sided image,
// and x's reference coordinates there.
double straight_min_barycentric(const HostMesh& m, int64_t k, const double x[3], double rst[3]) {
  const double* X = &m.xyz[size_t(k) * 12];
  const double* G = &m.drst_dx[size_t(k) * 9];
  const double d[3] = {x[0] - X[0], x[1] - X[1], x[2] - X[2]};
  // x - v0 = sum_a (1 + r_a)/2 (v_a - v0): (1 + r_a) = G[a] . (x - v0)
  double l[4];
  for (int a = 0; a < 3; ++a) l[a + 1] = 0.5 * (G[a * 3] * d[0] + G[a * 3 + 1] * d[1] + G[a * 3 + 2] * d[2]);
  l[0] = 1.0 - l[1] - l[2] - l[3];
  for (int a = 0; a < 3; ++a) rst[a] = 2.0 * l[a + 1] - 1.0;
  return std::min(std::min(l[0], l[1]), std::min(l[2], l[3]));
}

// Smallest barycentric coordinate of the reference point rst.
double ref_min_barycentric(const double rst[3]) {
  const double l0 = -0.5 * (1.0 + rst[0] + rst[1] + rst[2]);
  return std::min(std::min(l0, 0.5 * (1.0 + rst[0])),
                  std::min(0.5 * (1.0 + rst[1]), 0.5 * (1.0 + rst[2])));
}

}  // namespace

int64_t locate_point(const HostMesh& m, const double x[3], double tol, double rst[3]) {
  int64_t best = -1;
  double best_min = -1e300;
  for (int64_t k = 0; k < m.K; ++k) {
    double r[3];
    const double mn = straight_min_barycentric(m, k, x, r);
    if (mn > best_min) {
      best_min = mn;
      best = k;
      for (int a = 0; a < 3; ++a) rst[a] = r[a];
    }
  }
  return best_min >= -tol ? best : -1;
}

int64_t locate_point_curved(const RefOps& ops, const HostMesh& m,
                            const std::vector<int64_t>& curved, const double* xc,
                            const double x[3], double tol, double rst[3]) {
  const int64_t k = locate_point(m, x, tol, rst);
  if (k >= 0 && !std::binary_search(curved.begin(), curved.end(), k)) return k;
  // candidates: curved elements whose straight-sided image is near x, nearest first
  std::vector<std::pair<double, size_t>> near;
  for (size_t i = 0; i < curved.size(); ++i) {
    double r[3];
    const double mn = straight_min_barycentric(m, curved[i], x, r);
    if (mn >= -0.5) near.emplace_back(-mn, i);
  }
  std::stable_sort(near.begin(), near.end(),
                   [](const std::pair<double, size_t>& a, const std::pair<double, size_t>& b) {
                     return a.first < b.first;
                   });
  const int Np = ops.Np;
  int64_t best = -1;
  double best_min = -1e300;
  bool own_failed = false;
  for (const auto& c : near) {
    const int64_t kc = curved[c.second];
    double r[3];
    (void)straight_min_barycentric(m, kc, x, r);
    if (!invert_element_map(ops, xc + c.second * size_t(Np) * 3, x, r)) {
      own_failed = own_failed || kc == k;
      continue;
    }
    const double mn = ref_min_barycentric(r);
    if (mn > best_min) {
      best_min = mn;
      best = kc;
      for (int a = 0; a < 3; ++a) rst[a] = r[a];
    }
  }
  if (best >= 0 && best_min >= -tol) return best;
  return own_failed ? -2 : -1;
}

void interpolation_weights(const RefOps& ops, const double rst[3], double* w) {
  const int N = ops.N, Np = ops.Np;
  std::vector<double> psi(Np);
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k, ++m) {
        double v, vr, vs, vt;
        basis3(i, j, k, rst[0], rst[1], rst[2], v, vr, vs, vt);
        psi[m] = v;
      }
  // u(x) = sum_m psi_m(x) c_m with c = V^-1 u, so w_i = sum_m psi_m(x) Vinv[m][i]
  for (int i = 0; i < Np; ++i) {
    double acc = 0.0;
    for (int mm = 0; mm < Np; ++mm) acc += psi[mm] * ops.Vinv[size_t(mm) * Np + i];
    w[i] = acc;
  }
}

bool invert_element_map(const RefOps& ops, const double* xe, const double x[3], double rst[3]) {
  const int N = ops.N, Np = ops.Np;
  std::vector<double> psi(size_t(4) * Np), w(size_t(4) * Np);
  for (int it = 0; it < 50; ++it) {
    int m = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j)
        for (int k = 0; k <= N - i - j; ++k, ++m)
          basis3(i, j, k, rst[0], rst[1], rst[2], psi[m], psi[Np + m], psi[2 * Np + m],
                 psi[3 * Np + m]);
    // weights of the value and of its r, s, t derivatives at rst
    for (int c = 0; c < 4; ++c)
      for (int n = 0; n < Np; ++n) {
        double acc = 0.0;
        for (int mm = 0; mm < Np; ++mm) acc += psi[size_t(c) * Np + mm] * ops.Vinv[size_t(mm) * Np + n];
        w[size_t(c) * Np + n] = acc;
      }
    double f[3] = {-x[0], -x[1], -x[2]}, J[3][3] = {};
    for (int n = 0; n < Np; ++n)
      for (int d = 0; d < 3; ++d) {
        f[d] += w[n] * xe[n * 3 + d];
        for (int a = 0; a < 3; ++a) J[d][a] += w[size_t(a + 1) * Np + n] * xe[n * 3 + d];
      }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(std::fabs(det) > 0.0)) return false;
    // dr = J^-1 f by cofactors
    const double inv[3][3] = {
        {c00 / det, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det, (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det},
        {c01 / det, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det, (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det},
        {c02 / det, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det, (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det}};
    double step = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double dr = inv[a][0] * f[0] + inv[a][1] * f[1] + inv[a][2] * f[2];
      rst[a] -= dr;
      step = std::max(step, std::fabs(dr));
    }
    if (!std::isfinite(step)) return false;
    if (step <= 1e-13) return true;
  }
  return false;
}

namespace {

// Gauss-Jacobi rule with n points for the weight (1-x)^al on [-1,1]: the
// zeros of P_n^(al,0) by Newton's method from the Chebyshev-Gauss points,
// weights 1 / sum_{k<n} p_k(x)^2 (p_k the orthonormal Jacobi polynomials).
void gauss_jacobi(int n, double al, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double z = -std::cos(M_PI * (2.0 * j + 1.0) / (2.0 * n));
    for (int it = 0; it < 200; ++it) {
      // deflate the zeros already found
      double f = jacobi_norm(z, n, al, 0.0), df = jacobi_norm_deriv(z, n, al, 0.0);
      double sum = 0.0;
      for (int i = 0; i < j; ++i) sum += 1.0 / (z - x[i]);
      const double dz = f / (df - f * sum);
      z -= dz;
      if (std::fabs(dz) < 1e-15) break;
    }
    x[j] = z;
  }
  std::sort(x.begin(), x.end());
  for (int j = 0; j < n; ++j) {
    double s2 = 0.0;
    for (int k = 0; k < n; ++k) {
      const double pk = jacobi_norm(x[j], k, al, 0.0);
      s2 += pk * pk;
    }
    w[j] = 1.0 / s2;
  }
}

// Lagrange basis of the nodes (values, and reference derivatives when d is
// not null: d[a * Np + i]) at a reference point.
void lagrange_at(const RefOps& ops, const double rst[3], double* l, double* d) {
  const int N = ops.N, Np = ops.Np;
  std::vector<double> psi(Np), dpsi(3 * size_t(Np));
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k, ++m)
        basis3(i, j, k, rst[0], rst[1], rst[2], psi[m], dpsi[m], dpsi[Np + m], dpsi[2 * Np + m]);
  for (int i = 0; i < Np; ++i) {
    double v = 0.0, dr = 0.0, ds = 0.0, dt = 0.0;
    for (int mm = 0; mm < Np; ++mm) {
      const double c = ops.Vinv[size_t(mm) * Np + i];
      v += psi[mm] * c;
      dr += dpsi[mm] * c;
      ds += dpsi[Np + mm] * c;
      dt += dpsi[2 * Np + mm] * c;
    }
    l[i] = v;
    if (d) {
      d[i] = dr;
      d[Np + i] = ds;
      d[2 * Np + i] = dt;
    }
  }
}

}  // namespace

std::string build_quadrature(const RefOps& ops, QuadOps& Q) {
  const int N = ops.N, Np = ops.Np, n = N + 1;
  Q.N = N;
  Q.Np = Np;
  // M^-1 of the nodal basis: V V^T (V the orthonormal Vandermonde)
  std::vector<double> V(size_t(Np) * Np);
  {
    std::vector<double> Vi = ops.Vinv;
    if (!invert(Vi, Np)) return "singular Vandermonde inverse";
    V = Vi;
  }
  const std::vector<double> Minv = matmul(V, transpose(V, Np, Np), Np, Np, Np);

  // volume rule: r = (1+a)(1-b)(1-c)/4 - 1, s = (1+b)(1-c)/2 - 1, t = c,
  // dr ds dt = (1-b)/2 ((1-c)/2)^2 da db dc
  std::vector<double> xa, wa, xb, wb, xc, wc;
  gauss_jacobi(n, 0.0, xa, wa);
  gauss_jacobi(n, 1.0, xb, wb);
  gauss_jacobi(n, 2.0, xc, wc);
  Q.Nq = n * n * n;
  Q.xq.clear();
  Q.wq.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double a = xa[i], b = xb[j], c = xc[k];
        Q.xq.push_back(0.25 * (1 + a) * (1 - b) * (1 - c) - 1);
        Q.xq.push_back(0.5 * (1 + b) * (1 - c) - 1);
        Q.xq.push_back(c);
        Q.wq.push_back(wa[i] * wb[j] * wc[k] * 0.5 * 0.25);
      }
  // face rule: Radon's seven-point rule of degree 5 (>= 2N + 1 for N <= 2),
  // symmetric under every permutation of the face's vertices, so the two
  // elements of a face integrate the numerical flux at the same points; as
  // barycentrics on the face's three vertices, weights for area 2
  if (N > 2) return "the face rule covers N <= 2";
  Q.Nfq = 7;
  std::vector<double> fb = {1.0 / 3, 1.0 / 3, 1.0 / 3};  // [Nfq][3]
  Q.wf.assign(1, 2.0 * 9.0 / 40.0);
  const double r15 = std::sqrt(15.0);
  for (int orbit = 0; orbit < 2; ++orbit) {
    const double a = orbit == 0 ? (6 - r15) / 21 : (6 + r15) / 21;
    const double w = orbit == 0 ? (155 - r15) / 1200 : (155 + r15) / 1200;
    const double b = 1 - 2 * a;
    const double pts[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
    for (const auto& pt : pts) {
      fb.insert(fb.end(), pt, pt + 3);
      Q.wf.push_back(2.0 * w);
    }
  }
  auto bary_to_rst = [](const double lam[4], double rst[3]) {
    for (int a = 0; a < 3; ++a) rst[a] = 2.0 * lam[a + 1] - 1.0;
  };

  const int Nq = Q.Nq, Nfq = Q.Nfq;
  std::vector<double> l(Np), d(3 * size_t(Np));
  Q.Bv.assign(size_t(Nq) * Np, 0.0);
  Q.Dw.assign(size_t(3) * Np * Nq, 0.0);
  for (int q = 0; q < Nq; ++q) {
    lagrange_at(ops, &Q.xq[size_t(q) * 3], l.data(), d.data());
    for (int i = 0; i < Np; ++i) Q.Bv[size_t(q) * Np + i] = l[i];
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < Np; ++i) {
        double acc = 0.0;
        for (int j = 0; j < Np; ++j) acc += Minv[size_t(i) * Np + j] * d[size_t(a) * Np + j];
        Q.Dw[(size_t(a) * Np + i) * Nq + q] = acc * Q.wq[q];
      }
  }
  Q.Bf.assign(size_t(4) * Nfq * Np, 0.0);
  Q.Lq.assign(size_t(4) * Np * Nfq, 0.0);
  Q.xf.assign(size_t(4) * Nfq * 3, 0.0);
  for (int f = 0; f < 4; ++f)
    for (int q = 0; q < Nfq; ++q) {
      double lam[4] = {0, 0, 0, 0}, rst[3];
      for (int j = 0; j < 3; ++j) lam[kFaceVerts[f][j]] = fb[size_t(q) * 3 + j];
      bary_to_rst(lam, rst);
      for (int a = 0; a < 3; ++a) Q.xf[(size_t(f) * Nfq + q) * 3 + a] = rst[a];
      lagrange_at(ops, rst, l.data(), nullptr);
      for (int i = 0; i < Np; ++i) Q.Bf[(size_t(f) * Nfq + q) * Np + i] = l[i];
      for (int i = 0; i < Np; ++i) {
        double acc = 0.0;
        for (int j = 0; j < Np; ++j) acc += Minv[size_t(i) * Np + j] * l[j];
        Q.Lq[(size_t(f) * Np + i) * Nfq + q] = acc * Q.wf[q];
      }
    }
  // neighbour's values at my face points: my face vertex j is vertex
  // kPerms[o][j] of the neighbour's face f2
  Q.Bnb.assign(size_t(96) * Nfq * Np, 0.0);
  for (int f = 0; f < 4; ++f)
    for (int f2 = 0; f2 < 4; ++f2)
      for (int o = 0; o < 6; ++o)
        for (int q = 0; q < Nfq; ++q) {
          double lam[4] = {0, 0, 0, 0}, rst[3];
          for (int j = 0; j < 3; ++j) lam[kFaceVerts[f2][kPerms[o][j]]] = fb[size_t(q) * 3 + j];
          bary_to_rst(lam, rst);
          lagrange_at(ops, rst, l.data(), nullptr);
          for (int i = 0; i < Np; ++i)
            Q.Bnb[((size_t((f * 4 + f2) * 6 + o)) * Nfq + q) * Np + i] = l[i];
        }
  return "";
}

}  // namespace dg
