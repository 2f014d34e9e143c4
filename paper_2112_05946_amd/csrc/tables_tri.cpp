// Host tables of the triangle path (Sec. 3.1 reference triangle (-1,-1), (1,-1),
// (-1,1); Sec. 3.5 multi-dimensional FR), FP64.
//
// Modal basis: the orthonormal Proriol-Koornwinder-Dubiner polynomials
// psi_ij(r, s) = 2 P_i(a) P_j^(2i+1,0)(b) (1-b)^i, a = 2(1+r)/(1-s) - 1, b = s,
// with orthonormal Jacobi polynomials (unit norm under (1/2) int_T).  Solution
// points: warp-and-blend nodes (equispaced lattice, edge displacements to the
// Legendre-Gauss-Lobatto points blended into the interior, no optimisation
// parameter).  Correction fields: the DG-equivalent choice, whose divergence at
// the solution points is the lifting (1/2)(L_f/2) w_k sum_m psi_m(r_j) psi_m(x_fk)
// (the reproducing kernel of the degree-p polynomials on T).
#include <cmath>

#include "internal.hpp"

namespace frsg {
namespace {

constexpr double kRefFaceLen[3] = {2.0, 2.8284271247461903, 2.0};

// orthonormal Jacobi polynomials P_0..P_N^(al,be)(x), weight (1-x)^al (1+x)^be on [-1, 1]
void jacobi(int N, double al, double be, double x, double* P) {
  P[0] = std::sqrt(std::pow(2.0, -al - be - 1.0) * std::tgamma(al + be + 2.0) /
                   (std::tgamma(al + 1.0) * std::tgamma(be + 1.0)));
  if (N == 0) return;
  P[1] = P[0] * ((al + be + 2.0) * x / 2.0 + (al - be) / 2.0) * std::sqrt((al + be + 3.0) / ((al + 1.0) * (be + 1.0)));
  double aold = 2.0 / (2.0 + al + be) * std::sqrt((al + 1.0) * (be + 1.0) / (al + be + 3.0));
  for (int i = 1; i < N; ++i) {
    const double h1 = 2.0 * i + al + be;
    const double anew = 2.0 / (h1 + 2.0) *
                        std::sqrt((i + 1.0) * (i + 1.0 + al + be) * (i + 1.0 + al) * (i + 1.0 + be) /
                                  ((h1 + 1.0) * (h1 + 3.0)));
    const double bnew = -(al * al - be * be) / (h1 * (h1 + 2.0));
    P[i + 1] = (-aold * P[i - 1] + (x - bnew) * P[i]) / anew;
    aold = anew;
  }
}

double jacobi_n(int n, double al, double be, double x) {
  double P[2 * kTriMaxDeg + 4];
  jacobi(n, al, be, x, P);
  return P[n];
}

// d/dx of the orthonormal P_n^(al,be) = sqrt(n (n+al+be+1)) P_{n-1}^(al+1,be+1)
double jacobi_d(int n, double al, double be, double x) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + al + be + 1.0)) * jacobi_n(n - 1, al + 1.0, be + 1.0, x);
}

// all modes i + j <= p at (r, s): values and gradients
void pkd(int p, double r, double s, std::vector<double>& v, std::vector<double>& dr, std::vector<double>& ds) {
  const double a = (s < 1.0) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  const double b = s, om = 1.0 - b;
  v.clear();
  dr.clear();
  ds.clear();
  for (int i = 0; i <= p; ++i)
    for (int j = 0; i + j <= p; ++j) {
      const double f = jacobi_n(i, 0.0, 0.0, a), fp = jacobi_d(i, 0.0, 0.0, a);
      const double g = jacobi_n(j, 2.0 * i + 1.0, 0.0, b), gp = jacobi_d(j, 2.0 * i + 1.0, 0.0, b);
      const double omi = std::pow(om, i);
      const double omi1 = i >= 1 ? std::pow(om, i - 1) : 0.0;
      v.push_back(2.0 * f * g * omi);
      dr.push_back(i >= 1 ? 4.0 * fp * g * omi1 : 0.0);
      ds.push_back((i >= 1 ? 2.0 * fp * (1.0 + a) * g * omi1 : 0.0) + 2.0 * f * (gp * omi - i * g * omi1));
    }
}

// Legendre polynomial P_n and its derivative at x
void legendre_pd(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int m = 1; m < n; ++m) {
    const double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// N+1 Legendre-Gauss-Lobatto points: -1, 1 and the roots of P_N' (Newton from
// the Chebyshev-Gauss-Lobatto points, P_N'' = (2x P_N' - N(N+1) P_N) / (1 - x^2))
std::vector<double> lgl(int N) {
  std::vector<double> x(N + 1);
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double xi = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre_pd(N, xi, P, dP);
      const double d2P = (2.0 * xi * dP - N * (N + 1.0) * P) / (1.0 - xi * xi);
      const double dx = dP / d2P;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    x[i] = xi;
  }
  return x;
}

// edge warp at x in [-1, 1], divided by the edge blend 1 - x^2 (0 at the ends)
double warp(int N, const std::vector<double>& xl, double x) {
  double w = 0.0;
  for (int i = 0; i <= N; ++i) {
    double li = 1.0;
    const double xi = -1.0 + 2.0 * i / N;
    for (int m = 0; m <= N; ++m)
      if (m != i) li *= (x - (-1.0 + 2.0 * m / N)) / (xi - (-1.0 + 2.0 * m / N));
    w += (xl[i] - xi) * li;
  }
  return std::fabs(x) < 1.0 - 1e-10 ? w / (1.0 - x * x) : 0.0;
}

// warp-and-blend nodes, rows of constant s (b = 0..N) and r increasing in a row
void warp_blend(int N, std::vector<double>& r, std::vector<double>& s) {
  const std::vector<double> xl = lgl(N);
  r.clear();
  s.clear();
  const double sq3 = std::sqrt(3.0);
  for (int b = 0; b <= N; ++b)
    for (int a = 0; a + b <= N; ++a) {
      const double l2 = (double)a / N, l3 = (double)b / N, l1 = 1.0 - l2 - l3;
      // equilateral triangle, vertices (-1, -1/sqrt3), (1, -1/sqrt3), (0, 2/sqrt3) for l1, l2, l3
      double X = -l1 + l2, Y = (-l1 - l2 + 2.0 * l3) / sq3;
      const double lam[3] = {l1, l2, l3};
      for (int e = 0; e < 3; ++e) {
        const double la = lam[e], lb = lam[(e + 1) % 3];
        const double wv = 4.0 * la * lb * warp(N, xl, lb - la);
        const double ang = 2.0 * M_PI * e / 3.0;
        X += std::cos(ang) * wv;
        Y += std::sin(ang) * wv;
      }
      const double m3 = (sq3 * Y + 1.0) / 3.0;
      const double m2 = (X + 1.0 - m3) / 2.0;
      const double m1 = 1.0 - m2 - m3;
      r.push_back(-m1 + m2 - m3);
      s.push_back(-m1 - m2 + m3);
    }
}

void face_point(int f, double t, double& r, double& s) {
  if (f == 0) {
    r = t;
    s = -1.0;
  } else if (f == 1) {
    r = -t;
    s = t;
  } else {
    r = -1.0;
    s = -t;
  }
}

}  // namespace

bool build_tri_tables(const fr_sg_problem& P, TriTables& T, std::string& err) {
  const int p = P.fr_degree;
  T.p = p;
  T.np = (p + 1) * (p + 2) / 2;
  T.nfp = p + 1;
  const int n = T.np, nf = 3 * T.nfp;
  warp_blend(p, T.r, T.s);
  std::vector<double> V(n * n), Vr(n * n), Vs(n * n), v, dr, ds;
  for (int j = 0; j < n; ++j) {
    pkd(p, T.r[j], T.s[j], v, dr, ds);
    for (int m = 0; m < n; ++m) {
      V[j * n + m] = v[m];
      Vr[j * n + m] = dr[m];
      Vs[j * n + m] = ds[m];
    }
  }
  std::vector<double> Vi;
  if (!invert_matrix(n, V, Vi)) {
    err = "singular Vandermonde matrix on the triangle";
    return false;
  }
  T.Dr.assign(n * n, 0.0);
  T.Ds.assign(n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m) {
        T.Dr[j * n + i] += Vr[j * n + m] * Vi[m * n + i];
        T.Ds[j * n + i] += Vs[j * n + m] * Vi[m * n + i];
      }
  std::vector<double> tq, wq;
  gauss_rule(T.nfp, tq, wq);
  T.Lf.assign(nf * n, 0.0);
  T.lift.assign(n * nf, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int k = 0; k < T.nfp; ++k) {
      double fr, fs;
      face_point(f, tq[k], fr, fs);
      pkd(p, fr, fs, v, dr, ds);
      const int fk = f * T.nfp + k;
      for (int i = 0; i < n; ++i)
        for (int m = 0; m < n; ++m) T.Lf[fk * n + i] += v[m] * Vi[m * n + i];
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int m = 0; m < n; ++m) acc += V[j * n + m] * v[m];
        T.lift[j * nf + fk] = kRefFaceLen[f] / 4.0 * wq[k] * acc;
      }
    }
  // mode (0, 0) is first and equals 1: the element mean is its coefficient
  T.mean_w.assign(Vi.begin(), Vi.begin() + n);
  T.V = V;
  T.Vinv = Vi;

  // mesh: orientation, links, boundary kinds; per-element geometry
  const int E = P.n_tri;
  T.geo.assign((size_t)E * kTriGeo, 0.0);
  T.nbr.assign((size_t)E * 6, 0);
  T.xy_pts.assign((size_t)E * n * 2, 0.0);
  for (int e = 0; e < E; ++e) {
    const double* X = P.tri_xy + 6 * e;
    for (int j = 0; j < n; ++j) {
      // x = lam1 x1 + lam2 x2 + lam3 x3, lam1 = -(r+s)/2, lam2 = (r+1)/2, lam3 = (s+1)/2
      const double l1 = -(T.r[j] + T.s[j]) / 2.0, l2 = (T.r[j] + 1.0) / 2.0, l3 = (T.s[j] + 1.0) / 2.0;
      T.xy_pts[((size_t)e * n + j) * 2] = l1 * X[0] + l2 * X[2] + l3 * X[4];
      T.xy_pts[((size_t)e * n + j) * 2 + 1] = l1 * X[1] + l2 * X[3] + l3 * X[5];
    }
    const double xr = (X[2] - X[0]) / 2.0, yr = (X[3] - X[1]) / 2.0;
    const double xs = (X[4] - X[0]) / 2.0, ys = (X[5] - X[1]) / 2.0;
    const double det = xr * ys - xs * yr;
    if (!(det > 0.0)) {
      err = "triangle " + std::to_string(e) + " is clockwise or degenerate";
      return false;
    }
    double* g = &T.geo[(size_t)e * kTriGeo];
    g[kGeoRx] = ys / det;
    g[kGeoRy] = -xs / det;
    g[kGeoSx] = -yr / det;
    g[kGeoSy] = xr / det;
    g[kGeoDet] = det;
    double perim = 0.0;
    for (int f = 0; f < 3; ++f) {
      const int f1 = (f + 1) % 3;
      const double dx = X[2 * f1] - X[2 * f], dy = X[2 * f1 + 1] - X[2 * f + 1];
      const double L = std::sqrt(dx * dx + dy * dy);
      g[kGeoN0 + 2 * f] = dy / L;
      g[kGeoN0 + 2 * f + 1] = -dx / L;
      g[kGeoSc0 + f] = L / kRefFaceLen[f] / det;
      perim += L;
    }
    g[kGeoDin] = 4.0 * (2.0 * det) / perim;
    for (int f = 0; f < 3; ++f) {
      const int nb = P.tri_nbr[3 * e + f];
      const int nf_ = P.tri_nbr_face[3 * e + f];
      if (nb >= 0) {
        if (nb >= E || nf_ < 0 || nf_ > 2 || P.tri_nbr[3 * nb + nf_] != e || P.tri_nbr_face[3 * nb + nf_] != f) {
          err = "triangle " + std::to_string(e) + " face " + std::to_string(f) + ": neighbour link not mutual";
          return false;
        }
      } else {
        const int side = -1 - nb;
        if (side > 3) {
          err = "triangle " + std::to_string(e) + " face " + std::to_string(f) + ": boundary side out of range";
          return false;
        }
        if (P.bc[side] == FRSG_BC_PERIODIC) {
          err = "boundary face on a side with periodic bc (periodicity comes from the neighbour links)";
          return false;
        }
      }
      T.nbr[(size_t)e * 6 + f] = nb;
      T.nbr[(size_t)e * 6 + 3 + f] = nb >= 0 ? nf_ : 0;
    }
  }
  return true;
}

// Sensor shell, filter factors and element-mean weights for triangles, in place of
// the tensor-product ones: a mode of the orthonormal basis carries its total
// degree d (i + j of psi_ij) where a quadrilateral mode carries one degree per
// direction.  Exponential: exponent (d/p)^s + (|k|/N_c)^s; L2: 1 / (1 + d^2 (d+1)^2
// / (eps1 p^2 (p+1)^2) + |k|^2 (|k|+1)^2 / (eps2 N_c^2 (N_c+1)^2)); shell: d = p or
// |k| = N_c; element mean: the coefficient of psi_00 (= 1).
void tri_filter_tables(const fr_sg_problem& P, const TriTables& R, HostTables& T) {
  const int p = R.p, n = R.np, Nc = P.gpc_order;
  std::vector<int> deg;
  for (int i = 0; i <= p; ++i)
    for (int j = 0; i + j <= p; ++j) deg.push_back(i + j);
  T.filt.assign((size_t)T.M * n, 1.0);
  T.shell.assign((size_t)T.M * n, 0.0);
  const double a1 = 1.0 / (P.eps1 * (p + 1.0) * (p + 1.0) * p * p);
  const double a2 = (Nc > 0) ? 1.0 / (P.eps2 * Nc * Nc * (Nc + 1.0) * (Nc + 1.0)) : 0.0;
  for (int k = 0; k < T.M; ++k) {
    const int kk = T.kdeg[k];
    for (int m = 0; m < n; ++m) {
      const int d = deg[m];
      T.shell[k * n + m] = (d == p || kk == Nc) ? 1.0 : 0.0;
      if (P.filter == FRSG_FILTER_EXP)
        T.filt[k * n + m] = exp_filter_term((double)d / p, P.nstar / p, P.s) +
                            ((Nc > 0) ? exp_filter_term((double)kk / Nc, P.nstar / Nc, P.s) : 0.0);
      else if (P.filter == FRSG_FILTER_L2)
        T.filt[k * n + m] = 1.0 / (1.0 + a1 * d * d * (d + 1.0) * (d + 1.0) + a2 * kk * kk * (kk + 1.0) * (kk + 1.0));
    }
  }
  T.swts = R.mean_w;
}

}  // namespace frsg
