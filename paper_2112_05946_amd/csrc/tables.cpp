// Host-side FP64 operator tables for the FR-SG path.
//
// Physical space (Sec. 3.2-3.3): Legendre-Gauss solution points, Lagrange
// basis, derivative matrix, face values, Radau correction derivatives.
// Nodal/modal transform (Sec. 4, Eq. vandermonde matrix): V[j][k] = Psi_k(r_j)
// with Psi_k = sqrt(2k+1) P_k (orthonormal under dr/2).  Random space
// (Sec. 2.1): Legendre chaos Phi_k = sqrt(2k+1) P_k on the Gauss-Legendre
// rule with weights summing to one; total-degree products in two dimensions.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace frsg {
namespace {

// P_0..P_n at x (Bonnet recurrence)
void legendre(int n, double x, double* P) {
  P[0] = 1.0;
  if (n >= 1) P[1] = x;
  for (int m = 1; m < n; ++m) P[m + 1] = ((2.0 * m + 1.0) * x * P[m] - m * P[m - 1]) / (m + 1.0);
}

// P_0'..P_n' at x from P'_{m+1} = P'_{m-1} + (2m+1) P_m
void legendre_deriv(int n, double x, double* dP) {
  std::vector<double> P(n + 2);
  legendre(n, x, P.data());
  dP[0] = 0.0;
  if (n >= 1) dP[1] = 1.0;
  for (int m = 1; m < n; ++m) dP[m + 1] = dP[m - 1] + (2.0 * m + 1.0) * P[m];
}

// n-point Gauss-Legendre rule by Newton iteration on P_n from Chebyshev-like
// starting values; nodes ascending, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  if (n == 1) {
    w[0] = 2.0;
    return;
  }
  std::vector<double> P(n + 1), dP(n + 1);
  for (int i = 0; i < n; ++i) {
    double xi = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre(n, xi, P.data());
      legendre_deriv(n, xi, dP.data());
      double dx = P[n] / dP[n];
      xi -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    legendre_deriv(n, xi, dP.data());
    x[n - 1 - i] = xi;
    w[n - 1 - i] = 2.0 / ((1.0 - xi * xi) * dP[n] * dP[n]);
  }
}

// ||sqrt(2j+1) P_j||_1 under dr/2 on [-1, 1]: P_j keeps one sign between
// consecutive roots, so it is integrated piece by piece with a (j+1)-point
// Gauss rule (exact for degree j) and the absolute values are summed
double legendre_l1(int j) {
  std::vector<double> cut(1, -1.0), gx, gw, xr, wr;
  if (j > 0) {
    gauss_legendre(j, xr, wr);
    cut.insert(cut.end(), xr.begin(), xr.end());
  }
  cut.push_back(1.0);
  gauss_legendre(j + 1, gx, gw);
  std::vector<double> P(j + 1);
  double total = 0.0;
  for (size_t i = 0; i + 1 < cut.size(); ++i) {
    const double h = 0.5 * (cut[i + 1] - cut[i]), c = 0.5 * (cut[i + 1] + cut[i]);
    double piece = 0.0;
    for (int g = 0; g < j + 1; ++g) {
      legendre(j, c + h * gx[g], P.data());
      piece += gw[g] * P[j];
    }
    total += std::fabs(h * piece);
  }
  return std::sqrt(2.0 * j + 1.0) * 0.5 * total;
}

double lagrange(const std::vector<double>& r, int j, double x) {
  double v = 1.0;
  for (size_t m = 0; m < r.size(); ++m)
    if ((int)m != j) v *= (x - r[m]) / (r[j] - r[m]);
  return v;
}

// Gauss-Jordan inverse with partial pivoting (n small)
bool invert(int n, const std::vector<double>& A, std::vector<double>& Ainv) {
  std::vector<double> a(A);
  Ainv.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    if (a[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[c * n + k], a[piv * n + k]);
        std::swap(Ainv[c * n + k], Ainv[piv * n + k]);
      }
    double d = a[c * n + c];
    for (int k = 0; k < n; ++k) {
      a[c * n + k] /= d;
      Ainv[c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[r * n + k] -= f * a[c * n + k];
        Ainv[r * n + k] -= f * Ainv[c * n + k];
      }
    }
  }
  return true;
}

}  // namespace

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) { gauss_legendre(n, x, w); }
bool invert_matrix(int n, const std::vector<double>& A, std::vector<double>& Ainv) { return invert(n, A, Ainv); }

double exp_filter_term(double eta, double eta_star, double s) {
  if (eta < eta_star) return 0.0;
  return std::pow((eta - eta_star) / (1.0 - eta_star), s);
}

bool build_host_tables(const fr_sg_problem& P, HostTables& T, std::string& err) {
  const int p = P.fr_degree;
  const int n = p + 1;
  T.np1 = n;
  gauss_legendre(n, T.r, T.w);

  // derivative matrix by the barycentric formula: D_ij = (c_i / c_j) / (r_i - r_j), D_ii = sum 1/(r_i - r_m)
  std::vector<double> c(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m)
      if (m != i) c[i] *= (T.r[i] - T.r[m]);
  T.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (i != j) {
        T.D[i * n + j] = (c[i] / c[j]) / (T.r[i] - T.r[j]);
      } else {
        double s = 0.0;
        for (int m = 0; m < n; ++m)
          if (m != i) s += 1.0 / (T.r[i] - T.r[m]);
        T.D[i * n + i] = s;
      }
    }
  T.lL.resize(n);
  T.lR.resize(n);
  for (int j = 0; j < n; ++j) {
    T.lL[j] = lagrange(T.r, j, -1.0);
    T.lR[j] = lagrange(T.r, j, 1.0);
  }
  // Radau: h_L = ((-1)^(p+1) / 2) (P_{p+1} - P_p), h_R(r) = h_L(-r)
  T.dhL.resize(n);
  T.dhR.resize(n);
  std::vector<double> dP(p + 3);
  const double sgn = ((p + 1) % 2 == 0) ? 0.5 : -0.5;
  for (int j = 0; j < n; ++j) {
    legendre_deriv(p + 1, T.r[j], dP.data());
    T.dhL[j] = sgn * (dP[p + 1] - dP[p]);
    legendre_deriv(p + 1, -T.r[j], dP.data());
    T.dhR[j] = -sgn * (dP[p + 1] - dP[p]);
  }
  // Vandermonde of the orthonormal modal basis
  T.V.assign(n * n, 0.0);
  std::vector<double> Pv(n + 1);
  for (int j = 0; j < n; ++j) {
    legendre(p, T.r[j], Pv.data());
    for (int k = 0; k < n; ++k) T.V[j * n + k] = std::sqrt(2.0 * k + 1.0) * Pv[k];
  }
  if (!invert(n, T.V, T.Vinv)) {
    err = "singular Vandermonde matrix";
    return false;
  }

  // random space
  const int Nc = P.gpc_order;
  T.rdim = P.rdim;
  T.kidx.clear();
  if (P.rdim == 1) {
    for (int k = 0; k <= Nc; ++k) T.kidx.push_back({k, 0});
  } else {
    for (int d = 0; d <= Nc; ++d)
      for (int k2 = 0; k2 <= d; ++k2) T.kidx.push_back({d - k2, k2});
  }
  T.M = (int)T.kidx.size();
  T.kdeg.resize(T.M);
  for (int k = 0; k < T.M; ++k) T.kdeg[k] = T.kidx[k][0] + T.kidx[k][1];
  std::vector<double> z1, w1;
  gauss_legendre(P.nq1d, z1, w1);
  for (auto& v : w1) v *= 0.5;
  const int nq = P.nq1d;
  T.Nq = (P.rdim == 1) ? nq : nq * nq;
  T.z.assign((size_t)T.Nq * P.rdim, 0.0);
  T.wq.assign(T.Nq, 0.0);
  // 1D chaos values at the 1D nodes: chi[k][a] = sqrt(2k+1) P_k(z1_a)
  std::vector<double> chi((size_t)(Nc + 1) * nq), Pc(Nc + 2);
  for (int a = 0; a < nq; ++a) {
    legendre(Nc, z1[a], Pc.data());
    for (int k = 0; k <= Nc; ++k) chi[k * nq + a] = std::sqrt(2.0 * k + 1.0) * Pc[k];
  }
  T.Phi.assign((size_t)T.M * T.Nq, 0.0);
  if (P.rdim == 1) {
    for (int q = 0; q < nq; ++q) {
      T.z[q] = z1[q];
      T.wq[q] = w1[q];
    }
    for (int k = 0; k < T.M; ++k)
      for (int q = 0; q < nq; ++q) T.Phi[k * T.Nq + q] = chi[T.kidx[k][0] * nq + q];
  } else {
    for (int b = 0; b < nq; ++b)
      for (int a = 0; a < nq; ++a) {
        int q = a + nq * b;
        T.z[2 * q] = z1[a];
        T.z[2 * q + 1] = z1[b];
        T.wq[q] = w1[a] * w1[b];
      }
    for (int k = 0; k < T.M; ++k)
      for (int b = 0; b < nq; ++b)
        for (int a = 0; a < nq; ++a)
          T.Phi[k * T.Nq + a + nq * b] = chi[T.kidx[k][0] * nq + a] * chi[T.kidx[k][1] * nq + b];
  }
  T.PW.resize(T.Phi.size());
  for (int k = 0; k < T.M; ++k)
    for (int q = 0; q < T.Nq; ++q) T.PW[k * T.Nq + q] = T.Phi[k * T.Nq + q] * T.wq[q];

  // per (mode, spatial modal index) tables for the sensor and the filters
  const int dim = (P.equation == FRSG_EULER2D) ? 2 : 1;
  const int nsp = (dim == 2) ? n * n : n;
  T.filt.assign((size_t)T.M * nsp, 1.0);
  T.shell.assign((size_t)T.M * nsp, 0.0);
  const double a1 = 1.0 / (P.eps1 * n * n * (n - 1) * (n - 1));
  const double a2 = (Nc > 0) ? 1.0 / (P.eps2 * Nc * Nc * (Nc + 1) * (Nc + 1)) : 0.0;
  for (int k = 0; k < T.M; ++k) {
    const int kk = T.kdeg[k];
    for (int j = 0; j < nsp; ++j) {
      int dj[2] = {j % n, (dim == 2) ? j / n : 0};
      int jmax = std::max(dj[0], dim == 2 ? dj[1] : 0);
      T.shell[k * nsp + j] = (jmax == p || kk == Nc) ? 1.0 : 0.0;
      if (P.filter == FRSG_FILTER_EXP) {
        double ex = 0.0;
        for (int d = 0; d < dim; ++d) ex += exp_filter_term((double)dj[d] / p, P.nstar / p, P.s);
        double ez = (Nc > 0) ? exp_filter_term((double)kk / Nc, P.nstar / Nc, P.s) : 0.0;
        T.filt[k * nsp + j] = ex + ez;
      } else if (P.filter == FRSG_FILTER_L2) {
        long sx = 0;
        for (int d = 0; d < dim; ++d) sx += (long)dj[d] * dj[d] * (dj[d] + 1) * (dj[d] + 1);
        double pen = a1 * (double)sx + a2 * kk * kk * (kk + 1) * (kk + 1);
        T.filt[k * nsp + j] = 1.0 / (1.0 + pen);
      } else if (P.filter == FRSG_FILTER_LASSO) {
        // ||Psi_j Phi_k||_1 (one physical, one random dimension): the kernels
        // form the data-dependent factors from it
        T.filt[k * nsp + j] = legendre_l1(j) * legendre_l1(kk);
      }
    }
  }
  // derivative matrix that also removes the interpolated flux at both faces
  T.Dt.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < n; ++c) T.Dt[i * n + c] = T.D[i * n + c] - T.dhL[i] * T.lL[c] - T.dhR[i] * T.lR[c];
  T.cmax.assign(T.M, 0.0);
  for (int k = 0; k < T.M; ++k)
    for (int q = 0; q < T.Nq; ++q) T.cmax[k] = std::max(T.cmax[k], std::fabs(T.Phi[k * T.Nq + q]));
  T.PhiT.assign((size_t)T.Nq * T.M, 0.0);
  T.PWT.assign((size_t)T.Nq * T.M, 0.0);
  for (int k = 0; k < T.M; ++k)
    for (int q = 0; q < T.Nq; ++q) {
      T.PhiT[q * T.M + k] = T.Phi[k * T.Nq + q];
      T.PWT[q * T.M + k] = T.PW[k * T.Nq + q];
    }
  T.swts.assign(nsp, 0.0);
  for (int j = 0; j < nsp; ++j)
    T.swts[j] = (dim == 1) ? T.w[j] / 2.0 : (T.w[j % n] / 2.0) * (T.w[j / n] / 2.0);
  return true;
}

}  // namespace frsg
