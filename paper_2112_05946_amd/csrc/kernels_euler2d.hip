// Fused FR-SG stage kernel for the 2D Euler equations on quadrilaterals with
// p = 3 (4 x 4 Legendre-Gauss solution points), any gPC size M and random
// node count NQ fixed at compile time.
//
// One kernel per SSP-RK3 stage does the whole right-hand side (Sec. 2.1, Sec.
// 3.2-3.5) and the stage epilogue, reading each input coefficient from HBM
// once and writing each output coefficient once:
//
//   * a workgroup owns a 4 x 4 tile of elements; thread (e, j) holds the 4 x M
//     gPC coefficients of solution point j of element e in registers;
//   * for each random node q: the gPC expansion at the node (Eq. polynomial
//     chaos), the fluxes F, G there (Eq. local direct flux), solution traces at
//     the 16 flux points of each element by Lagrange interpolation, the
//     Lax-Friedrichs flux per node (Sec. 3.3), and the nodal residual
//       R = -(1/Jx) [Dt F + F*_L h_L' + F*_R h_R']_x - (1/Jy) [...]_y,
//     with Dt = D - h_L' l(-1)^T - h_R' l(+1)^T the derivative matrix that
//     already subtracts the interpolated discontinuous flux at the faces
//     (Sec. 3.4: the correction (F* - F^D) h' split into F* h' and -F^D h');
//     R is Galerkin-projected on the fly (Eq. discrete expectation value),
//     so the residual of the whole stage is never stored;
//   * traces of elements outside the tile come from their modal face traces,
//     interpolated once per stage (the interpolation and the chaos expansion
//     are both linear, so the order does not matter);
//   * epilogue: SSP-RK3 combination, then the positivity limiter (Sec. 4.3) on
//     stage outputs, or, after the third stage, the detector (Sec. 4.2), the
//     modal filter (Sec. 4.1), the limiter and the CFL maximum of the new
//     state for the next step.
//
// The limiter decision is first taken from rigorous modal bounds of density,
// momentum and energy at every solution and flux point (|Phi_k| <= max_q
// |Phi_k(z_q)|); only elements whose bound comes within a safety margin of the
// threshold evaluate density and pressure node by node, so both routes give the
// same decision as the node-by-node test.
//
// Exchanges inside an element use DPP: the 16 threads of an element form one
// 16-lane DPP row, quad_perm rotations move along x (a) and row_ror:4k along y
// (b).  Exchanges between elements of the tile go through LDS.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace frsg {
namespace {

constexpr int NP = 4;
constexpr int NSP = 16;
constexpr int TE = 16;      // elements per tile (4 x 4)
constexpr int BLK = 256;    // threads per workgroup

// ---------------------------------------------------------------------------
// lane exchange within an element row of 16 lanes, lane r = a + 4 b
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xf, 0xf, false);
}
// value at point ((a + k) & 3, b)
template <int K>
__device__ __forceinline__ double xrot(double v) {
  if constexpr (K == 0) return v;
  else if constexpr (K == 1) return dpp<0x39>(v);
  else if constexpr (K == 2) return dpp<0x4E>(v);
  else return dpp<0x93>(v);
}
// value at point (a, (b - k) & 3)
template <int K>
__device__ __forceinline__ double yrot(double v) {
  if constexpr (K == 0) return v;
  else return dpp<0x120 + 4 * K>(v);
}

// sum_c w[c] v(c, b) with wx[k] = w[(a + k) & 3]
__device__ __forceinline__ double xdot(const double* wx, double v) {
  return wx[0] * v + wx[1] * xrot<1>(v) + wx[2] * xrot<2>(v) + wx[3] * xrot<3>(v);
}
// sum_c w[c] v(a, c) with wy[k] = w[(b - k) & 3]
__device__ __forceinline__ double ydot(const double* wy, double v) {
  return wy[0] * v + wy[1] * yrot<1>(v) + wy[2] * yrot<2>(v) + wy[3] * yrot<3>(v);
}
__device__ __forceinline__ double xmin4(double v) {
  return fmin(fmin(v, xrot<1>(v)), fmin(xrot<2>(v), xrot<3>(v)));
}
__device__ __forceinline__ double ymin4(double v) {
  return fmin(fmin(v, yrot<1>(v)), fmin(yrot<2>(v), yrot<3>(v)));
}
__device__ __forceinline__ double xmax4(double v) {
  return fmax(fmax(v, xrot<1>(v)), fmax(xrot<2>(v), xrot<3>(v)));
}
__device__ __forceinline__ double ymax4(double v) {
  return fmax(fmax(v, yrot<1>(v)), fmax(yrot<2>(v), yrot<3>(v)));
}

__device__ __forceinline__ double xsum4(double v) { return v + xrot<1>(v) + xrot<2>(v) + xrot<3>(v); }
__device__ __forceinline__ double ysum4(double v) { return v + yrot<1>(v) + yrot<2>(v) + yrot<3>(v); }
// value of lane 0 of this lane's 16-lane row (makes per-element sums identical on all lanes)
__device__ __forceinline__ double row_bcast0(double v) { return __shfl(v, (int)(threadIdx.x & ~15u)); }

// per-lane rotated copies of a 4-vector for xdot / ydot
struct Rot4 {
  double x[4];  // w[(a + k) & 3]
  double y[4];  // w[(b - k) & 3]
};
__device__ __forceinline__ void make_rot(const double* w, int a, int b, Rot4& r) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r.x[k] = w[(a + k) & 3];
    r.y[k] = w[(b - k) & 3];
  }
}

__device__ __forceinline__ double euler_p(const double* U, double g) {
  const double kin = 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0];
  return (g - 1.0) * (U[3] - kin);
}

// flux F (x) and G (y) of the 2D Euler equations
__device__ __forceinline__ void euler_fg(const double* U, double* F, double* G, double g) {
  const double rho = U[0], mx = U[1], my = U[2], E = U[3];
  const double p = euler_p(U, g);
  const double vx = mx / rho, vy = my / rho;
  F[0] = mx;
  F[1] = mx * vx + p;
  F[2] = my * vx;
  F[3] = (E + p) * vx;
  G[0] = my;
  G[1] = mx * vy;
  G[2] = my * vy + p;
  G[3] = (E + p) * vy;
}

// ---------------------------------------------------------------------------
// arguments
// ---------------------------------------------------------------------------
struct StageArgs {
  const double* in;          // right-hand-side input state (already limited)
  const double* u;           // u^n for the stage combination
  double* out;               // output state (may equal u in stage 3)
  double cu, cw;             // out = cu u + cw (in + dt R)
  int stage;                 // 0: right-hand side only; 1, 2: limited stage output; 3: end of step
  unsigned char* flag_lim;   // per element: limiter acted on the output (stages 1-3)
  unsigned char* flag_filt;  // per element: filter acted (stage 3)
  unsigned long long* lam_next;  // stage 3: CFL accumulator of the new state (may be null)
  const double* Dt;          // 4 x 4 modified derivative matrix
  const double* cmax;        // [M] max_q |Phi_k(z_q)|
};

// ---------------------------------------------------------------------------
// positivity limiter on the 16 lanes of one element (Sec. 4.3)
// o[s][k]: this lane's coefficients (solution point j = a + 4 b)
// returns 1 on lanes of elements that were limited
// ---------------------------------------------------------------------------
template <int M, int NQ>
__device__ int limit_element(const KParams& P, double (&o)[4][M], int a, int b, const Rot4& rw, const Rot4& rl,
                             const Rot4& rr, const double* cmax, bool active) {
  const double g = P.gamma;
  // element x random mean: sum_j (w_a/2)(w_b/2) o[s][0](j)
  double ub[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) ub[s] = row_bcast0(ydot(rw.y, xdot(rw.x, o[s][0])));
  const double pb = euler_p(ub, g);
  const bool realizable = ub[0] > 0.0 && pb > 0.0 && isfinite(ub[0]) && isfinite(ub[1]) && isfinite(ub[2]) &&
                          isfinite(ub[3]);
  if (active && !realizable && a == 0 && b == 0) atomicOr(P.status, kStatusNotRealizable);
  const double eps = fmin(1e-8, fmin(ub[0], pb));

  // rigorous bounds: value(z) = mean + sum_{k>=1} c_k Phi_k(z), |Phi_k(z_q)| <= cmax_k
  double mean[4], var[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    mean[s] = o[s][0];
    double v = 0.0;
#pragma unroll
    for (int k = 1; k < M; ++k) v += fabs(o[s][k]) * cmax[k];
    var[s] = v;
  }
  auto safe = [&](const double* mn, const double* vr) {
    const double rlo = mn[0] - vr[0];
    const double elo = mn[3] - vr[3];
    const double mx = fabs(mn[1]) + vr[1];
    const double my = fabs(mn[2]) + vr[2];
    const double tol_r = 1e-10 * (fabs(mn[0]) + vr[0]) + 1e-300;
    if (!(rlo > eps + tol_r)) return false;
    const double kin = 0.5 * (mx * mx + my * my) / rlo;
    const double plo = (g - 1.0) * (elo - kin);
    const double tol_p = 1e-10 * (g - 1.0) * (fabs(mn[3]) + vr[3] + kin);
    return plo > eps + tol_p;
  };
  bool ok = safe(mean, var);
  // flux points on this lane's row (x faces) and column (y faces)
  {
    double mn[4], vr[4];
    Rot4 al, ar;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      al.x[k] = fabs(rl.x[k]);
      al.y[k] = fabs(rl.y[k]);
      ar.x[k] = fabs(rr.x[k]);
      ar.y[k] = fabs(rr.y[k]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      mn[s] = xdot(rl.x, mean[s]);
      vr[s] = xdot(al.x, var[s]);
    }
    ok = ok && safe(mn, vr);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      mn[s] = xdot(rr.x, mean[s]);
      vr[s] = xdot(ar.x, var[s]);
    }
    ok = ok && safe(mn, vr);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      mn[s] = ydot(rl.y, mean[s]);
      vr[s] = ydot(al.y, var[s]);
    }
    ok = ok && safe(mn, vr);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      mn[s] = ydot(rr.y, mean[s]);
      vr[s] = ydot(ar.y, var[s]);
    }
    ok = ok && safe(mn, vr);
  }
  // element-wide: every lane of the row must be safe
  double okd = ok ? 1.0 : 0.0;
  okd = ymin4(xmin4(okd));
  bool need = active && realizable && okd < 0.5;
  if (__ballot(need) == 0) return 0;

  // node-by-node test on the elements that need it (all lanes of the wave take part)
  const double* Phi = P.tab.Phi;
  double rmin = INFINITY, pmin = INFINITY;
  for (int q = 0; q < NQ; ++q) {
    double U[4], TxL[4], TxR[4], TyL[4], TyR[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) acc += o[s][k] * Phi[k * NQ + q];
      U[s] = acc;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      TxL[s] = xdot(rl.x, U[s]);
      TxR[s] = xdot(rr.x, U[s]);
      TyL[s] = ydot(rl.y, U[s]);
      TyR[s] = ydot(rr.y, U[s]);
    }
    rmin = fmin(rmin, fmin(fmin(U[0], TxL[0]), fmin(TxR[0], fmin(TyL[0], TyR[0]))));
    pmin = fmin(pmin, fmin(fmin(euler_p(U, g), euler_p(TxL, g)),
                           fmin(euler_p(TxR, g), fmin(euler_p(TyL, g), euler_p(TyR, g)))));
  }
  rmin = ymin4(xmin4(rmin));
  pmin = ymin4(xmin4(pmin));
  const bool on = need && (fmin(rmin, pmin) < eps);
  if (__ballot(on) == 0) return 0;
  const double beta1 = (rmin >= eps) ? 1.0 : (ub[0] - eps) / (ub[0] - rmin);
  double bmin = 1.0;
  for (int q = 0; q < NQ; ++q) {
    double U[4], T[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) acc += o[s][k] * Phi[k * NQ + q];
      U[s] = acc;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      T[0][s] = xdot(rl.x, U[s]);
      T[1][s] = xdot(rr.x, U[s]);
      T[2][s] = ydot(rl.y, U[s]);
      T[3][s] = ydot(rr.y, U[s]);
    }
    U[0] = beta1 * (U[0] - ub[0]) + ub[0];
    if (euler_p(U, g) < eps) bmin = fmin(bmin, pressure_root<kEuler2>(ub, U, eps, g));
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      T[f][0] = beta1 * (T[f][0] - ub[0]) + ub[0];
      if (euler_p(T[f], g) < eps) bmin = fmin(bmin, pressure_root<kEuler2>(ub, T[f], eps, g));
    }
  }
  const double beta2 = ymin4(xmin4(bmin));
  if (on) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double m0 = (k == 0) ? 1.0 : 0.0;
      o[0][k] = beta1 * (o[0][k] - ub[0] * m0) + ub[0] * m0;
#pragma unroll
      for (int s = 0; s < 4; ++s) o[s][k] = beta2 * (o[s][k] - ub[s] * m0) + ub[s] * m0;
    }
  }
  return on ? 1 : 0;
}

// ---------------------------------------------------------------------------
// detector + modal filter on one element (Sec. 4.1, 4.2)
// ---------------------------------------------------------------------------
template <int M>
__device__ int sensor_filter_element(const KParams& P, double (&o)[4][M], int j, const Rot4& rvi, const Rot4& rv,
                                     const double* lam, bool active) {
  // spatial modal coefficients of the first state: (V^-1 x V^-1) per chaos mode
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double t = ydot(rvi.y, xdot(rvi.x, o[0][k]));
    const double e2 = t * t;
    num += e2 * P.tab.shell[k * NSP + j];
    den += e2;
  }
  // sums over the 16 lanes of the element
  num = row_bcast0(ysum4(xsum4(num)));
  den = row_bcast0(ysum4(xsum4(den)));
  bool flag = (P.sensor == FRSG_SENSOR_ALWAYS) || (den > 0.0 && num / den > P.sensor_thr);
  flag = flag && active;
  if (__ballot(flag) == 0) return 0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double t = ydot(rvi.y, xdot(rvi.x, o[s][k])) * lam[k * NSP + j];
      const double back = ydot(rv.y, xdot(rv.x, t));
      if (flag) o[s][k] = back;
    }
  }
  return flag ? 1 : 0;
}

// ---------------------------------------------------------------------------
// the stage kernel
// ---------------------------------------------------------------------------
template <int M, int NQ>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_stage2d(KParams P, StageArgs A) {
  __shared__ double sU[2][TE][NSP][4];
  __shared__ double sF[2][TE][NSP][4];
  __shared__ double sG[2][TE][NSP][4];
  __shared__ double sH[2][16][NP][4];
  __shared__ double sFs[TE][NSP][4];
  __shared__ double sLam[M * NSP];
  __shared__ double sRed[BLK / 64];

  const int tid = threadIdx.x;
  const int le = tid >> 4, j = tid & 15;
  const int a = j & 3, b = j >> 2;
  const int lx = le & 3, ly = le >> 2;
  const int ntx = P.nx / 4;
  // XCD-aware order: consecutive workgroups go to different XCDs, so give each
  // XCD a contiguous band of tiles (neighbouring halos then share its L2)
  const int ntiles = ntx * (P.ny / 4);
  int tile = blockIdx.x;
  {
    const int per = (ntiles + 7) / 8;
    const int t2 = (tile % 8) * per + tile / 8;
    if (ntiles % 8 == 0) tile = t2;
  }
  const int tx = tile % ntx, ty = tile / ntx;
  const int ix = 4 * tx + lx, iy = 4 * ty + ly;
  const int e = iy * P.nx + ix;
  const long EN = (long)P.E * NSP;
  const double g = P.gamma;
  const double* Phi = P.tab.Phi;
  const double* PW = P.tab.PW;
  const double dt = (A.stage == 0) ? 0.0 : *P.dt;

  // operator rows for this lane
  Rot4 rl, rr, rw;
  make_rot(P.tab.lL, a, b, rl);
  make_rot(P.tab.lR, a, b, rr);
  {
    double wh[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) wh[c] = P.tab.w[c] * 0.5;
    make_rot(wh, a, b, rw);
  }
  double dxr[NP], dyr[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    dxr[c] = A.Dt[a * NP + c];
    dyr[c] = A.Dt[b * NP + c];
  }
  const double dhLa = P.tab.dhL[a], dhRa = P.tab.dhR[a], dhLb = P.tab.dhL[b], dhRb = P.tab.dhR[b];
  const double iJx = 1.0 / P.Jx, iJy = 1.0 / P.Jy;

  // filter factors (stage 3)
  if (A.stage == 3) {
    for (int i = tid; i < M * NSP; i += BLK) {
      const double f = P.tab.filt[i];
      sLam[i] = (P.filter == FRSG_FILTER_EXP) ? exp(-P.alpha * dt * f) : f;
    }
  }

  // own coefficients
  double m[4][M];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int k = 0; k < M; ++k) m[s][k] = A.in[((long)s * M + k) * EN + (long)e * NSP + j];

  // halo role: (face hf of the tile, flux point fp, state hs); modal trace of the outside neighbour
  const int hf = tid >> 4, hfp = (tid >> 2) & 3, hs = tid & 3;
  double th[M];
  {
    const int side = hf >> 2, pos = hf & 3;
    int nix, niy;
    const double* l;
    bool along_x;
    if (side == 0) { nix = 4 * tx - 1; niy = 4 * ty + pos; l = P.tab.lR; along_x = true; }
    else if (side == 1) { nix = 4 * tx + 4; niy = 4 * ty + pos; l = P.tab.lL; along_x = true; }
    else if (side == 2) { nix = 4 * tx + pos; niy = 4 * ty - 1; l = P.tab.lR; along_x = false; }
    else { nix = 4 * tx + pos; niy = 4 * ty + 4; l = P.tab.lL; along_x = false; }
    bool valid = true;
    if (nix < 0) { if (P.bc[0] == FRSG_BC_PERIODIC) nix += P.nx; else valid = false; }
    if (nix >= P.nx) { if (P.bc[1] == FRSG_BC_PERIODIC) nix -= P.nx; else valid = false; }
    if (niy < 0) { if (P.bc[2] == FRSG_BC_PERIODIC) niy += P.ny; else valid = false; }
    if (niy >= P.ny) { if (P.bc[3] == FRSG_BC_PERIODIC) niy -= P.ny; else valid = false; }
    const int ne = valid ? niy * P.nx + nix : 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double acc = 0.0;
      if (valid) {
        const double* src = A.in + ((long)hs * M + k) * EN + (long)ne * NSP;
#pragma unroll
        for (int c = 0; c < NP; ++c) acc += l[c] * src[along_x ? (c + NP * hfp) : (hfp + NP * c)];
      }
      th[k] = acc;
    }
  }

  // face-point role of this lane: side = j >> 2 (x-lo, x-hi, y-lo, y-hi), flux point i = j & 3
  const int fside = j >> 2, fi = j & 3;
  int nbr_le = -1;  // neighbour inside the tile
  int nbr_halo = -1;
  bool boundary = false;
  if (fside == 0) {
    if (lx > 0) nbr_le = le - 1;
    else if (ix == 0 && P.bc[0] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = ly;
  } else if (fside == 1) {
    if (lx < 3) nbr_le = le + 1;
    else if (ix == P.nx - 1 && P.bc[1] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = 4 + ly;
  } else if (fside == 2) {
    if (ly > 0) nbr_le = le - 4;
    else if (iy == 0 && P.bc[2] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = 8 + lx;
  } else {
    if (ly < 3) nbr_le = le + 4;
    else if (iy == P.ny - 1 && P.bc[3] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = 12 + lx;
  }
  // interpolation weights: own side and neighbour side of this face
  const double* lown = (fside == 0 || fside == 2) ? P.tab.lL : P.tab.lR;
  const double* lnbr = (fside == 0 || fside == 2) ? P.tab.lR : P.tab.lL;
  double wown[4], wnbr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    wown[c] = lown[c];
    wnbr[c] = lnbr[c];
  }

  double acc[4][M];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int k = 0; k < M; ++k) acc[s][k] = 0.0;

  for (int q = 0; q < NQ; ++q) {
    const int par = q & 1;
    // (1) nodal state and fluxes at this lane's solution point; halo traces
    double U[4], F[4], G[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) t += m[s][k] * Phi[k * NQ + q];
      U[s] = t;
    }
    euler_fg(U, F, G, g);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      sU[par][le][j][s] = U[s];
      sF[par][le][j][s] = F[s];
      sG[par][le][j][s] = G[s];
    }
    {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) t += th[k] * Phi[k * NQ + q];
      sH[par][hf][hfp][hs] = t;
    }
    __syncthreads();

    // (2) interface flux at this lane's flux point
    {
      double own[4], nb[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < NP; ++c) t += wown[c] * sU[par][le][fside < 2 ? (c + NP * fi) : (fi + NP * c)][s];
        own[s] = t;
      }
      if (nbr_le >= 0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          double t = 0.0;
#pragma unroll
          for (int c = 0; c < NP; ++c)
            t += wnbr[c] * sU[par][nbr_le][fside < 2 ? (c + NP * fi) : (fi + NP * c)][s];
          nb[s] = t;
        }
      } else if (boundary) {
        ghost<kEuler2>(P, fside, own, nb);
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) nb[s] = sH[par][nbr_halo][fi][s];
      }
      double Fs[4];
      const bool lo = (fside == 0 || fside == 2);
      if (fside < 2)
        rusanov<kEuler2, 0>(lo ? nb : own, lo ? own : nb, Fs, 0.0, g);
      else
        rusanov<kEuler2, 1>(lo ? nb : own, lo ? own : nb, Fs, 0.0, g);
#pragma unroll
      for (int s = 0; s < 4; ++s) sFs[le][j][s] = Fs[s];
    }
    __syncthreads();

    // (3) nodal residual at this lane's solution point, projected onto the chaos
    {
      double R[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double ax = 0.0, ay = 0.0;
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          ax += dxr[c] * sF[par][le][c + NP * b][s];
          ay += dyr[c] * sG[par][le][a + NP * c][s];
        }
        ax += sFs[le][0 + b][s] * dhLa + sFs[le][4 + b][s] * dhRa;
        ay += sFs[le][8 + a][s] * dhLb + sFs[le][12 + a][s] * dhRb;
        R[s] = -ax * iJx - ay * iJy;
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double w = PW[k * NQ + q];
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s][k] += w * R[s];
      }
    }
  }

  // ----------------------------------------------------------------- epilogue
  const long base = (long)e * NSP + j;
  if (A.stage == 0) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < M; ++k) A.out[((long)s * M + k) * EN + base] = acc[s][k];
    return;
  }
  // stage combination (acc becomes the output)
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const long idx = ((long)s * M + k) * EN + base;
      const double uu = (A.cu != 0.0) ? A.u[idx] : 0.0;
      acc[s][k] = A.cu * uu + A.cw * (m[s][k] + dt * acc[s][k]);
    }

  if (A.stage == 3 && P.filter != FRSG_FILTER_NONE) {
    __syncthreads();  // sLam ready
    Rot4 rvi, rv;
    // x: row a of V^-1 acting on x; y: row b acting on y
    {
      double tx_[4], ty_[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        tx_[c] = P.tab.Vinv[a * NP + c];
        ty_[c] = P.tab.Vinv[b * NP + c];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        rvi.x[k] = tx_[(a + k) & 3];
        rvi.y[k] = ty_[(b - k) & 3];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        tx_[c] = P.tab.V[a * NP + c];
        ty_[c] = P.tab.V[b * NP + c];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        rv.x[k] = tx_[(a + k) & 3];
        rv.y[k] = ty_[(b - k) & 3];
      }
    }
    const int ff = sensor_filter_element<M>(P, acc, j, rvi, rv, sLam, true);
    if (j == 0 && A.flag_filt) A.flag_filt[e] = (unsigned char)ff;
  } else if (A.stage == 3 && j == 0 && A.flag_filt) {
    A.flag_filt[e] = 0;
  }

  if (P.limiter) {
    const int lf = limit_element<M, NQ>(P, acc, a, b, rw, rl, rr, A.cmax, true);
    if (j == 0 && A.flag_lim) A.flag_lim[e] = (unsigned char)lf;
  } else if (j == 0 && A.flag_lim) {
    A.flag_lim[e] = 0;
  }

#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int k = 0; k < M; ++k) A.out[((long)s * M + k) * EN + base] = acc[s][k];

  // CFL maximum of the new state for the next step
  if (A.stage == 3 && A.lam_next) {
    double rate = 0.0;
    for (int q = 0; q < NQ; ++q) {
      double U[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) t += acc[s][k] * Phi[k * NQ + q];
        U[s] = t;
      }
      double r = speed<kEuler2, 0>(U, 0.0, g) / P.dx + speed<kEuler2, 1>(U, 0.0, g) / P.dy;
      if (!(r == r)) r = __longlong_as_double(0x7ff0000000000000ll);
      rate = fmax(rate, r);
    }
    // wave then workgroup maximum
    rate = ymax4(xmax4(rate));
    rate = fmax(rate, __shfl_xor(rate, 16));
    rate = fmax(rate, __shfl_xor(rate, 32));
    if ((tid & 63) == 0) sRed[tid >> 6] = rate;
    __syncthreads();
    if (tid == 0) {
      double r = sRed[0];
      for (int w = 1; w < BLK / 64; ++w) r = fmax(r, sRed[w]);
      atomicMax(A.lam_next, (unsigned long long)__double_as_longlong(r));
    }
  }
}

// ---------------------------------------------------------------------------
// CFL maximum of a state (used when no previous step recorded it)
// ---------------------------------------------------------------------------
template <int M, int NQ>
__global__ void __launch_bounds__(BLK) k_cfl2d(KParams P, const double* __restrict__ u,
                                               unsigned long long* lam) {
  __shared__ double sRed[BLK / 64];
  const long t = blockIdx.x * (long)BLK + threadIdx.x;
  const long EN = (long)P.E * NSP;
  double rate = 0.0;
  if (t < EN) {
    double o[4][M];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < M; ++k) o[s][k] = u[((long)s * M + k) * EN + t];
    for (int q = 0; q < NQ; ++q) {
      double U[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) acc += o[s][k] * P.tab.Phi[k * NQ + q];
        U[s] = acc;
      }
      double r = speed<kEuler2, 0>(U, 0.0, P.gamma) / P.dx + speed<kEuler2, 1>(U, 0.0, P.gamma) / P.dy;
      if (!(r == r)) r = __longlong_as_double(0x7ff0000000000000ll);
      rate = fmax(rate, r);
    }
  }
  for (int o = 32; o > 0; o >>= 1) rate = fmax(rate, __shfl_xor(rate, o));
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = rate;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sRed[0];
    for (int w = 1; w < BLK / 64; ++w) r = fmax(r, sRed[w]);
    atomicMax(lam, (unsigned long long)__double_as_longlong(r));
  }
}

__global__ void k_dt_from(KParams P, const unsigned long long* lam, unsigned long long* lam_reset, double* dt_used) {
  const double l = __longlong_as_double((long long)*lam);
  const double dt = P.cfl / (P.np1 * l);
  if (!(dt > 0.0) || !isfinite(dt)) atomicOr(P.status, kStatusNonFinite);
  *P.dt = dt;
  if (dt_used) *dt_used = dt;
  if (lam_reset) *lam_reset = 0ull;
}

__global__ void k_set_dt(KParams P, double dt, double* dt_used, unsigned long long* lam_reset) {
  *P.dt = dt;
  if (dt_used) *dt_used = dt;
  if (lam_reset) *lam_reset = 0ull;
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

}  // namespace

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int M, int NQ>
static hipError_t launch_stage_t(const KParams& P, const FusedStage& S, hipStream_t s) {
  StageArgs A;
  A.in = S.in;
  A.u = S.u;
  A.out = S.out;
  A.cu = S.cu;
  A.cw = S.cw;
  A.stage = S.stage;
  A.flag_lim = S.flag_lim;
  A.flag_filt = S.flag_filt;
  A.lam_next = S.lam_next;
  A.Dt = S.Dt;
  A.cmax = S.cmax;
  const int ntiles = (P.nx / 4) * (P.ny / 4);
  hipLaunchKernelGGL((k_stage2d<M, NQ>), dim3(ntiles), dim3(BLK), 0, s, P, A);
  return hipGetLastError();
}

template <int M, int NQ>
static hipError_t launch_cfl_t(const KParams& P, const double* u, unsigned long long* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, lam);
  const long EN = (long)P.E * NSP;
  hipLaunchKernelGGL((k_cfl2d<M, NQ>), dim3((unsigned)((EN + BLK - 1) / BLK)), dim3(BLK), 0, s, P, u, lam);
  return hipGetLastError();
}

#define FRSG_FUSED_SIZES(X) X(15, 25) X(10, 16) X(6, 9) X(3, 4) X(5, 5)

bool fused2d_supported(const KParams& P) {
  if (P.eq != kEuler2 || P.np1 != 4 || P.nx % 4 != 0 || P.ny % 4 != 0) return false;
#define X(MM, QQ) if (P.M == MM && P.Nq == QQ) return true;
  FRSG_FUSED_SIZES(X)
#undef X
  return false;
}

hipError_t launch_fused_stage(const KParams& P, const FusedStage& S, hipStream_t s) {
#define X(MM, QQ) if (P.M == MM && P.Nq == QQ) return launch_stage_t<MM, QQ>(P, S, s);
  FRSG_FUSED_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_fused_cfl(const KParams& P, const double* u, unsigned long long* lam, hipStream_t s) {
#define X(MM, QQ) if (P.M == MM && P.Nq == QQ) return launch_cfl_t<MM, QQ>(P, u, lam, s);
  FRSG_FUSED_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_dt_from(const KParams& P, const unsigned long long* lam, unsigned long long* lam_reset,
                          double* dt_used, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_from, dim3(1), dim3(1), 0, s, P, lam, lam_reset, dt_used);
  return hipGetLastError();
}

hipError_t launch_set_dt(const KParams& P, double dt, double* dt_used, unsigned long long* lam_reset,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(1), 0, s, P, dt, dt_used, lam_reset);
  return hipGetLastError();
}

}  // namespace frsg
