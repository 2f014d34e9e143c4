// Fused FR-SG stage kernel for the 2D Euler equations on quadrilaterals with
// p = 3 (4 x 4 Legendre-Gauss solution points), any gPC size M and random
// node count NQ fixed at compile time.
//
// One kernel per SSP-RK3 stage does the whole right-hand side (Sec. 2.1, Sec.
// 3.2-3.5) and the stage epilogue, reading each input coefficient from HBM
// once and writing each output coefficient once:
//
//   * a workgroup owns a 4 x 2 tile of elements, 32 threads per element;
//     thread (e, h, j) holds the M gPC coefficients of conserved variables 2h
//     and 2h + 1 at solution point j of element e in registers, and
//     accumulates their projected residual there;
//   * random nodes go in pairs (q0, q1): each thread expands its own pair of
//     variables at both nodes (Eq. polynomial chaos), then the two rows of an
//     element trade halves so that rows h = 0 hold all four variables at q0
//     and rows h = 1 at q1; at that node each thread evaluates the fluxes F,
//     G (Eq. local direct flux), the solution trace at flux point j by
//     Lagrange interpolation along its line, the Lax-Friedrichs flux there
//     (Sec. 3.3) and the nodal residual
//       R = -(1/Jx) [Dt F + F*_L h_L' + F*_R h_R']_x - (1/Jy) [...]_y,
//     with Dt = D - h_L' l(-1)^T - h_R' l(+1)^T the derivative matrix that
//     already subtracts the interpolated discontinuous flux at the faces
//     (Sec. 3.4: the correction (F* - F^D) h' split into F* h' and -F^D h');
//     the residuals are traded back and Galerkin-projected on the fly (Eq.
//     discrete expectation value), so the residual of the stage is never
//     stored;
//   * traces of elements outside the tile come from their modal face traces,
//     interpolated once per stage and expanded at every node (the
//     interpolation and the chaos expansion are both linear, so the order does
//     not matter);
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
// FP32-mixed precision (R = float): the node loop (expansion, fluxes, traces,
// interface fluxes, residual, projection of the modes k >= 1) runs in FP32 on
// the coefficients and tables rounded to FP32; the mean mode k = 0 is projected
// in FP64, and the stage combination, detector, filter, limiter, face traces for
// the neighbours and the CFL maximum are FP64.  Inside a tile both sides of a
// face read the same FP32 trace; across tiles the neighbour's side comes from
// its FP64 modal trace, so the two traces agree to FP32 rounding there.
//
// Exchanges inside an element: the 16 threads of an (element, h) form one
// 16-lane DPP row, quad_perm rotations move along x (a) and row_ror:4k along y
// (b); the two rows of an element trade values with v_permlane16_swap.
// Exchanges between elements of the tile go through LDS.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"
#include "quad_device.hpp"

namespace frsg {
namespace {

using namespace quad;
constexpr int BLK = 256;    // threads per workgroup of the element-wise kernels

// ---------------------------------------------------------------------------
// arguments
// ---------------------------------------------------------------------------
struct StageArgs {
  double cu, cw;             // out = cu u + cw (in + dt R)
  int stage;                 // 0: right-hand side only; 1, 2: limited stage output; 3: end of step
  unsigned char* flag_lim;   // per element: limiter acted on the output (stages 1-3)
  unsigned char* flag_filt;  // per element: filter acted (stage 3)
  unsigned long long* lam_next;  // stage 3: CFL accumulator of the new state (may be null)
  const double* Dt;          // 4 x 4 modified derivative matrix
  const double* cmax;        // [M] max_q |Phi_k(z_q)|
  const double* tr_in;       // modal face traces of the input, or null: interpolate from the neighbours
  double* tr_out;            // modal face traces of the output (may be null)
  // Butcher-row form (tab) instead of cu u + cw (in + dt R): out = u + dt (sum_m ka[m] kk[m]
  // + ka_cur R) over the earlier stage right-hand sides with nonzero coefficients, in stage
  // order, R last (skipped when ka_cur is 0); R is also stored in k_out (may be null)
  int tab, nt;
  const double* kk[kRkMaxTerms];
  double ka[kRkMaxTerms];
  double ka_cur;
  double* k_out;
  int flag_or;               // limiter flags OR-ed into flag_lim (set only where it acts)
};

// Lane layout of a workgroup (one TX x TY tile of elements, 32 threads per element):
//   tid = 32 le + 16 h + j,  j = a + 4 b,  le = lx + TX ly;
// lane (le, h, j) owns conserved variables 2h and 2h+1 at solution point j of
// local element le.  The 16 lanes with equal (le, h) form one DPP row, the two
// rows of an element are partners, and the 32 lanes of an element sit in one
// wave.
constexpr int TX = 4, TY = 2;
constexpr int TE = TX * TY;          // elements per tile
constexpr int BLKS = 32 * TE;        // threads per stage workgroup
constexpr int NHF = 2 * (TX + TY);   // element faces on the tile boundary
// modal face traces of one tile: per boundary face slot (x-lo rows, x-hi rows,
// y-lo columns, y-hi columns), variable, face point and mode
template <int M>
constexpr int TRACE_PER_TILE = NHF * 4 * NP * M;
#ifndef FRSG_FP32_WAVES
#define FRSG_FP32_WAVES 2  // waves per SIMD the FP32 node loop is compiled for (3 spills)
#endif
static_assert(BLKS % 64 == 0, "an element's 32 lanes must share a wave");

// value held by the partner lane (same point, other pair of variables): the
// 16-lane rows of each 32-lane half swap places.  Every lane of the wave must
// be active.
__device__ __forceinline__ unsigned other_half_u32(unsigned v) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (threadIdx.x & 16) ? r[0] : r[1];
}
__device__ __forceinline__ float other_half(float v) {
  return __uint_as_float(other_half_u32(__float_as_uint(v)));
}
__device__ __forceinline__ double other_half(double v) {
  const unsigned long long x = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = other_half_u32((unsigned)x), hi = other_half_u32((unsigned)(x >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// all four conserved variables from this lane's pair and the partner's pair
template <typename T>
__device__ __forceinline__ void full4(int h, T v0, T v1, T* U) {
  const T o0 = other_half(v0), o1 = other_half(v1);
  U[0] = h ? o0 : v0;
  U[1] = h ? o1 : v1;
  U[2] = h ? v0 : o0;
  U[3] = h ? v1 : o1;
}

// Exchange between the two 16-lane rows of each 32-lane half (v_permlane16_swap
// of a and b): afterwards b in row 0 holds row 1's a and a in row 1 holds row
// 0's b, while a in row 0 and b in row 1 keep their values.  Every lane of the
// wave must be active.
__device__ __forceinline__ void swap_rows_u32(unsigned& a, unsigned& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}
__device__ __forceinline__ void swap_rows(float& a, float& b) {
  unsigned x = __float_as_uint(a), y = __float_as_uint(b);
  swap_rows_u32(x, y);
  a = __uint_as_float(x);
  b = __uint_as_float(y);
}
__device__ __forceinline__ void swap_rows(double& a, double& b) {
  const unsigned long long x = (unsigned long long)__double_as_longlong(a);
  const unsigned long long y = (unsigned long long)__double_as_longlong(b);
  unsigned xl = (unsigned)x, xh = (unsigned)(x >> 32), yl = (unsigned)y, yh = (unsigned)(y >> 32);
  swap_rows_u32(xl, yl);
  swap_rows_u32(xh, yh);
  a = __longlong_as_double((long long)(((unsigned long long)xh << 32) | xl));
  b = __longlong_as_double((long long)(((unsigned long long)yh << 32) | yl));
}

struct LaneOps {
  double rlx[4], rly[4], rrx[4], rry[4];  // rotated l(-1), l(+1) for x (row a) and y (row b)
};

// ---------------------------------------------------------------------------
// positivity limiter on one element (Sec. 4.3); o[i][k]: this lane's pair
// ---------------------------------------------------------------------------
template <int M, int NQ>
__device__ int limit_pair(const KParams& P, const double* __restrict__ PhiT, double (&o)[2][M], int h, int a, int b,
                          const LaneOps& L, const double* cmax) {
  const double g = P.gamma;
  double rwx[4], rwy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rwx[k] = 0.5 * P.tab.w[(a + k) & 3];
    rwy[k] = 0.5 * P.tab.w[(b - k) & 3];
  }
  // element x random mean: sum_j (w_a/2)(w_b/2) o(j, mode 0)
  double ub[4];
  full4(h, row_bcast0(ydot(rwy, xdot(rwx, o[0][0]))), row_bcast0(ydot(rwy, xdot(rwx, o[1][0]))), ub);
  const double pb = euler_p(ub, g);
  const bool realizable = ub[0] > 0.0 && pb > 0.0 && isfinite(ub[0]) && isfinite(ub[1]) && isfinite(ub[2]) &&
                          isfinite(ub[3]);
  if (!realizable && a == 0 && b == 0 && h == 0) atomicOr(P.status, kStatusNotRealizable);
  const double eps = fmin(1e-8, fmin(ub[0], pb));

  // rigorous bounds: value(z) = mean + sum_{k>=1} c_k Phi_k(z), |Phi_k(z_q)| <= cmax_k
  double mean[2], var[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    mean[i] = o[i][0];
    double v = 0.0;
#pragma unroll
    for (int k = 1; k < M; ++k) v += fabs(o[i][k]) * cmax[k];
    var[i] = v;
  }
  // decision at one location from all four variables' means and bounds
  auto safe = [&](const double* mn, const double* vr) {
    const double rlo = mn[0] - vr[0];
    const double elo = mn[3] - vr[3];
    const double mx = fabs(mn[1]) + vr[1];
    const double my = fabs(mn[2]) + vr[2];
    const double tol_r = 1e-10 * (fabs(mn[0]) + vr[0]);
    if (!(rlo > eps + tol_r)) return false;
    const double kin = 0.5 * (mx * mx + my * my) / rlo;
    const double plo = (g - 1.0) * (elo - kin);
    const double tol_p = 1e-10 * (g - 1.0) * (fabs(mn[3]) + vr[3] + kin);
    return plo > eps + tol_p;
  };
  double ax[4], ay[4], bx[4], by[4];  // |l(-1)|, |l(+1)| rotated
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ax[k] = fabs(L.rlx[k]);
    ay[k] = fabs(L.rly[k]);
    bx[k] = fabs(L.rrx[k]);
    by[k] = fabs(L.rry[k]);
  }
  // own pair's mean and bound at the solution point and at the four face
  // points of its row (x) and column (y)
  double lm[5][2], lv[5][2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    lm[0][i] = mean[i];
    lv[0][i] = var[i];
    lm[1][i] = xdot(L.rlx, mean[i]);
    lv[1][i] = xdot(ax, var[i]);
    lm[2][i] = xdot(L.rrx, mean[i]);
    lv[2][i] = xdot(bx, var[i]);
    lm[3][i] = ydot(L.rly, mean[i]);
    lv[3][i] = ydot(ay, var[i]);
    lm[4][i] = ydot(L.rry, mean[i]);
    lv[4][i] = ydot(by, var[i]);
  }
  // locations in pairs: row 0 tests location A, row 1 location B, each with
  // all four variables after one exchange (every lane takes part in each)
  auto test_pair = [&](int A, int B) {
    double mn[4] = {lm[A][0], lm[A][1], lm[B][0], lm[B][1]};
    double vr[4] = {lv[A][0], lv[A][1], lv[B][0], lv[B][1]};
    swap_rows(mn[0], mn[2]);
    swap_rows(mn[1], mn[3]);
    swap_rows(vr[0], vr[2]);
    swap_rows(vr[1], vr[3]);
    return safe(mn, vr);
  };
  const bool t01 = test_pair(0, 1);
  const bool t23 = test_pair(2, 3);
  const bool t40 = test_pair(4, 0);
  const bool ok = t01 && t23 && t40;
  // element-wide decision
  double okd = ok ? 1.0 : 0.0;
  okd = ymin4(xmin4(okd));
  okd = fmin(okd, other_half(okd));
  const bool need = realizable && okd < 0.5;
  if (__ballot(need) == 0) return 0;

  // node-by-node test (all lanes of the wave take part)
  double rmin = INFINITY, pmin = INFINITY;
  for (int q = 0; q < NQ; ++q) {
    double u2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) t += o[i][k] * PhiT[q * M + k];
      u2[i] = t;
    }
    double U[4], T[4];
    full4(h, u2[0], u2[1], U);
    rmin = fmin(rmin, U[0]);
    pmin = fmin(pmin, euler_p(U, g));
    full4(h, xdot(L.rlx, u2[0]), xdot(L.rlx, u2[1]), T);
    rmin = fmin(rmin, T[0]);
    pmin = fmin(pmin, euler_p(T, g));
    full4(h, xdot(L.rrx, u2[0]), xdot(L.rrx, u2[1]), T);
    rmin = fmin(rmin, T[0]);
    pmin = fmin(pmin, euler_p(T, g));
    full4(h, ydot(L.rly, u2[0]), ydot(L.rly, u2[1]), T);
    rmin = fmin(rmin, T[0]);
    pmin = fmin(pmin, euler_p(T, g));
    full4(h, ydot(L.rry, u2[0]), ydot(L.rry, u2[1]), T);
    rmin = fmin(rmin, T[0]);
    pmin = fmin(pmin, euler_p(T, g));
  }
  rmin = ymin4(xmin4(rmin));
  pmin = ymin4(xmin4(pmin));
  const bool on = need && (fmin(rmin, pmin) < eps);
  if (__ballot(on) == 0) return 0;
  const double beta1 = (rmin >= eps) ? 1.0 : (ub[0] - eps) / (ub[0] - rmin);
  double bmin = 1.0;
  for (int q = 0; q < NQ; ++q) {
    double u2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) t += o[i][k] * PhiT[q * M + k];
      u2[i] = t;
    }
    double T[4];
    auto check = [&](double v0, double v1) {
      full4(h, v0, v1, T);
      T[0] = beta1 * (T[0] - ub[0]) + ub[0];
      if (euler_p(T, g) < eps) bmin = fmin(bmin, pressure_root<kEuler2>(ub, T, eps, g));
    };
    check(u2[0], u2[1]);
    check(xdot(L.rlx, u2[0]), xdot(L.rlx, u2[1]));
    check(xdot(L.rrx, u2[0]), xdot(L.rrx, u2[1]));
    check(ydot(L.rly, u2[0]), ydot(L.rly, u2[1]));
    check(ydot(L.rry, u2[0]), ydot(L.rry, u2[1]));
  }
  double beta2 = ymin4(xmin4(bmin));
  beta2 = fmin(beta2, other_half(beta2));
  if (on) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double m0 = (k == 0) ? 1.0 : 0.0;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int s = 2 * h + i;
        double v = o[i][k];
        if (s == 0) v = beta1 * (v - ub[0] * m0) + ub[0] * m0;
        o[i][k] = beta2 * (v - ub[s] * m0) + ub[s] * m0;
      }
    }
  }
  return on ? 1 : 0;
}

// ---------------------------------------------------------------------------
// detector + modal filter on one element (Sec. 4.1, 4.2)
// ---------------------------------------------------------------------------
template <int M>
__device__ int sensor_filter_pair(const KParams& P, double (&o)[2][M], int h, int a, int b, int j,
                                  const double* lam) {
  double vix[4], viy[4], vx[4], vy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    vix[k] = P.tab.Vinv[a * NP + ((a + k) & 3)];
    viy[k] = P.tab.Vinv[b * NP + ((b - k) & 3)];
    vx[k] = P.tab.V[a * NP + ((a + k) & 3)];
    vy[k] = P.tab.V[b * NP + ((b - k) & 3)];
  }
  // energies of the first variable's spatial-chaos modes (meaningful on the h = 0 row)
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double t = ydot(viy, xdot(vix, o[0][k]));
    const double e2 = t * t;
    num += e2 * P.tab.shell[k * NSP + j];
    den += e2;
  }
  num = row_bcast0(ysum4(xsum4(num)));
  den = row_bcast0(ysum4(xsum4(den)));
  const double onum = other_half(num), oden = other_half(den);
  if (h) {
    num = onum;
    den = oden;
  }
  const bool flag = (P.sensor == FRSG_SENSOR_ALWAYS) || (den > 0.0 && num / den > P.sensor_thr);
  if (__ballot(flag) == 0) return 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double t = ydot(viy, xdot(vix, o[i][k])) * lam[k * NSP + j];
      const double back = ydot(vy, xdot(vx, t));
      if (flag) o[i][k] = back;
    }
  }
  return flag ? 1 : 0;
}

// ---------------------------------------------------------------------------
// the stage kernel; R is the type of the node loop (nodal values, fluxes,
// residuals, projection), the epilogue runs in FP64
// ---------------------------------------------------------------------------
template <int M, int NQ, typename R, int FLUX>
__global__ void __launch_bounds__(BLKS) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 2 : FRSG_FP32_WAVES)))
k_stage2d(KParams P, StageArgs A, const double* __restrict__ PhiTd,
                                                  const R* __restrict__ PhiT, const R* __restrict__ PWT,
                                                  const double* __restrict__ in, const double* __restrict__ uin,
                                                  double* out) {
  constexpr bool kFP64 = sizeof(R) == sizeof(double);
  // per element and row h (node q0 or q1 of the pair in hand): nodal values at
  // the solution points, traces at the flux points (x-lo row i, x-hi row i,
  // y-lo column i, y-hi column i; two pairs in flight) and interface fluxes
  // (traces of elements outside the tile at every node in sH); the epilogue
  // reuses the space to stage the new state for its face traces
  struct LoopLds {
    Half2<R> sU[TE][2][2][NSP];     // [element][row h][plane][point]
    Half2<R> sT[2][TE][2][2][NSP];  // [pair parity][element][row h][plane][flux point]
    Half2<R> sFs[TE][2][2][NSP];
    Quad4<R> sH[NQ][NHF][NP];
  };
  union StageLds {
    LoopLds loop;
    double sO[TE][4][NSP][M];
  };
  __shared__ StageLds lds;
  auto& sU = lds.loop.sU;
  auto& sT = lds.loop.sT;
  auto& sFs = lds.loop.sFs;
  auto& sH = lds.loop.sH;
  __shared__ double sLam[M * NSP];
  constexpr int NQP = (NQ + 1) & ~1;  // rows padded to whole 16-byte pairs
  __shared__ __attribute__((aligned(16))) double sPhiK[M][NQP];  // chaos basis, mode-major
  __shared__ double sRed[BLKS / 64];

  const int tid = threadIdx.x;
  const int le = tid >> 5, h = (tid >> 4) & 1, j = tid & 15;
  const int a = j & 3, b = j >> 2;
  const int lx = le % TX, ly = le / TX;
  const int ntx = P.nx / TX;
  // XCD-aware order: consecutive workgroups go to different XCDs, so give each
  // XCD a contiguous band of tiles (neighbouring halos then share its L2)
  const int nty = P.ny / TY, ntiles = ntx * nty;
  int tile = blockIdx.x;
  if (ntiles % 8 == 0) tile = (tile % 8) * (ntiles / 8) + tile / 8;
  // within that order, walk blocks of 8 x 8 tiles: the tiles resident on an XCD
  // at one time then form a compact block, most of whose halo faces are read by
  // tiles of the same block while the data is in L2
  int tx, ty;
  if (ntx % 8 == 0 && nty % 8 == 0) {
    const int blk = tile >> 6, w = tile & 63, nbx = ntx / 8;
    tx = (blk % nbx) * 8 + (w & 7);
    ty = (blk / nbx) * 8 + (w >> 3);
  } else {
    tx = tile % ntx;
    ty = tile / ntx;
  }
  const int ix = TX * tx + lx, iy = TY * ty + ly;
  const int e = iy * P.nx + ix;
  const long EN = (long)P.E * NSP;
  const R g = (R)P.gamma;
  const double dt = (A.stage == 0) ? 0.0 : *P.dt;

  if (A.stage == 3) {
    for (int i = tid; i < M * NSP; i += BLKS) {
      const double f = P.tab.filt[i];
      sLam[i] = (P.filter == FRSG_FILTER_EXP) ? exp(-P.alpha * dt * f) : f;
    }
  }

  // the basis table for the halo first (its loads are waited for first)
  constexpr int NPHI = (NQ * M + BLKS - 1) / BLKS;
  double phv[NPHI];
  {
    const auto rp = state_rsrc(PhiTd, (unsigned)(NQ * M * sizeof(double)));
#pragma unroll
    for (int r = 0; r < NPHI; ++r) phv[r] = bload(rp, (unsigned)((tid + r * BLKS) * sizeof(double)), 0u);
  }

  // own coefficients: variables 2h, 2h+1 (the state is below 4 GiB, checked by the host)
  const unsigned sbytes = (unsigned)(4 * M * EN * (long)sizeof(double));
  const unsigned voff = (unsigned)(((long)(2 * h) * M * EN + (long)e * NSP + j) * (long)sizeof(double));
  auto soff = [&](int i, int k) { return (unsigned)(((long)i * M + k) * EN * (long)sizeof(double)); };
  // the input in FP64 for the epilogue's combination, and in the loop's type (the same
  // registers in FP64; the FP32 loop keeps both, 255 registers without spills)
  R m[2][M];
  double md[2][M];
  {
    const auto rin = state_rsrc(in, sbytes);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) {
        md[i][k] = bload_stream(rin, voff, soff(i, k));
        m[i][k] = (R)md[i][k];
      }
  }

  // traces of the elements around the tile at every node: one thread per
  // (face hf, face point hfp, variable hs); faces: TY x-lo, TY x-hi, TX y-lo, TX y-hi
  const bool halo_thread = tid < NHF * NP * 4;
  double th[M];  // modal trace of this thread's neighbour variable at its face point
  {
    const int hf = (tid >> 4) % NHF, hfp = (tid >> 2) & 3, hs = tid & 3;
    int nix, niy;
    bool along_x, from_lo;  // from_lo: the face is the neighbour's lo face (trace at -1)
    if (hf < TY) { nix = TX * tx - 1; niy = TY * ty + hf; along_x = true; from_lo = false; }
    else if (hf < 2 * TY) { nix = TX * tx + TX; niy = TY * ty + hf - TY; along_x = true; from_lo = true; }
    else if (hf < 2 * TY + TX) { nix = TX * tx + hf - 2 * TY; niy = TY * ty - 1; along_x = false; from_lo = false; }
    else { nix = TX * tx + hf - 2 * TY - TX; niy = TY * ty + TY; along_x = false; from_lo = true; }
    bool valid = halo_thread;
    if (nix < 0) { if (P.bc[0] == FRSG_BC_PERIODIC) nix += P.nx; else valid = false; }
    if (nix >= P.nx) { if (P.bc[1] == FRSG_BC_PERIODIC) nix -= P.nx; else valid = false; }
    if (niy < 0) { if (P.bc[2] == FRSG_BC_PERIODIC) niy += P.ny; else valid = false; }
    if (niy >= P.ny) { if (P.bc[3] == FRSG_BC_PERIODIC) niy -= P.ny; else valid = false; }
    // all loads first, without branches, so that they are in flight together; a
    // face without a neighbour (domain boundary) reads tile or element 0
    // instead, and its trace is never used: the lanes on that face take the
    // ghost state
    if (A.tr_in) {  // uniform: the traces were written by the launch that wrote the input
      // the neighbour tile's face slot that faces this one (x-lo halo <- x-hi slot, ...)
      const int slot = hf < TY ? TY + hf
                     : hf < 2 * TY ? hf - TY
                     : hf < 2 * TY + TX ? hf + TX
                     : hf - TX;
      const int nt = valid ? (niy / TY) * ntx + nix / TX : 0;
      const auto rtr = state_rsrc(A.tr_in, (unsigned)((long)ntiles * TRACE_PER_TILE<M> * (long)sizeof(double)));
      const unsigned to = (unsigned)(((long)nt * TRACE_PER_TILE<M> + ((slot * 4 + hs) * NP + hfp) * M) *
                                     (long)sizeof(double));
      if (halo_thread) {  // uniform per wave
#pragma unroll
        for (int k = 0; k < M; ++k) th[k] = bload(rtr, to, (unsigned)(k * sizeof(double)));
      }
    } else {
      const int ne = valid ? niy * P.nx + nix : 0;
      double lw[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) lw[c] = from_lo ? P.tab.lL[c] : P.tab.lR[c];
      const auto rh = state_rsrc(in, sbytes);
      unsigned ho[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c)
        ho[c] = (unsigned)((((long)hs * M) * EN + (long)ne * NSP + (along_x ? c + NP * hfp : hfp + NP * c)) *
                           (long)sizeof(double));
      if (halo_thread) {  // uniform per wave
        double hv[M][NP];
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
          for (int c = 0; c < NP; ++c) hv[k][c] = bload(rh, ho[c], soff(0, k));
#pragma unroll
        for (int k = 0; k < M; ++k)
          th[k] = lw[0] * hv[k][0] + lw[1] * hv[k][1] + lw[2] * hv[k][2] + lw[3] * hv[k][3];
      }
    }
  }
  // chaos basis at the nodes, mode-major, for the expansion of the halo traces
#pragma unroll
  for (int r = 0; r < NPHI; ++r) {
    const int i = tid + r * BLKS;  // node-major index q * M + k
    if (i < NQ * M) sPhiK[i % M][i / M] = phv[r];
  }
  __syncthreads();
  if (halo_thread) {
    // all nodes at once, mode by mode: independent accumulators, one pass over the table
    const int hf = tid >> 4, hfp = (tid >> 2) & 3, hs = tid & 3;
    double tq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) tq[q] = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
      for (int q = 0; q < NQ; ++q) tq[q] += th[k] * sPhiK[k][q];
#pragma unroll
    for (int q = 0; q < NQ; ++q) sH[q][hf][hfp].v[hs] = (R)tq[q];
  }

  // per-lane rows of the modified derivative matrix, rotated for xdot / ydot
  R dx[4], dy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    dx[k] = (R)A.Dt[a * NP + ((a + k) & 3)];
    dy[k] = (R)A.Dt[b * NP + ((b - k) & 3)];
  }
  const R dhLa = (R)P.tab.dhL[a], dhRa = (R)P.tab.dhR[a], dhLb = (R)P.tab.dhL[b], dhRb = (R)P.tab.dhR[b];
  const R iJx = (R)(1.0 / P.Jx), iJy = (R)(1.0 / P.Jy);

  // face-point role: flux point j of this element, side = j >> 2 (x-lo, x-hi, y-lo, y-hi), i = j & 3
  const int fside = j >> 2, fi = j & 3;
  int nbr_le = -1, nbr_halo = 0;
  bool boundary = false;
  if (fside == 0) {
    if (lx > 0) nbr_le = le - 1;
    else if (ix == 0 && P.bc[0] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = ly;
  } else if (fside == 1) {
    if (lx < TX - 1) nbr_le = le + 1;
    else if (ix == P.nx - 1 && P.bc[1] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = TY + ly;
  } else if (fside == 2) {
    if (ly > 0) nbr_le = le - TX;
    else if (iy == 0 && P.bc[2] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = 2 * TY + lx;
  } else {
    if (ly < TY - 1) nbr_le = le + TX;
    else if (iy == P.ny - 1 && P.bc[3] != FRSG_BC_PERIODIC) boundary = true;
    else nbr_halo = 2 * TY + TX + lx;
  }
  // boundary rule of this lane's face (Sec. 2.1 boundary operator, ghost state per node)
  const int gkind = P.bc[fside];
  R gstate[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) gstate[s] = (R)P.bc_state[fside][s];
  const int gnormal = fside < 2 ? 1 : 2;
  // the neighbour's flux point facing ours: x-lo <-> x-hi, y-lo <-> y-hi
  const int mirror = (fside ^ 1) * 4 + fi;
  const bool lo_side = (fside == 0 || fside == 2);
  const bool wave_at_boundary = __ballot(boundary) != 0;

  // the line of solution points through flux point j and its Lagrange weights
  // (l(-1) on a lo side, l(+1) on a hi side)
  int line[4];
  R wl[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    line[c] = (fside < 2) ? c + NP * fi : fi + NP * c;
    wl[c] = (R)(lo_side ? P.tab.lL[c] : P.tab.lR[c]);
  }

  R acc[2][M];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < M; ++k) acc[i][k] = R(0);
  // the mean mode k = 0 of the FP32 loop is projected in FP64 (weights w_q = PW[0][q])
  double acc0[2] = {0.0, 0.0};

  // own pair at (j, q): gPC expansion at the node
  auto expand = [&](int q, R* u2) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      R t = R(0);
#pragma unroll
      for (int k = 0; k < M; ++k) t += m[i][k] * PhiT[q * M + k];
      u2[i] = t;
    }
  };
  // Random nodes go in pairs (q0, q1 = q0 + 1).  Rows h = 0 work on node q0 and
  // rows h = 1 on node q1 with all four variables of their point (fluxes,
  // trace, interface flux, residual), so each of these is evaluated once per
  // point and node; the expansion and the projection stay with the lane's own
  // pair of variables at both nodes.  With an odd node count the last pair
  // repeats its node and counts it once.
  constexpr int NIT = (NQ + 1) / 2;
  R ua[2], ub[2];  // own pair at q0 and at q1; the next pair's are expanded one step ahead
  expand(0, ua);
  expand(NQ > 1 ? 1 : 0, ub);

#pragma unroll 1
  for (int t = 0; t < NIT; ++t) {
    const int q0 = 2 * t;
    const int q1 = (q0 + 1 < NQ) ? q0 + 1 : q0;
    const int qh = h ? q1 : q0;
    const int par = t & 1;
    // (1) all four variables at (j, qh): row 0 takes the partner's pair at q0,
    // row 1 the partner's pair at q1
    R U[4] = {ua[0], ua[1], ub[0], ub[1]};
    swap_rows(U[0], U[2]);
    swap_rows(U[1], U[3]);
    sU[le][h][0][j] = Half2<R>{U[0], U[1]};
    sU[le][h][1][j] = Half2<R>{U[2], U[3]};
    R F[4], G[4];
    {
      const R ir = recip(U[0]);
      const R p = (g - R(1)) * (U[3] - R(0.5) * (U[1] * U[1] + U[2] * U[2]) * ir);
      const R vx = U[1] * ir, vy = U[2] * ir;
      F[0] = U[1];
      F[1] = U[1] * vx + p;
      F[2] = U[2] * vx;
      F[3] = (U[3] + p) * vx;
      G[0] = U[2];
      G[1] = U[1] * vy;
      G[2] = U[2] * vy + p;
      G[3] = (U[3] + p) * vy;
    }
    // the nodal values of an element are written and read by the same wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // (2) solution trace at flux point j, by Lagrange interpolation along its line
    {
      R T[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const Half2<R> x0 = sU[le][h][0][line[c]], x1 = sU[le][h][1][line[c]];
        T[0] += wl[c] * x0.x;
        T[1] += wl[c] * x0.y;
        T[2] += wl[c] * x1.x;
        T[3] += wl[c] * x1.y;
      }
      sT[par][le][h][0][j] = Half2<R>{T[0], T[1]};
      sT[par][le][h][1][j] = Half2<R>{T[2], T[3]};
    }
    __syncthreads();

    // (3) Lax-Friedrichs flux at flux point j and node qh
    {
      const Half2<R>* src0 = (nbr_le >= 0) ? &sT[par][nbr_le][h][0][mirror]
                                           : reinterpret_cast<const Half2<R>*>(&sH[qh][nbr_halo][fi]);
      const Half2<R>* src1 = (nbr_le >= 0) ? &sT[par][nbr_le][h][1][mirror] : src0 + 1;
      const Half2<R> ow0 = sT[par][le][h][0][j], ow1 = sT[par][le][h][1][j], nq0 = *src0, nq1 = *src1;
      // next pair, independent of the reads above
      if (t + 1 < NIT) {
        const int n0 = q0 + 2, n1 = (n0 + 1 < NQ) ? n0 + 1 : n0;
        expand(n0, ua);
        expand(n1, ub);
      }
      R own[4] = {ow0.x, ow0.y, ow1.x, ow1.y};
      R nb[4] = {nq0.x, nq0.y, nq1.x, nq1.y};
      if (wave_at_boundary) {  // uniform: only waves with a domain-boundary face pay for the ghosts
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          R gh = (gkind == FRSG_BC_DIRICHLET) ? gstate[s] : own[s];
          if (gkind == FRSG_BC_REFLECT && s == gnormal) gh = -gh;
          nb[s] = boundary ? gh : nb[s];
        }
      }
      R Fs[4];
      if constexpr (FLUX == FRSG_FLUX_HLL)
        hll_e2(own, nb, lo_side, Fs, g, fside >> 1);
      else
        rusanov_e2(own, nb, lo_side, Fs, g, fside >> 1);
      sFs[le][h][0][j] = Half2<R>{Fs[0], Fs[1]};
      sFs[le][h][1][j] = Half2<R>{Fs[2], Fs[3]};
    }
    // the interface fluxes of an element are written and read by the same wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // (4) nodal residual at (j, qh), all four variables; then each lane takes
    // its own pair at both nodes (variable 2h + i: r[i] at q0, r[2 + i] at q1)
    // and projects it onto the chaos
    {
      const Half2<R> fxl0 = sFs[le][h][0][0 + b], fxr0 = sFs[le][h][0][4 + b];
      const Half2<R> fyl0 = sFs[le][h][0][8 + a], fyr0 = sFs[le][h][0][12 + a];
      const Half2<R> fxl1 = sFs[le][h][1][0 + b], fxr1 = sFs[le][h][1][4 + b];
      const Half2<R> fyl1 = sFs[le][h][1][8 + a], fyr1 = sFs[le][h][1][12 + a];
      const R fxl[4] = {fxl0.x, fxl0.y, fxl1.x, fxl1.y}, fxr[4] = {fxr0.x, fxr0.y, fxr1.x, fxr1.y};
      const R fyl[4] = {fyl0.x, fyl0.y, fyl1.x, fyl1.y}, fyr[4] = {fyr0.x, fyr0.y, fyr1.x, fyr1.y};
      R r[4];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        r[s] = -(xdot(dx, F[s]) + fxl[s] * dhLa + fxr[s] * dhRa) * iJx -
               (ydot(dy, G[s]) + fyl[s] * dhLb + fyr[s] * dhRb) * iJy;
      swap_rows(r[0], r[2]);
      swap_rows(r[1], r[3]);
      constexpr int K0 = kFP64 ? 0 : 1;
      if constexpr (!kFP64) {
        const double w0 = P.tab.PW[q0];
        acc0[0] += w0 * (double)r[0];
        acc0[1] += w0 * (double)r[1];
      }
#pragma unroll
      for (int k = K0; k < M; ++k) {
        acc[0][k] += PWT[q0 * M + k] * r[0];
        acc[1][k] += PWT[q0 * M + k] * r[1];
      }
      if (q1 != q0) {
        if constexpr (!kFP64) {
          const double w1 = P.tab.PW[q1];
          acc0[0] += w1 * (double)r[2];
          acc0[1] += w1 * (double)r[3];
        }
#pragma unroll
        for (int k = K0; k < M; ++k) {
          acc[0][k] += PWT[q1 * M + k] * r[2];
          acc[1][k] += PWT[q1 * M + k] * r[3];
        }
      }
    }
  }

  // ----------------------------------------------------------------- epilogue
  // projected residual of mode k of variable 2h + i, in FP64
  auto res = [&](int i, int k) { return (!kFP64 && k == 0) ? acc0[i] : (double)acc[i][k]; };
  const auto rout = state_rsrc(out, sbytes);
  if (A.stage == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) bstore(res(i, k), rout, voff, soff(i, k));
    return;
  }
  double o[2][M];
  if (A.tab) {
    // the earlier stages' terms first, in stage order, then this stage's
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) o[i][k] = 0.0;
    for (int t = 0; t < A.nt; ++t) {
      const auto rk = state_rsrc(A.kk[t], sbytes);
      const double at = A.ka[t];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < M; ++k) o[i][k] = o[i][k] + at * bload_stream(rk, voff, soff(i, k));
    }
    const auto ru = state_rsrc(uin, sbytes);
    const auto rko = state_rsrc(A.k_out, A.k_out ? sbytes : 0u);  // no k_out: an empty range drops the stores
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double r = res(i, k);
        bstore(r, rko, voff, soff(i, k));
        const double t = (A.ka_cur != 0.0) ? o[i][k] + A.ka_cur * r : o[i][k];
        o[i][k] = bload_stream(ru, voff, soff(i, k)) + dt * t;
      }
  } else {
    const auto ru = state_rsrc(uin, A.cu != 0.0 ? sbytes : 0u);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double uu = bload_stream(ru, voff, soff(i, k));  // 0 from an empty range when cu = 0
        o[i][k] = A.cu * uu + A.cw * (md[i][k] + dt * res(i, k));
      }
  }

  if (A.stage == 3) {
    int ff = 0;
    if (P.filter != FRSG_FILTER_NONE) ff = sensor_filter_pair<M>(P, o, h, a, b, j, sLam);
    if (tid % 32 == 0 && A.flag_filt) A.flag_filt[e] = (unsigned char)ff;
  }
  if (P.limiter) {
    LaneOps L;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      L.rlx[k] = P.tab.lL[(a + k) & 3];
      L.rrx[k] = P.tab.lR[(a + k) & 3];
      L.rly[k] = P.tab.lL[(b - k) & 3];
      L.rry[k] = P.tab.lR[(b - k) & 3];
    }
    const int lf = limit_pair<M, NQ>(P, PhiTd, o, h, a, b, L, A.cmax);
    if (tid % 32 == 0 && A.flag_lim && (lf || !A.flag_or)) A.flag_lim[e] = (unsigned char)lf;
  } else if (tid % 32 == 0 && A.flag_lim && !A.flag_or) {
    A.flag_lim[e] = 0;
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < M; ++k) bstore(o[i][k], rout, voff, soff(i, k));

  // modal face traces of the new state on the tile's boundary faces, for the
  // next launch's neighbours: the same interpolation, in the same order, as
  // their own prologue would take from the stored state
  if (A.tr_out) {  // uniform
    __syncthreads();  // the node loop's LDS is free
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) lds.sO[le][2 * h + i][j][k] = o[i][k];
    __syncthreads();
    const int tile_id = ty * ntx + tx;
    const auto rtr = state_rsrc(A.tr_out, (unsigned)((long)ntiles * TRACE_PER_TILE<M> * (long)sizeof(double)));
    const unsigned tbase = (unsigned)((long)tile_id * TRACE_PER_TILE<M> * (long)sizeof(double));
    constexpr int NR = (TRACE_PER_TILE<M> + BLKS - 1) / BLKS;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int oi = tid + r * BLKS;  // ((slot * 4 + s) * NP + point) * M + mode
      if (oi < TRACE_PER_TILE<M>) {
        const int k = oi % M, fp = (oi / M) % NP, sv = (oi / (M * NP)) % 4, slot = oi / (M * NP * 4);
        int ex, ey;
        bool ax, lo;
        if (slot < TY) { ex = 0; ey = slot; ax = true; lo = true; }
        else if (slot < 2 * TY) { ex = TX - 1; ey = slot - TY; ax = true; lo = false; }
        else if (slot < 2 * TY + TX) { ex = slot - 2 * TY; ey = 0; ax = false; lo = true; }
        else { ex = slot - 2 * TY - TX; ey = TY - 1; ax = false; lo = false; }
        const int el = ex + TX * ey;
        double v[NP], w[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          v[c] = lds.sO[el][sv][ax ? c + NP * fp : fp + NP * c][k];
          w[c] = lo ? P.tab.lL[c] : P.tab.lR[c];
        }
        bstore(w[0] * v[0] + w[1] * v[1] + w[2] * v[2] + w[3] * v[3], rtr, tbase + (unsigned)(oi * sizeof(double)), 0u);
      }
    }
  }

  // CFL maximum of the new state for the next step
  if (A.stage == 3 && A.lam_next) {
    const double gd = P.gamma, idx = 1.0 / P.dx, idy = 1.0 / P.dy;
    // (|vx| + c) / dx + (|vy| + c) / dy at one node; NaN counts as infinity
    auto node_rate = [&](const double* U) {
      const double ir = recip(U[0]);
      const double vx = U[1] * ir, vy = U[2] * ir;
      const double p = (gd - 1.0) * (U[3] - 0.5 * (U[1] * vx + U[2] * vy));
      const double c = sqrt(gd * p * ir);
      const double r = (fabs(vx) + c) * idx + (fabs(vy) + c) * idy;
      return (r == r) ? r : __longlong_as_double(0x7ff0000000000000ll);
    };
    auto nodal = [&](int q, double* u2) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) t += o[i][k] * PhiTd[q * M + k];
        u2[i] = t;
      }
    };
    double rate = 0.0;
    // nodes in pairs: lane h = 0 completes node q, lane h = 1 node q + 1, each
    // taking the partner's pair of variables at its node
    int q = 0;
    // two pairs per iteration, so that their table loads and sums overlap (four
    // pairs per iteration measured slower)
#pragma unroll 2
    for (; q + 1 < NQ; q += 2) {
      double a2[2], b2[2];
      nodal(q, a2);
      nodal(q + 1, b2);
      double U[4] = {a2[0], a2[1], b2[0], b2[1]};
      swap_rows(U[0], U[2]);
      swap_rows(U[1], U[3]);
      rate = fmax(rate, node_rate(U));
    }
    if (q < NQ) {
      double a2[2], U[4];
      nodal(q, a2);
      full4(h, a2[0], a2[1], U);
      rate = fmax(rate, node_rate(U));
    }
    for (int w = 32; w > 0; w >>= 1) rate = fmax(rate, __shfl_xor(rate, w));
    if ((tid & 63) == 0) sRed[tid >> 6] = rate;
    __syncthreads();
    if (tid == 0) {
      double r = sRed[0];
      for (int w = 1; w < BLKS / 64; ++w) r = fmax(r, sRed[w]);
      atomicMax(A.lam_next, (unsigned long long)__double_as_longlong(r));
    }
  }
}

// ---------------------------------------------------------------------------
// Element-wise passes on a state with the stage kernel's lane layout: the
// sensor-gated filter (Sec. 4.1, 4.2) and/or the positivity limiter (Sec. 4.3),
// in that order, in place.  Used where they are not fused into a stage (the
// tableau integrators, fr_sg_limit).
// ---------------------------------------------------------------------------
template <int M, int NQ>
__global__ void __launch_bounds__(BLKS) __attribute__((amdgpu_waves_per_eu(2)))
k_post2d(KParams P, const double* __restrict__ PhiTd, const double* __restrict__ cmax, double* u, int do_filter,
         int do_limit, unsigned char* flag_filt, unsigned char* flag_lim) {
  __shared__ double sLam[M * NSP];
  const int tid = threadIdx.x;
  const int le = tid >> 5, h = (tid >> 4) & 1, j = tid & 15;
  const int a = j & 3, b = j >> 2;
  const int lx = le % TX, ly = le / TX;
  const int ntx = P.nx / TX;
  const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
  const int e = (TY * ty + ly) * P.nx + TX * tx + lx;
  const long EN = (long)P.E * NSP;
  if (do_filter) {
    const double dt = *P.dt;
    for (int i = tid; i < M * NSP; i += BLKS) {
      const double f = P.tab.filt[i];
      sLam[i] = (P.filter == FRSG_FILTER_EXP) ? exp(-P.alpha * dt * f) : f;
    }
    __syncthreads();
  }
  const unsigned sbytes = (unsigned)(4 * M * EN * (long)sizeof(double));
  const unsigned voff = (unsigned)(((long)(2 * h) * M * EN + (long)e * NSP + j) * (long)sizeof(double));
  auto soff = [&](int i, int k) { return (unsigned)(((long)i * M + k) * EN * (long)sizeof(double)); };
  const auto ru = state_rsrc(u, sbytes);
  double o[2][M];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < M; ++k) o[i][k] = bload_stream(ru, voff, soff(i, k));
  if (do_filter) {
    const int ff = sensor_filter_pair<M>(P, o, h, a, b, j, sLam);
    if (tid % 32 == 0 && flag_filt) flag_filt[e] = (unsigned char)ff;
  }
  if (do_limit) {
    LaneOps L;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      L.rlx[k] = P.tab.lL[(a + k) & 3];
      L.rrx[k] = P.tab.lR[(a + k) & 3];
      L.rly[k] = P.tab.lL[(b - k) & 3];
      L.rry[k] = P.tab.lR[(b - k) & 3];
    }
    const int lf = limit_pair<M, NQ>(P, PhiTd, o, h, a, b, L, cmax);
    if (tid % 32 == 0 && flag_lim) flag_lim[e] = (unsigned char)lf;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < M; ++k) bstore(o[i][k], ru, voff, soff(i, k));
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
  const double dt = (P.dim == 1 ? P.cfl * P.dx : P.cfl) / (P.np1 * l);  // 1D: CFL dx / ((p+1) lambda)
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
  A.cu = S.cu;
  A.cw = S.cw;
  A.stage = S.stage;
  A.flag_lim = S.flag_lim;
  A.flag_filt = S.flag_filt;
  A.lam_next = S.lam_next;
  A.Dt = S.Dt;
  A.cmax = S.cmax;
  A.tr_in = S.tr_in;
  A.tr_out = S.tr_out;
  A.tab = S.tab;
  A.nt = S.tab ? S.terms.n : 0;
  for (int t = 0; t < kRkMaxTerms; ++t) {
    A.kk[t] = t < A.nt ? S.terms.K[t] : nullptr;
    A.ka[t] = t < A.nt ? S.terms.a[t] : 0.0;
  }
  A.ka_cur = S.ka_cur;
  A.k_out = S.k_out;
  A.flag_or = S.tab;
  const int ntiles = (P.nx / TX) * (P.ny / TY);
  if (S.fp32) {
    if (P.flux == FRSG_FLUX_HLL)
      hipLaunchKernelGGL((k_stage2d<M, NQ, float, FRSG_FLUX_HLL>), dim3(ntiles), dim3(BLKS), 0, s, P, A, S.PhiT,
                         S.PhiT32, S.PWT32, S.in, S.u, S.out);
    else
      hipLaunchKernelGGL((k_stage2d<M, NQ, float, FRSG_FLUX_RUSANOV>), dim3(ntiles), dim3(BLKS), 0, s, P, A, S.PhiT,
                         S.PhiT32, S.PWT32, S.in, S.u, S.out);
  } else {
    if (P.flux == FRSG_FLUX_HLL)
      hipLaunchKernelGGL((k_stage2d<M, NQ, double, FRSG_FLUX_HLL>), dim3(ntiles), dim3(BLKS), 0, s, P, A, S.PhiT,
                         S.PhiT, S.PWT, S.in, S.u, S.out);
    else
      hipLaunchKernelGGL((k_stage2d<M, NQ, double, FRSG_FLUX_RUSANOV>), dim3(ntiles), dim3(BLKS), 0, s, P, A,
                         S.PhiT, S.PhiT, S.PWT, S.in, S.u, S.out);
  }
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

size_t fused2d_trace_count(int nx, int ny, int M) {
  return (size_t)(nx / TX) * (size_t)(ny / TY) * (size_t)(NHF * 4 * NP) * (size_t)M;
}

bool fused2d_supported(const KParams& P) {
  if (P.eq != kEuler2 || P.np1 != 4 || P.nx % TX != 0 || P.ny % TY != 0) return false;
  // raw buffer offsets are 32-bit: the state must stay below 4 GiB
  if ((double)4 * P.M * P.E * NSP * sizeof(double) >= 4294967296.0) return false;
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

template <int M, int NQ>
static hipError_t launch_post_t(const KParams& P, const double* PhiTd, const double* cmax, double* u, int do_filter,
                                int do_limit, unsigned char* flag_filt, unsigned char* flag_lim, hipStream_t s) {
  const int ntiles = (P.nx / TX) * (P.ny / TY);
  hipLaunchKernelGGL((k_post2d<M, NQ>), dim3(ntiles), dim3(BLKS), 0, s, P, PhiTd, cmax, u, do_filter, do_limit,
                     flag_filt, flag_lim);
  return hipGetLastError();
}

hipError_t launch_fused_post(const KParams& P, const double* PhiTd, const double* cmax, double* u, int do_filter,
                             int do_limit, unsigned char* flag_filt, unsigned char* flag_lim, hipStream_t s) {
#define X(MM, QQ) \
  if (P.M == MM && P.Nq == QQ) return launch_post_t<MM, QQ>(P, PhiTd, cmax, u, do_filter, do_limit, flag_filt, flag_lim, s);
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
