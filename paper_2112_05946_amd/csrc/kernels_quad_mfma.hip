// Matrix-core stage kernel of the FR-SG scheme for the 2D Euler equations on
// quadrilaterals with p = 3 (4 x 4 Legendre-Gauss solution points), for the
// gPC sizes M <= 16 and random node counts N_q <= 32 of the fused set.
//
// One launch per SSP-RK3 stage does the whole right-hand side (Sec. 2.1,
// Sec. 3.2-3.5) and the stage epilogue (Sec. 4.1-4.3, CFL maximum).  The
// random-space transforms are dense contractions and run on the matrix cores:
//
//   * nodal values U(z_q) = sum_k u_k Phi_k(z_q) (Eq. polynomial chaos) at the
//     solution points, the element's own solution traces at its 16 flux
//     points and the neighbours' traces there are each a 16 x 16 x 16 product
//     (nodes x points x modes) per conserved variable and block of 16 nodes;
//   * the Galerkin projection of the nodal residual (Eq. discrete expectation
//     value) is the transposed product, accumulated over the node blocks.
//
// Traces are expanded from modal face traces (the four-term Lagrange
// interpolation of the coefficients, Sec. 3.2), the same values on both sides
// of every face, so the interactive flux is single-valued and the scheme stays
// conservative in every precision.
//
// Precision (template MODE):
//   kQF64  FP64 matrix instructions (16 x 16 x 4), everything in FP64;
//   kQBF16 each operand of the transforms split into a high and a low
//          bfloat16 part, products hi*hi + hi*lo + lo*hi accumulated in FP32
//          (16 x 16 x 16 bfloat16 instructions); fluxes and residual in FP32;
//          the mean mode's projection, the stage combination, detector,
//          filter, limiter and CFL maximum in FP64.
//
// Layout: a workgroup owns a 2 x 2 tile of elements, one element per wave.
// Lane l = 16 g + j of a wave holds solution point j = a + 4 b (and flux point
// j) of its element; its lane group g selects the random nodes 16 nb + g + 4 r
// in register r of node block nb, and the gPC modes of its coefficient
// registers t (4 t + g for kQF64, 4 g + t for kQBF16).  All four conserved
// variables of a point sit in one lane, so fluxes, traces and interactive
// fluxes need no exchange; the derivative along x and y moves values inside the
// 16-lane row with DPP, as in the other quadrilateral kernels.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"
#include "mfma_bf16.hpp"
#include "quad_device.hpp"

namespace frsg {
namespace {

using namespace quad;

typedef double v4d __attribute__((ext_vector_type(4)));

enum { kQF64 = 0, kQBF16 = 1 };

constexpr int QTX = 2, QTY = 2;       // elements per tile along x and y
constexpr int QTE = QTX * QTY;        // elements (waves) per workgroup
constexpr int QBLK = 64 * QTE;        // threads per workgroup
constexpr int QNHF = 2 * (QTX + QTY); // element faces on the tile boundary
static_assert(QTX == 2 && QTY == 2, "every element of the tile has one boundary face per direction");

// gPC mode held in coefficient register t of lane group g
template <int MODE>
__device__ __forceinline__ int qmode(int t, int g) {
  return MODE == kQF64 ? 4 * t + g : 4 * g + t;
}
// registers of node block nb that hold at least one node (node 16 nb + g + 4 r)
__host__ __device__ constexpr int qslots(int NQ, int nb) {
  return (NQ - 16 * nb >= 16) ? 4 : (NQ - 16 * nb + 3) / 4;
}

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4s as_v4s(double d) { return __builtin_bit_cast(v4s, d); }

// The four-term Lagrange interpolation of a line of coefficients to a face, in
// one fixed order: every producer and consumer of face traces uses it, so the
// traces of a face agree bit for bit wherever they are formed.
__device__ __forceinline__ double trace4(const double* w, double v0, double v1, double v2, double v3) {
  return fma(w[3], v3, fma(w[2], v2, fma(w[1], v1, w[0] * v0)));
}

// modal face traces of one tile: [face slot][variable][mode][face point]
template <int M>
constexpr int QTRACE_PER_TILE = QNHF * 4 * M * NP;

struct QArgs {
  double cu, cw;                 // out = cu u + cw (in + dt R)
  int stage;                     // 0: right-hand side only; 1, 2: limited stage output; 3: end of step
  unsigned char* flag_lim;
  unsigned char* flag_filt;
  unsigned long long* lam_next;  // stage 3: CFL accumulator of the new state (may be null)
  const double* in;              // stage input
  const double* u;               // u^n (read when cu != 0)
  double* out;
  const double* tr_in;           // modal face traces of `in` on tile boundaries
  double* tr_out;                // those of `out` (may be null)
  const double* frag;            // operand tables (QuadFragLayout)
  const double* cmax;            // [M] max_q |Phi_k(z_q)|
  const double* Dt;              // 4 x 4 derivative matrix less the interpolated face flux
};

template <typename T, int NB>
struct QLds {
  double tm[QTE][16][64];            // per wave: staging of 16 doubles per lane; own modal traces
  double th[QTE][2][16][16];         // per wave: modal traces across the tile-boundary x / y face
  // per wave: interactive fluxes of two node slots (FP64), or of the four of a node
  // block (bfloat16-split, T = float, whose node loop forms all of them before the residuals)
  Half2<T> fs[QTE][sizeof(T) == 8 ? 2 : 4][4][2][16];
  double fA[NB * 4 * 64];            // FP64 expansion operands (this kernel's mode mapping)
  double fP[NB * 4 * 64];            // FP64 projection operands, or the bfloat16 pairs
  double fW[NB * 16];                // quadrature weight per (register, lane group)
  double red[QTE];
};

// tile of workgroup blockIdx.x: consecutive workgroups go to different XCDs, so
// each XCD gets a contiguous band of tiles, walked in 8 x 8 blocks
__device__ __forceinline__ void tile_of(int ntx, int nty, int& tx, int& ty) {
  const int ntiles = ntx * nty;
  int tile = blockIdx.x;
  if (ntiles % 8 == 0) tile = (tile % 8) * (ntiles / 8) + tile / 8;
  if (ntx % 8 == 0 && nty % 8 == 0) {
    const int blk = tile >> 6, w = tile & 63, nbx = ntx / 8;
    tx = (blk % nbx) * 8 + (w & 7);
    ty = (blk / nbx) * 8 + (w >> 3);
  } else {
    tx = tile % ntx;
    ty = tile / ntx;
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sums and extrema over the 64 lanes of a wave (every lane gets the result)
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// sum over the four lane groups (same point j)
__device__ __forceinline__ double group_sum(double v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}

// FP64 expansion of one variable in node block nb: D(node, point) from the
// coefficients (or modal traces) b[t] of this lane, with the LDS operand table
__device__ __forceinline__ v4d expand64(const double* fA_nb, const double (&b)[4], int l) {
  v4d d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < 4; ++t) d = mfma64(fA_nb[t * 64 + l], b[t], d);
  return d;
}
// bfloat16-split expansion: the small cross terms first, the main product last
__device__ __forceinline__ v4f expand_bf(v4s ah, v4s al, v4s bh, v4s bl) {
  const v4f d = {0.0f, 0.0f, 0.0f, 0.0f};
  return mfma_split(ah, al, bh, bl, d);
}

// ---------------------------------------------------------------------------
// per-lane geometry of the element and of flux point j
// ---------------------------------------------------------------------------
struct QLane {
  int w, l, g, j, a, b;
  int side, fi;          // flux point j: face side (x-lo, x-hi, y-lo, y-hi), index along the face
  int nbr_w;             // wave of the in-tile neighbour across flux point j, or -1
  bool halo;             // the neighbour lies in another tile (its traces from tr_in)
  bool boundary;         // no neighbour: domain boundary, ghost state
  int hf;                // 0: x face, 1: y face
  int mirror;            // the neighbour's flux point facing j
  bool lo_side;
};

// modal traces at flux point j of the coefficients staged in LDS (s, t, lane):
// the line of points through j, interpolated to the face
__device__ __forceinline__ void modal_traces(const KParams& P, const QLane& Q, const double (&st)[16][64],
                                             double (&tr)[4][4]) {
  double wl[4];
  int line[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    line[c] = Q.g * 16 + ((Q.side < 2) ? c + NP * Q.fi : Q.fi + NP * c);
    wl[c] = Q.lo_side ? P.tab.lL[c] : P.tab.lR[c];
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double* r = st[s * 4 + t];
      tr[s][t] = trace4(wl, r[line[0]], r[line[1]], r[line[2]], r[line[3]]);
    }
}

// ---------------------------------------------------------------------------
// positivity limiter on the element of this wave (Sec. 4.3); o[s][t]: this
// lane's coefficients (point j, modes qmode(t, g))
// ---------------------------------------------------------------------------
template <int M, int NQ, int MODE>
__device__ int limit_q(const KParams& P, const QLane& Q, double (&o)[4][4], double (&st)[16][64], const double* fA,
                       const double* cmax) {
  constexpr int NB = (NQ + 15) / 16;
  const double gm = P.gamma;
  const int a = Q.a, b = Q.b, g = Q.g;
  // element x random mean from mode 0 (lane group 0, register 0)
  const double wj = 0.25 * P.tab.w[a] * P.tab.w[b];
  double ub[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) ub[s] = wave_sum(g == 0 ? wj * o[s][0] : 0.0);
  const double pb = (gm - 1.0) * (ub[3] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2]) / ub[0]);
  const bool realizable = ub[0] > 0.0 && pb > 0.0 && isfinite(ub[0]) && isfinite(ub[1]) && isfinite(ub[2]) &&
                          isfinite(ub[3]);
  if (!realizable && Q.l == 0) atomicOr(P.status, kStatusNotRealizable);
  const double eps = fmin(1e-8, fmin(ub[0], pb));

  // rigorous bounds: value(z) = c_0 + sum_{k>=1} c_k Phi_k(z), |Phi_k(z_q)| <= cmax_k
  double mean[4], var[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double v = 0.0, m0 = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = qmode<MODE>(t, g);
      if (k == 0) m0 = o[s][t];
      else if (k < M) v += fabs(o[s][t]) * cmax[k];
    }
    mean[s] = group_sum(m0);
    var[s] = group_sum(v);
  }
  // decision from the means and bounds of all four variables at one location
  auto safe = [&](const double* mn, const double* vr) {
    const double rlo = mn[0] - vr[0];
    const double elo = mn[3] - vr[3];
    const double mx = fabs(mn[1]) + vr[1];
    const double my = fabs(mn[2]) + vr[2];
    const double tol_r = 1e-10 * (fabs(mn[0]) + vr[0]);
    if (!(rlo > eps + tol_r)) return false;
    const double kin = 0.5 * (mx * mx + my * my) / rlo;
    const double plo = (gm - 1.0) * (elo - kin);
    const double tol_p = 1e-10 * (gm - 1.0) * (fabs(mn[3]) + vr[3] + kin);
    return plo > eps + tol_p;
  };
  double rlx[4], rrx[4], rly[4], rry[4], ax[4], bx[4], ay[4], by[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rlx[k] = P.tab.lL[(a + k) & 3];
    rrx[k] = P.tab.lR[(a + k) & 3];
    rly[k] = P.tab.lL[(b - k) & 3];
    rry[k] = P.tab.lR[(b - k) & 3];
    ax[k] = fabs(rlx[k]);
    bx[k] = fabs(rrx[k]);
    ay[k] = fabs(rly[k]);
    by[k] = fabs(rry[k]);
  }
  bool ok = safe(mean, var);
  {
    double m1[4], v1[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) { m1[s] = xdot(rlx, mean[s]); v1[s] = xdot(ax, var[s]); }
    ok = ok && safe(m1, v1);
#pragma unroll
    for (int s = 0; s < 4; ++s) { m1[s] = xdot(rrx, mean[s]); v1[s] = xdot(bx, var[s]); }
    ok = ok && safe(m1, v1);
#pragma unroll
    for (int s = 0; s < 4; ++s) { m1[s] = ydot(rly, mean[s]); v1[s] = ydot(ay, var[s]); }
    ok = ok && safe(m1, v1);
#pragma unroll
    for (int s = 0; s < 4; ++s) { m1[s] = ydot(rry, mean[s]); v1[s] = ydot(by, var[s]); }
    ok = ok && safe(m1, v1);
  }
  const bool need = realizable && (__ballot(!ok) != 0);
  if (!need) return 0;  // uniform over the wave

  // node by node: the state at every solution point and flux point and node
  double tr[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) st[s * 4 + t][Q.l] = o[s][t];
  wave_sync();
  modal_traces(P, Q, st, tr);
  wave_sync();
  double rmin = INFINITY, pmin = INFINITY;
  auto nodal = [&](int nb, const double (&c)[4][4], double (&U)[4][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const v4d d = expand64(fA + nb * 256, c[s], Q.l);
#pragma unroll
      for (int r = 0; r < 4; ++r) U[s][r] = d[r];
    }
  };
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    double U[4][4], V[4][4];
    nodal(nb, o, U);
    nodal(nb, tr, V);
#pragma unroll
    for (int r = 0; r < qslots(NQ, nb); ++r) {
      if (16 * nb + g + 4 * r >= NQ) continue;
      const double X[4] = {U[0][r], U[1][r], U[2][r], U[3][r]};
      const double Y[4] = {V[0][r], V[1][r], V[2][r], V[3][r]};
      rmin = fmin(rmin, fmin(X[0], Y[0]));
      pmin = fmin(pmin, fmin(euler_p(X, gm), euler_p(Y, gm)));
    }
  }
  rmin = wave_min(rmin);
  pmin = wave_min(pmin);
  if (!(fmin(rmin, pmin) < eps)) return 0;
  const double beta1 = (rmin >= eps) ? 1.0 : (ub[0] - eps) / (ub[0] - rmin);
  double bmin = 1.0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    double U[4][4], V[4][4];
    nodal(nb, o, U);
    nodal(nb, tr, V);
#pragma unroll
    for (int r = 0; r < qslots(NQ, nb); ++r) {
      if (16 * nb + g + 4 * r >= NQ) continue;
      double X[4] = {U[0][r], U[1][r], U[2][r], U[3][r]};
      double Y[4] = {V[0][r], V[1][r], V[2][r], V[3][r]};
      X[0] = beta1 * (X[0] - ub[0]) + ub[0];
      Y[0] = beta1 * (Y[0] - ub[0]) + ub[0];
      if (euler_p(X, gm) < eps) bmin = fmin(bmin, pressure_root<kEuler2>(ub, X, eps, gm));
      if (euler_p(Y, gm) < eps) bmin = fmin(bmin, pressure_root<kEuler2>(ub, Y, eps, gm));
    }
  }
  const double beta2 = wave_min(bmin);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = qmode<MODE>(t, g);
    const double m0 = (k == 0) ? 1.0 : 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double v = o[s][t];
      if (s == 0) v = beta1 * (v - ub[0] * m0) + ub[0] * m0;
      o[s][t] = (k < M) ? beta2 * (v - ub[s] * m0) + ub[s] * m0 : 0.0;
    }
  }
  return 1;
}

// ---------------------------------------------------------------------------
// detector + modal filter on the element of this wave (Sec. 4.1, 4.2)
// ---------------------------------------------------------------------------
template <int M, int MODE>
__device__ int sensor_filter_q(const KParams& P, const QLane& Q, double (&o)[4][4], double dt) {
  const int a = Q.a, b = Q.b, j = Q.j, g = Q.g;
  double vix[4], viy[4], vx[4], vy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    vix[k] = P.tab.Vinv[a * NP + ((a + k) & 3)];
    viy[k] = P.tab.Vinv[b * NP + ((b - k) & 3)];
    vx[k] = P.tab.V[a * NP + ((a + k) & 3)];
    vy[k] = P.tab.V[b * NP + ((b - k) & 3)];
  }
  // energies of the first variable's spatial-chaos modes
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = qmode<MODE>(t, g);
    const double m = ydot(viy, xdot(vix, o[0][t]));
    const double e2 = (k < M) ? m * m : 0.0;
    num += (k < M) ? e2 * P.tab.shell[k * NSP + j] : 0.0;
    den += e2;
  }
  num = wave_sum(num);
  den = wave_sum(den);
  const bool flag = (P.sensor == FRSG_SENSOR_ALWAYS) || (den > 0.0 && num / den > P.sensor_thr);
  if (!flag) return 0;  // uniform
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = qmode<MODE>(t, g);
    const double f = (k < M) ? P.tab.filt[k * NSP + j] : 0.0;
    const double lam = (P.filter == FRSG_FILTER_EXP) ? exp(-P.alpha * dt * f) : f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double m = ydot(viy, xdot(vix, o[s][t])) * lam;
      o[s][t] = (k < M) ? ydot(vy, xdot(vx, m)) : 0.0;
    }
  }
  return 1;
}

// ---------------------------------------------------------------------------
// the stage kernel
// ---------------------------------------------------------------------------
#ifndef FRSG_QUAD_F64_WAVES
#define FRSG_QUAD_F64_WAVES 1
#endif
template <int M, int NQ, int MODE, int FLUX>
__global__ void __launch_bounds__(QBLK) __attribute__((amdgpu_waves_per_eu(MODE == kQF64 ? FRSG_QUAD_F64_WAVES : 2)))
k_quad_stage(KParams P, QArgs A) {
  using T = typename std::conditional<MODE == kQF64, double, float>::type;
  constexpr int NB = (NQ + 15) / 16;
  __shared__ QLds<T, NB> L;
  const QuadFragLayout FL = quad_frag_layout(NQ);

  QLane Q;
  const int tid = threadIdx.x;
  Q.w = tid >> 6;
  Q.l = tid & 63;
  Q.g = Q.l >> 4;
  Q.j = Q.l & 15;
  Q.a = Q.j & 3;
  Q.b = Q.j >> 2;
  const int w = Q.w, l = Q.l, g = Q.g, j = Q.j, a = Q.a, b = Q.b;
  const int lx = w % QTX, ly = w / QTX;
  const int ntx = P.nx / QTX, nty = P.ny / QTY;
  int tx, ty;
  tile_of(ntx, nty, tx, ty);
  const int ix = QTX * tx + lx, iy = QTY * ty + ly;
  const int e = iy * P.nx + ix;
  const long EN = (long)P.E * NSP;
  const double dt = (A.stage == 0) ? 0.0 : *P.dt;

  // operand tables into LDS
  {
    const double* srcA = A.frag + (MODE == kQF64 ? FL.aexp_f : FL.aexp_b);
    for (int i = tid; i < NB * 256; i += QBLK) L.fA[i] = srcA[i];
    if (MODE == kQF64) {
      for (int i = tid; i < NB * 256; i += QBLK) L.fP[i] = A.frag[FL.aprj + i];
    } else {
      for (int i = tid; i < NB * 128; i += QBLK) L.fP[i] = A.frag[FL.bexp + i];
      for (int i = tid; i < NB * 128; i += QBLK) L.fP[NB * 128 + i] = A.frag[FL.bprj + i];
    }
    for (int i = tid; i < NB * 16; i += QBLK) L.fW[i] = A.frag[FL.wslot + i];
  }

  // flux point j of this lane and the element across it
  Q.side = j >> 2;
  Q.fi = j & 3;
  Q.lo_side = (Q.side == 0 || Q.side == 2);
  Q.mirror = (Q.side ^ 1) * 4 + Q.fi;
  Q.hf = Q.side >> 1;
  Q.nbr_w = -1;
  Q.halo = false;
  Q.boundary = false;
  int nt = 0, slot = 0;  // neighbour tile and its face slot facing this tile (halo lanes)
  {
    int ntx_ = tx, nty_ = ty;
    if (Q.side == 0) {
      if (lx > 0) Q.nbr_w = w - 1;
      else if (ix == 0 && P.bc[0] != FRSG_BC_PERIODIC) Q.boundary = true;
      else { Q.halo = true; ntx_ = (tx == 0) ? ntx - 1 : tx - 1; slot = QTY + ly; }
    } else if (Q.side == 1) {
      if (lx < QTX - 1) Q.nbr_w = w + 1;
      else if (ix == P.nx - 1 && P.bc[1] != FRSG_BC_PERIODIC) Q.boundary = true;
      else { Q.halo = true; ntx_ = (tx == ntx - 1) ? 0 : tx + 1; slot = ly; }
    } else if (Q.side == 2) {
      if (ly > 0) Q.nbr_w = w - QTX;
      else if (iy == 0 && P.bc[2] != FRSG_BC_PERIODIC) Q.boundary = true;
      else { Q.halo = true; nty_ = (ty == 0) ? nty - 1 : ty - 1; slot = 2 * QTY + QTX + lx; }
    } else {
      if (ly < QTY - 1) Q.nbr_w = w + QTX;
      else if (iy == P.ny - 1 && P.bc[3] != FRSG_BC_PERIODIC) Q.boundary = true;
      else { Q.halo = true; nty_ = (ty == nty - 1) ? 0 : ty + 1; slot = 2 * QTY + lx; }
    }
    nt = nty_ * ntx + ntx_;
  }

  // own coefficients, point j, modes qmode(t, g) (the state is below 4 GiB: host check)
  const unsigned sbytes = (unsigned)(4 * M * EN * (long)sizeof(double));
  const unsigned vlane = (unsigned)(((long)(MODE == kQF64 ? g : 4 * g) * EN + (long)e * NSP + j) * sizeof(double));
  auto uoff = [&](int s, int t) {
    return (unsigned)(((long)s * M + (MODE == kQF64 ? 4 * t : t)) * EN * (long)sizeof(double));
  };
  double cf[4][4];
  {
    const auto rin = state_rsrc(A.in, sbytes);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double v = bload_stream(rin, vlane, uoff(s, t));
        cf[s][t] = (qmode<MODE>(t, g) < M) ? v : 0.0;
      }
  }
  // modal traces of the neighbour tile across a tile-boundary face (all lanes
  // load; lanes without a halo neighbour read tile 0 and drop the values)
  {
    const auto rtr = state_rsrc(A.tr_in, (unsigned)((long)ntx * nty * QTRACE_PER_TILE<M> * (long)sizeof(double)));
    const int kl = (MODE == kQF64) ? g : 4 * g;
    const unsigned hb = (unsigned)((((long)(Q.halo ? nt : 0) * QNHF + (Q.halo ? slot : 0)) * 4 * M * NP + kl * NP +
                                    Q.fi) * (long)sizeof(double));
    double hv[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        hv[s][t] = bload(rtr, hb, (unsigned)((s * M * NP + (MODE == kQF64 ? 4 * t : t) * NP) * sizeof(double)));
    // lanes of the tile-boundary face of this direction store them
    const bool tb = Q.halo || Q.boundary;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (tb) L.th[w][Q.hf][s * 4 + t][g * 4 + Q.fi] = (Q.halo && qmode<MODE>(t, g) < M) ? hv[s][t] : 0.0;
  }
  // own modal traces at flux point j, published for the neighbours in the tile
  {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) L.tm[w][s * 4 + t][l] = cf[s][t];
    wave_sync();
    double tr[4][4];
    modal_traces(P, Q, L.tm[w], tr);
    wave_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) L.tm[w][s * 4 + t][l] = tr[s][t];
  }
  __syncthreads();

  // the neighbour's modal traces at this flux point: in-tile neighbour or halo
  const double* nsrc = (Q.nbr_w >= 0) ? &L.tm[Q.nbr_w][0][g * 16 + Q.mirror] : &L.th[w][Q.hf][0][g * 4 + Q.fi];
  const int nstride = (Q.nbr_w >= 0) ? 64 : 16;

  // per-lane constants of the residual
  T dx[4], dy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    dx[k] = (T)A.Dt[a * NP + ((a + k) & 3)];
    dy[k] = (T)A.Dt[b * NP + ((b - k) & 3)];
  }
  const T dhLa = (T)P.tab.dhL[a], dhRa = (T)P.tab.dhR[a], dhLb = (T)P.tab.dhL[b], dhRb = (T)P.tab.dhR[b];
  const T iJx = (T)(1.0 / P.Jx), iJy = (T)(1.0 / P.Jy);
  const T gm = (T)P.gamma;
  const int gkind = P.bc[Q.side];
  T gstate[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) gstate[s] = (T)P.bc_state[Q.side][s];
  const int gnormal = Q.side < 2 ? 1 : 2;
  const bool wave_at_boundary = __ballot(Q.boundary) != 0;

  // projection accumulators: FP64 products, or FP32 bfloat16-split products plus
  // the mean mode in FP64
  v4d acc64[4];
  v4f accbf[4];
  double acc0[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    acc64[s] = v4d{0.0, 0.0, 0.0, 0.0};
    accbf[s] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    acc0[s] = 0.0;
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    // interactive flux at the flux point of node slot r (own and neighbour traces
    // there), into flux buffer slot `slot`
    auto face_flux = [&](const T (&To)[4][4], const T (&Tn)[4][4], int r, int slot) {
      T own[4] = {To[0][r], To[1][r], To[2][r], To[3][r]};
      T nbv[4] = {Tn[0][r], Tn[1][r], Tn[2][r], Tn[3][r]};
      if (wave_at_boundary) {  // uniform: only waves with a domain-boundary face pay for the ghosts
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          T gh = (gkind == FRSG_BC_DIRICHLET) ? gstate[s] : own[s];
          if (gkind == FRSG_BC_REFLECT && s == gnormal) gh = -gh;
          nbv[s] = Q.boundary ? gh : nbv[s];
        }
      }
      T Fs[4];
      if constexpr (FLUX == FRSG_FLUX_HLL)
        hll_e2(own, nbv, Q.lo_side, Fs, gm, Q.side >> 1);
      else
        rusanov_e2(own, nbv, Q.lo_side, Fs, gm, Q.side >> 1);
      L.fs[w][slot][g][0][j] = Half2<T>{Fs[0], Fs[1]};
      L.fs[w][slot][g][1][j] = Half2<T>{Fs[2], Fs[3]};
    };
    // nodal residual of node slot r from its nodal values U[.][r] and the interactive
    // fluxes of the element's faces in flux buffer slot `slot`; it takes U's place
    auto residual = [&](T (&U)[4][4], int r, int slot) {
      T F[4], G[4];
      {
        const T U0 = U[0][r], U1 = U[1][r], U2 = U[2][r], U3 = U[3][r];
        const T ir = recip(U0);
        const T p = (gm - T(1)) * (U3 - T(0.5) * (U1 * U1 + U2 * U2) * ir);
        const T vx = U1 * ir, vy = U2 * ir;
        F[0] = U1;
        F[1] = U1 * vx + p;
        F[2] = U2 * vx;
        F[3] = (U3 + p) * vx;
        G[0] = U2;
        G[1] = U1 * vy;
        G[2] = U2 * vy + p;
        G[3] = (U3 + p) * vy;
      }
      const Half2<T> fxl0 = L.fs[w][slot][g][0][0 + b], fxr0 = L.fs[w][slot][g][0][4 + b];
      const Half2<T> fyl0 = L.fs[w][slot][g][0][8 + a], fyr0 = L.fs[w][slot][g][0][12 + a];
      const Half2<T> fxl1 = L.fs[w][slot][g][1][0 + b], fxr1 = L.fs[w][slot][g][1][4 + b];
      const Half2<T> fyl1 = L.fs[w][slot][g][1][8 + a], fyr1 = L.fs[w][slot][g][1][12 + a];
      const T fxl[4] = {fxl0.x, fxl0.y, fxl1.x, fxl1.y}, fxr[4] = {fxr0.x, fxr0.y, fxr1.x, fxr1.y};
      const T fyl[4] = {fyl0.x, fyl0.y, fyl1.x, fyl1.y}, fyr[4] = {fyr0.x, fyr0.y, fyr1.x, fyr1.y};
      const bool valid = 16 * nb + g + 4 * r < NQ;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const T res = -(xdot(dx, F[s]) + fxl[s] * dhLa + fxr[s] * dhRa) * iJx -
                      (ydot(dy, G[s]) + fyl[s] * dhLb + fyr[s] * dhRb) * iJy;
        U[s][r] = valid ? res : T(0);
      }
    };

    T U[4][4];
    if constexpr (MODE == kQF64) {
      // nodal values at the solution point, own trace and neighbour trace at the flux point
      T To[4][4], Tn[4][4];
      const double* fA = L.fA + nb * 256;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double ob[4], nbv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          ob[t] = L.tm[w][s * 4 + t][l];
          nbv[t] = nsrc[(s * 4 + t) * nstride];
        }
        const v4d du = expand64(fA, cf[s], l);
        const v4d dO = expand64(fA, ob, l);
        const v4d dN = expand64(fA, nbv, l);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          U[s][r] = du[r];
          To[s][r] = dO[r];
          Tn[s][r] = dN[r];
        }
      }
      // node slots in pairs: interactive fluxes at the flux points, then residuals
#pragma unroll
      for (int rp = 0; rp < 2; ++rp) {
        if (2 * rp >= qslots(NQ, nb)) break;
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
          const int r = 2 * rp + rr;
          if (r >= qslots(NQ, nb)) break;
          face_flux(To, Tn, r, rr);
        }
        wave_sync();
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
          const int r = 2 * rp + rr;
          if (r >= qslots(NQ, nb)) break;
          residual(U, r, rr);
        }
        wave_sync();  // the interactive fluxes of this pair are consumed
      }
    } else {
      // traces first: their bfloat16 operands and expansions, the interactive fluxes of
      // all four node slots; then the solution points' operands, expansion and
      // residuals.  The operands are formed again for every node block (held across
      // the blocks they took 48 registers), and the traces' values die before the
      // nodal values are formed.
      const v4s ah = as_v4s(L.fP[(nb * 2 + 0) * 64 + l]), al = as_v4s(L.fP[(nb * 2 + 1) * 64 + l]);
      {
        T To[4][4], Tn[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          float y[4], z[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            y[t] = (float)L.tm[w][s * 4 + t][l];
            z[t] = (float)nsrc[(s * 4 + t) * nstride];
          }
          v4s oh, ol, nh, nl;
          split4(y, oh, ol);
          split4(z, nh, nl);
          const v4f dO = expand_bf(ah, al, oh, ol);
          const v4f dN = expand_bf(ah, al, nh, nl);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            To[s][r] = dO[r];
            Tn[s][r] = dN[r];
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (r >= qslots(NQ, nb)) break;
          face_flux(To, Tn, r, r);
        }
      }
      wave_sync();
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        float x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = (float)cf[s][t];
        v4s ch, cl;
        split4(x, ch, cl);
        const v4f du = expand_bf(ah, al, ch, cl);
#pragma unroll
        for (int r = 0; r < 4; ++r) U[s][r] = du[r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r >= qslots(NQ, nb)) break;
        residual(U, r, r);
      }
      wave_sync();  // the interactive fluxes of this block are consumed
    }

    // Galerkin projection of the residuals of this node block
    if constexpr (MODE == kQF64) {
#pragma unroll
      for (int r = 0; r < qslots(NQ, nb); ++r) {
        const double ap = L.fP[(nb * 4 + r) * 64 + l];
#pragma unroll
        for (int s = 0; s < 4; ++s) acc64[s] = mfma64(ap, U[s][r], acc64[s]);
      }
    } else {
      const v4s ph = as_v4s(L.fP[NB * 128 + (nb * 2 + 0) * 64 + l]);
      const v4s pl = as_v4s(L.fP[NB * 128 + (nb * 2 + 1) * 64 + l]);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        float x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = (r < qslots(NQ, nb)) ? U[s][r] : 0.0f;
        v4s rh, rl;
        split4(x, rh, rl);
        accbf[s] = mfma_bf(pl, rh, accbf[s]);
        accbf[s] = mfma_bf(ph, rl, accbf[s]);
        accbf[s] = mfma_bf(ph, rh, accbf[s]);
        // the mean mode in FP64: sum_q w_q R_q
#pragma unroll
        for (int r = 0; r < qslots(NQ, nb); ++r) acc0[s] = fma(L.fW[nb * 16 + r * 4 + g], (double)x[r], acc0[s]);
      }
    }
  }

  // projected residual, lane (g, j), registers t: modes qmode(t, g)
  double R[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double m0 = (MODE == kQBF16) ? group_sum(acc0[s]) : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double v = (MODE == kQF64) ? acc64[s][t] : (double)accbf[s][t];
      if (MODE == kQBF16 && qmode<MODE>(t, g) == 0) v = m0;
      R[s][t] = v;
    }
  }

  // ----------------------------------------------------------------- epilogue
  const auto rout = state_rsrc(A.out, sbytes);
  if (A.stage == 0) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (qmode<MODE>(t, g) < M) bstore(R[s][t], rout, vlane, uoff(s, t));
    return;
  }
  double o[4][4];
  {
    const auto ru = state_rsrc(A.u, A.cu != 0.0 ? sbytes : 0u);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double uu = bload_stream(ru, vlane, uoff(s, t));  // 0 from an empty range when cu = 0
        o[s][t] = (qmode<MODE>(t, g) < M) ? A.cu * uu + A.cw * (cf[s][t] + dt * R[s][t]) : 0.0;
      }
  }
  __syncthreads();  // every wave is done with the published traces: L.tm becomes staging space
  if (A.stage == 3) {
    int ff = 0;
    if (P.filter != FRSG_FILTER_NONE) ff = sensor_filter_q<M, MODE>(P, Q, o, dt);
    if (l == 0 && A.flag_filt) A.flag_filt[e] = (unsigned char)ff;
  }
  if (P.limiter) {
    const int lf = limit_q<M, NQ, MODE>(P, Q, o, L.tm[w], L.fA, A.cmax);
    if (l == 0 && A.flag_lim) A.flag_lim[e] = (unsigned char)lf;
  } else if (l == 0 && A.flag_lim) {
    A.flag_lim[e] = 0;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (qmode<MODE>(t, g) < M) bstore(o[s][t], rout, vlane, uoff(s, t));

  // modal face traces of the new state on the tile's boundary faces, for the
  // next launch: the same interpolation, in the same order, as every other
  // producer of face traces
  if (A.tr_out) {  // uniform
    wave_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) L.tm[w][s * 4 + t][l] = o[s][t];
    wave_sync();
    double tr[4][4];
    modal_traces(P, Q, L.tm[w], tr);
    const bool tb = (Q.side == 0 && lx == 0) || (Q.side == 1 && lx == QTX - 1) || (Q.side == 2 && ly == 0) ||
                    (Q.side == 3 && ly == QTY - 1);
    // this tile's own face slot of flux point j
    const int myslot = Q.side == 0 ? ly : Q.side == 1 ? QTY + ly : Q.side == 2 ? 2 * QTY + lx : 2 * QTY + QTX + lx;
    const int tile_id = ty * ntx + tx;
    const auto rtr = state_rsrc(A.tr_out, (unsigned)((long)ntx * nty * QTRACE_PER_TILE<M> * (long)sizeof(double)));
    const int kl = (MODE == kQF64) ? g : 4 * g;
    const unsigned ob = (unsigned)((((long)tile_id * QNHF + myslot) * 4 * M * NP + kl * NP + Q.fi) *
                                   (long)sizeof(double));
    // one store instruction writes 32-byte pieces of four lines, the other three fill
    // the rest: cached stores, so that the L2 merges the pieces before they go out
    // (streaming stores here measured 2 % slower)
    if (tb) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (qmode<MODE>(t, g) < M)
            bstore_cached(tr[s][t], rtr, ob,
                          (unsigned)((s * M * NP + (MODE == kQF64 ? 4 * t : t) * NP) * sizeof(double)));
    }
  }

  // CFL maximum of the new state for the next step (FP64 expansion)
  if (A.stage == 3 && A.lam_next) {
    const double gd = P.gamma, idx = 1.0 / P.dx, idy = 1.0 / P.dy;
    double rate = 0.0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      double U[4][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const v4d d = expand64(L.fA + nb * 256, o[s], l);
#pragma unroll
        for (int r = 0; r < 4; ++r) U[s][r] = d[r];
      }
#pragma unroll
      for (int r = 0; r < qslots(NQ, nb); ++r) {
        if (16 * nb + g + 4 * r >= NQ) continue;
        const double ir = recip(U[0][r]);
        const double vx = U[1][r] * ir, vy = U[2][r] * ir;
        const double p = (gd - 1.0) * (U[3][r] - 0.5 * (U[1][r] * vx + U[2][r] * vy));
        const double c = sqrt(gd * p * ir);
        double rt = (fabs(vx) + c) * idx + (fabs(vy) + c) * idy;
        if (!(rt == rt)) rt = __longlong_as_double(0x7ff0000000000000ll);  // NaN counts as infinity
        rate = fmax(rate, rt);
      }
    }
    rate = wave_max(rate);
    if (l == 0) L.red[w] = rate;
    __syncthreads();
    if (tid == 0) {
      double r = L.red[0];
      for (int i = 1; i < QTE; ++i) r = fmax(r, L.red[i]);
      atomicMax(A.lam_next, (unsigned long long)__double_as_longlong(r));
    }
  }
}

// modal face traces of a state on every tile boundary face (for the first
// stage of a call): one thread per (tile, slot, variable, mode, face point)
template <int M>
__global__ void __launch_bounds__(256) k_quad_traces(KParams P, const double* __restrict__ u, double* tr) {
  const long n = (long)(P.nx / QTX) * (P.ny / QTY) * QTRACE_PER_TILE<M>;
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (i >= n) return;
  const int fp = (int)(i % NP), k = (int)((i / NP) % M), s = (int)((i / (NP * M)) % 4);
  const int slot = (int)((i / (NP * M * 4)) % QNHF);
  const long tile = i / (NP * M * 4 * QNHF);
  const int ntx = P.nx / QTX;
  const int tx = (int)(tile % ntx), ty = (int)(tile / ntx);
  int lx, ly, side;
  if (slot < QTY) { lx = 0; ly = slot; side = 0; }
  else if (slot < 2 * QTY) { lx = QTX - 1; ly = slot - QTY; side = 1; }
  else if (slot < 2 * QTY + QTX) { lx = slot - 2 * QTY; ly = 0; side = 2; }
  else { lx = slot - 2 * QTY - QTX; ly = QTY - 1; side = 3; }
  const long e = (long)(QTY * ty + ly) * P.nx + QTX * tx + lx;
  const long EN = (long)P.E * NSP;
  const double* base = u + ((long)s * M + k) * EN + e * NSP;
  const bool lo = (side == 0 || side == 2);
  double w[4], v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    w[c] = lo ? P.tab.lL[c] : P.tab.lR[c];
    v[c] = base[(side < 2) ? c + NP * fp : fp + NP * c];
  }
  tr[i] = trace4(w, v[0], v[1], v[2], v[3]);
}

}  // namespace

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define FRSG_QUAD_SIZES(X) X(15, 25) X(10, 16) X(6, 9) X(3, 4) X(5, 5)

bool quad_mfma_supported(const KParams& P) {
  if (P.eq != kEuler2 || P.np1 != 4 || P.nx % QTX != 0 || P.ny % QTY != 0) return false;
  if ((double)4 * P.M * P.E * NSP * sizeof(double) >= 4294967296.0) return false;
#define X(MM, QQ) if (P.M == MM && P.Nq == QQ) return true;
  FRSG_QUAD_SIZES(X)
#undef X
  return false;
}

size_t quad_trace_count(int nx, int ny, int M) { return (size_t)(nx / QTX) * (ny / QTY) * QNHF * 4 * M * NP; }

template <int M, int NQ>
static hipError_t launch_quad_t(const KParams& P, const QuadStage& S, hipStream_t s) {
  QArgs A;
  A.cu = S.cu;
  A.cw = S.cw;
  A.stage = S.stage;
  A.flag_lim = S.flag_lim;
  A.flag_filt = S.flag_filt;
  A.lam_next = S.lam_next;
  A.in = S.in;
  A.u = S.u;
  A.out = S.out;
  A.tr_in = S.tr_in;
  A.tr_out = S.tr_out;
  A.frag = S.frag;
  A.cmax = S.cmax;
  A.Dt = S.Dt;
  const unsigned ntiles = (unsigned)((P.nx / QTX) * (P.ny / QTY));
  const bool hll = P.flux == FRSG_FLUX_HLL;
  if (S.bf16) {
    if (hll)
      hipLaunchKernelGGL((k_quad_stage<M, NQ, kQBF16, FRSG_FLUX_HLL>), dim3(ntiles), dim3(QBLK), 0, s, P, A);
    else
      hipLaunchKernelGGL((k_quad_stage<M, NQ, kQBF16, FRSG_FLUX_RUSANOV>), dim3(ntiles), dim3(QBLK), 0, s, P, A);
  } else {
    if (hll)
      hipLaunchKernelGGL((k_quad_stage<M, NQ, kQF64, FRSG_FLUX_HLL>), dim3(ntiles), dim3(QBLK), 0, s, P, A);
    else
      hipLaunchKernelGGL((k_quad_stage<M, NQ, kQF64, FRSG_FLUX_RUSANOV>), dim3(ntiles), dim3(QBLK), 0, s, P, A);
  }
  return hipGetLastError();
}

hipError_t launch_quad_stage(const KParams& P, const QuadStage& S, hipStream_t s) {
  if (!S.tr_in) return hipErrorInvalidValue;
#define X(MM, QQ) if (P.M == MM && P.Nq == QQ) return launch_quad_t<MM, QQ>(P, S, s);
  FRSG_QUAD_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_quad_traces(const KParams& P, const double* u, double* tr, hipStream_t s) {
  const long n = (long)quad_trace_count(P.nx, P.ny, P.M);
  const unsigned grid = (unsigned)((n + 255) / 256);
#define X(MM, QQ) \
  if (P.M == MM && P.Nq == QQ) { \
    hipLaunchKernelGGL((k_quad_traces<MM>), dim3(grid), dim3(256), 0, s, P, u, tr); \
    return hipGetLastError(); \
  }
  FRSG_QUAD_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace frsg
