// Triangle path of the 2D Euler right-hand side (Sec. 3.5 multi-dimensional FR
// on the triangles of Sec. 3.1), multi-pass like the generic quadrilateral path:
// the nodal values and fluxes at (node, element, solution point) come from the
// shared nodal pass; this file adds the interactive fluxes at the flux points,
// the nodal residual (flux divergence plus the correction-field lifting) and
// the CFL maximum.  Nodal arrays: [S][Nq][E][N_p]; face jumps: [S][Nq][E][3 nfp].
#include "device_common.hpp"

namespace frsg {
namespace {

constexpr int kBlockT = 256;

__device__ __forceinline__ double euler2_p(const double* U, double gamma) {
  return (gamma - 1.0) * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]);
}

// normal flux F . n of the 2D Euler equations, unit normal (nx, ny)
__device__ __forceinline__ void normal_flux(const double* U, double nx, double ny, double gamma, double* F,
                                            double& vn, double& c) {
  const double p = euler2_p(U, gamma);
  vn = (U[1] * nx + U[2] * ny) / U[0];
  c = sqrt(gamma * p / U[0]);
  F[0] = U[0] * vn;
  F[1] = U[1] * vn + p * nx;
  F[2] = U[2] * vn + p * ny;
  F[3] = (U[3] + p) * vn;
}

// interactive flux along the normal, per random node: Lax-Friedrichs with the
// larger of |v.n| + c on the two sides, or HLL with Davis's speeds
__device__ __forceinline__ void flux_n(int kind, const double* L, const double* R, double nx, double ny, double gamma,
                                       double* Fs) {
  double FL[4], FR[4], uL, cL, uR, cR;
  normal_flux(L, nx, ny, gamma, FL, uL, cL);
  normal_flux(R, nx, ny, gamma, FR, uR, cR);
  if (kind == FRSG_FLUX_HLL) {
    const double SL = fmin(uL - cL, uR - cR), SR = fmax(uL + cL, uR + cR);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      Fs[s] = (SL >= 0.0) ? FL[s] : (SR <= 0.0) ? FR[s] : (SR * FL[s] - SL * FR[s] + (SL * SR) * (R[s] - L[s])) / (SR - SL);
  } else {
    const double lam = fmax(fabs(uL) + cL, fabs(uR) + cR);
#pragma unroll
    for (int s = 0; s < 4; ++s) Fs[s] = 0.5 * (FL[s] + FR[s]) - 0.5 * lam * (R[s] - L[s]);
  }
}

// 1/x: hardware estimate and two Newton steps (full double accuracy for the
// positive densities it is applied to)
__device__ __forceinline__ double rcp2(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// a[s] for a run-time s without indexing a private array
__device__ __forceinline__ double pick4(const double* a, int s) {
  return s == 0 ? a[0] : (s == 1 ? a[1] : (s == 2 ? a[2] : a[3]));
}

// component s of the interactive flux along the normal, with one reciprocal of the
// density per side (the fused kernel's lanes each produce one conserved variable)
__device__ __forceinline__ double flux_n_comp(int kind, const double* L, const double* R, double nx, double ny,
                                              double gamma, int s, double Ls, double Rs) {
  const double iL = rcp2(L[0]), iR = rcp2(R[0]);
  const double uL = (L[1] * nx + L[2] * ny) * iL, uR = (R[1] * nx + R[2] * ny) * iR;
  const double pL = (gamma - 1.0) * (L[3] - 0.5 * (L[1] * L[1] + L[2] * L[2]) * iL);
  const double pR = (gamma - 1.0) * (R[3] - 0.5 * (R[1] * R[1] + R[2] * R[2]) * iR);
  const double cL = sqrt(gamma * pL * iL), cR = sqrt(gamma * pR * iR);
  const double ns = s == 1 ? nx : (s == 2 ? ny : 0.0);
  // Ls = L[s] and Rs = R[s] are the lane's own values
  const double FL = (s == 3 ? Ls + pL : Ls) * uL + pL * ns;
  const double FR = (s == 3 ? Rs + pR : Rs) * uR + pR * ns;
  const double dU = Rs - Ls;
  if (kind == FRSG_FLUX_HLL) {
    const double SL = fmin(uL - cL, uR - cR), SR = fmax(uL + cL, uR + cR);
    return (SL >= 0.0) ? FL : (SR <= 0.0) ? FR : (SR * FL - SL * FR + (SL * SR) * dU) / (SR - SL);
  }
  const double lam = fmax(fabs(uL) + cL, fabs(uR) + cR);
  return 0.5 * (FL + FR) - 0.5 * lam * dU;
}

// ghost state outside a boundary face of kind bc[side] (reflection about the face)
__device__ __forceinline__ void ghost_n(const KParams& P, int side, const double* in, double nx, double ny,
                                        double* out) {
  const int kind = P.bc[side];
#pragma unroll
  for (int s = 0; s < 4; ++s) out[s] = (kind == FRSG_BC_DIRICHLET) ? P.bc_state[side][s] : in[s];
  if (kind == FRSG_BC_REFLECT) {
    const double mn = in[1] * nx + in[2] * ny;
    out[1] = in[1] - 2.0 * mn * nx;
    out[2] = in[2] - 2.0 * mn * ny;
  }
}

// thread per (node q, element e, face f, flux point k): traces of both sides
// (the neighbour runs the shared face the other way), interactive flux minus the
// interpolated flux along the outward normal, times (face length / reference
// face length / det) for the lifting
__global__ void __launch_bounds__(kBlockT) k_faces_tri(KParams P, const double* __restrict__ Un,
                                                       const double* __restrict__ Fn, const double* __restrict__ Gn,
                                                       double* __restrict__ Jump) {
  const int np = P.nsp, nfp = P.nfp, E = P.E;
  const long NF = (long)P.Nq * E * 3 * nfp;
  const long t = blockIdx.x * (long)kBlockT + threadIdx.x;
  if (t >= NF) return;
  const int k = (int)(t % nfp);
  const int f = (int)((t / nfp) % 3);
  const long qe = t / (3 * nfp);
  const int e = (int)(qe % E);
  const long q = qe / E;
  const long total = (long)P.Nq * E * np;
  const double* geo = P.tri_geo + (long)e * kTriGeo;
  const double nx = geo[kGeoN0 + 2 * f], ny = geo[kGeoN0 + 2 * f + 1];
  const double* Lrow = P.tri_Lf + (f * nfp + k) * np;
  const long base = qe * np;
  double UL[4], FD[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double u = 0.0, fx = 0.0, fy = 0.0;
    for (int i = 0; i < np; ++i) {
      const double l = Lrow[i];
      u += l * Un[s * total + base + i];
      fx += l * Fn[s * total + base + i];
      fy += l * Gn[s * total + base + i];
    }
    UL[s] = u;
    FD[s] = nx * fx + ny * fy;
  }
  double UR[4];
  const int nb = P.tri_nbr[e * 6 + f];
  if (nb >= 0) {
    const int g = P.tri_nbr[e * 6 + 3 + f];
    const double* Lnb = P.tri_Lf + (g * nfp + (nfp - 1 - k)) * np;
    const long nbase = (q * E + nb) * np;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double u = 0.0;
      for (int i = 0; i < np; ++i) u += Lnb[i] * Un[s * total + nbase + i];
      UR[s] = u;
    }
  } else {
    ghost_n(P, -1 - nb, UL, nx, ny, UR);
  }
  double Fs[4];
  flux_n(P.flux, UL, UR, nx, ny, P.gamma, Fs);
  const double sc = geo[kGeoSc0 + f];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    Jump[s * NF + t] = (Fs[s] - FD[s]) * sc;
  }
}

// thread per (node q, element e, solution point j): -(div F^D + sum_fk lift_jfk jump_fk)
__global__ void __launch_bounds__(kBlockT) k_resid_tri(KParams P, const double* __restrict__ Fn,
                                                       const double* __restrict__ Gn,
                                                       const double* __restrict__ Jump, double* __restrict__ Rn) {
  const int np = P.nsp, nf = 3 * P.nfp, E = P.E;
  const long total = (long)P.Nq * E * np;
  const long t = blockIdx.x * (long)kBlockT + threadIdx.x;
  if (t >= total) return;
  const int j = (int)(t % np);
  const long qe = t / np;
  const int e = (int)(qe % E);
  const double* geo = P.tri_geo + (long)e * kTriGeo;
  const double rx = geo[kGeoRx], ry = geo[kGeoRy], sx = geo[kGeoSx], sy = geo[kGeoSy];
  const double* Dr = P.tri_Dr + j * np;
  const double* Ds = P.tri_Ds + j * np;
  const double* lift = P.tri_lift + j * nf;
  const long NF = (long)P.Nq * E * nf;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double* F = Fn + s * total + qe * np;
    const double* G = Gn + s * total + qe * np;
    double dr = 0.0, ds = 0.0;
    for (int i = 0; i < np; ++i) {
      const double fr = rx * F[i] + ry * G[i];
      const double fs = sx * F[i] + sy * G[i];
      dr += Dr[i] * fr;
      ds += Ds[i] * fs;
    }
    const double* J = Jump + s * NF + qe * nf;
    double c = 0.0;
    for (int m = 0; m < nf; ++m) c += lift[m] * J[m];
    Rn[s * total + t] = -(dr + ds + c);
  }
}

// CFL maximum over (node, element, solution point) of (|v| + c) / d_e, from the
// nodal values; exact max, so the reduction order does not matter
__global__ void __launch_bounds__(kBlockT) k_cfl_tri(KParams P, const double* __restrict__ Un) {
  __shared__ double sm[kBlockT];
  const int np = P.nsp, E = P.E;
  const long total = (long)P.Nq * E * np;
  const long t = blockIdx.x * (long)kBlockT + threadIdx.x;
  double rate = 0.0;
  if (t < total) {
    const int e = (int)((t / np) % E);
    double U[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) U[s] = Un[s * total + t];
    const double p = euler2_p(U, P.gamma);
    const double lam = sqrt(U[1] * U[1] + U[2] * U[2]) / U[0] + sqrt(P.gamma * p / U[0]);
    rate = lam / P.tri_geo[(long)e * kTriGeo + kGeoDin];
    if (!(rate == rate)) rate = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf, dt -> 0
  }
  sm[threadIdx.x] = rate;
  __syncthreads();
  for (int o = kBlockT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(P.lam_bits, (unsigned long long)__double_as_longlong(sm[0]));
}

unsigned blocks(long n) { return (unsigned)((n + kBlockT - 1) / kBlockT); }

}  // namespace

hipError_t launch_faces_tri(const KParams& P, const double* Un, const double* Fn, const double* Gn, double* Jump,
                            hipStream_t s) {
  if (P.eq != FRSG_EULER2D || P.nsp > kTriMaxNp || P.nfp < 1) return hipErrorInvalidValue;
  const long NF = (long)P.Nq * P.E * 3 * P.nfp;
  hipLaunchKernelGGL(k_faces_tri, dim3(blocks(NF)), dim3(kBlockT), 0, s, P, Un, Fn, Gn, Jump);
  return hipGetLastError();
}

hipError_t launch_resid_tri(const KParams& P, const double* Fn, const double* Gn, const double* Jump, double* Rn,
                            hipStream_t s) {
  if (P.eq != FRSG_EULER2D || P.nsp > kTriMaxNp) return hipErrorInvalidValue;
  const long total = (long)P.Nq * P.E * P.nsp;
  hipLaunchKernelGGL(k_resid_tri, dim3(blocks(total)), dim3(kBlockT), 0, s, P, Fn, Gn, Jump, Rn);
  return hipGetLastError();
}

hipError_t launch_cfl_tri(const KParams& P, const double* Un, hipStream_t s) {
  if (P.eq != FRSG_EULER2D) return hipErrorInvalidValue;
  const long total = (long)P.Nq * P.E * P.nsp;
  hipLaunchKernelGGL(k_cfl_tri, dim3(blocks(total)), dim3(kBlockT), 0, s, P, Un);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// fused stage kernel: one launch per Runge-Kutta stage on triangles
// ---------------------------------------------------------------------------
// Each element gets 4 x SLOTS threads, thread (state s, slot): slot < N_p is
// solution point j, slot < 3 nfp is flux point fk.  A thread keeps its own
// chaos coefficients of state s at point j, the neighbour's modal trace at flux
// point fk and the projection accumulators of (s, j) in registers; per random
// node it expands both, and the element's nodal values, fluxes, traces and face
// jumps pass through LDS.  The residual is projected on the fly and combined
// with the stage inputs in the epilogue, so a stage reads the state once and
// writes it once; the neighbours' modal traces come from a trace pass
// (E x 3 nfp x S x M doubles) over the stage input.
namespace {

template <int PD>
struct TriShape {
  static constexpr int NPT = (PD + 1) * (PD + 2) / 2;
  static constexpr int NFP = PD + 1;
  static constexpr int NF = 3 * NFP;
  static constexpr int SLOTS = NPT > NF ? NPT : NF;
  static constexpr int TPE = 4 * SLOTS;           // threads per element
  static constexpr int EPB = 256 / TPE;           // elements per block
};

// modal traces of every element at its flux points, flux point by flux point:
//   Tm[e][fk][s][k] = sum_j Lf[fk][j] u[s][k][e][j],
// so that the 4 M values of one flux point, and the NFP points of one face, are
// contiguous: a neighbour's face is one 32 NFP M-byte run (whole cache lines).
template <int PD>
__global__ void __launch_bounds__(256) k_trace_tri(KParams P, const double* __restrict__ u, double* __restrict__ Tm) {
  using Sh = TriShape<PD>;
  const int M = P.M;
  const long E = P.E;
  const long n = 4l * M * E;
  const long t = blockIdx.x * 256l + threadIdx.x;  // (s M + k) E + e
  if (t >= n) return;
  const long e = t % E, sk = t / E;
  double v[Sh::NPT];
#pragma unroll
  for (int j = 0; j < Sh::NPT; ++j) v[j] = u[t * Sh::NPT + j];
#pragma unroll
  for (int fk = 0; fk < Sh::NF; ++fk) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < Sh::NPT; ++j) acc += P.tri_Lf[fk * Sh::NPT + j] * v[j];
    Tm[(e * Sh::NF + fk) * 4 * M + sk] = acc;
  }
}

// broadcast lane C of each group of four lanes (DPP quad permutation, all lanes active)
template <int C>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctrl = C * 85;  // quad_perm(C, C, C, C)
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, ctrl, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), ctrl, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ void quad_gather(double v, double* all) {
  all[0] = quad_bcast<0>(v);
  all[1] = quad_bcast<1>(v);
  all[2] = quad_bcast<2>(v);
  all[3] = quad_bcast<3>(v);
}

// LDS of the end-of-stage work below, per block
template <int PD, int M>
struct TriPostShared {
  using Sh = TriShape<PD>;
  double lam[M * Sh::NPT];  // filter factors of the step (exponential: exp(-alpha dt f))
  double red[Sh::EPB][4][2];
  double mn[Sh::EPB][Sh::TPE];
  int filt[Sh::EPB], need[Sh::EPB], any;
};

// End-of-stage work on triangles with the stage kernel's lane layout: the sensor-gated
// modal filter (Sec. 4.1, 4.2), then the positivity limiter (Sec. 4.3).  Lane (slot, s)
// keeps the coefficients c[] of variable s at solution point `slot`; sC holds those of
// the block's elements.  The limiter decision first uses rigorous bounds per point
// (|Phi_k(z_q)| <= cmax_k, a relative margin of 1e-10 for their rounding) at the
// solution point and, as a flux-point lane, at flux point `slot`; only blocks holding an
// element whose bound fails run the node-by-node minimum and the pressure roots, so the
// decision is the node-by-node one.  The element mean is the constant chaos mode
// averaged with the triangle's quadrature weights.  c[] and sC are updated in place;
// returns whether the lane's element changed.  Every thread of the block calls it, with
// sC complete and visible.
template <int PD, int M, int NQ>
__device__ __forceinline__ bool post_tri(const KParams& P, double (&c)[M],
                                         double (&sC)[TriShape<PD>::EPB][4][M][TriShape<PD>::NPT],
                                         TriPostShared<PD, M>& sh, const int e, const int le, const int rem,
                                         const bool active, const TriPost& post) {
  using Sh = TriShape<PD>;
  constexpr int NPT = Sh::NPT, NF = Sh::NF, TPE = Sh::TPE, EPB = Sh::EPB;
  const int slot = rem >> 2, s = rem & 3;
  const bool pt = active && slot < NPT;
  const bool fp = active && slot < NF;
  if ((int)threadIdx.x < EPB) sh.need[threadIdx.x] = 0;
  if (threadIdx.x == 0) sh.any = 0;
  bool filtered = false;
  if (post.filter) {
    const double dt = *P.dt;
    for (int i = threadIdx.x; i < M * NPT; i += blockDim.x) {
      const double f = P.tab.filt[i];
      sh.lam[i] = P.filter == FRSG_FILTER_EXP ? exp(-P.alpha * dt * f) : f;
    }
    // spatial modal coefficient m = slot of variable s for every chaos mode: (V^-1 u)_m
    double um[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double acc = 0.0;
      if (pt) {
#pragma unroll
        for (int l = 0; l < NPT; ++l) acc += P.tri_Vinv[slot * NPT + l] * sC[le][s][k][l];
      }
      um[k] = acc;
    }
    // detector: energy of the outer shell over the total, first variable
    double num = 0.0, den = 0.0;
    if (pt && s == 0 && P.sensor == FRSG_SENSOR_DETECTOR) {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double e2 = um[k] * um[k];
        num += e2 * P.tab.shell[k * NPT + slot];
        den += e2;
      }
    }
    if (active) sh.mn[le][rem] = num;
    __syncthreads();
    if (active && rem == 0) {
      double a0 = 0.0;
      for (int i = 0; i < TPE; ++i) a0 += sh.mn[le][i];
      sh.red[le][2][0] = a0;
    }
    __syncthreads();
    if (active) sh.mn[le][rem] = den;
    __syncthreads();
    if (active && rem == 0) {
      double a0 = 0.0;
      for (int i = 0; i < TPE; ++i) a0 += sh.mn[le][i];
      const double nm = sh.red[le][2][0];
      sh.filt[le] = P.sensor != FRSG_SENSOR_DETECTOR ? 1 : ((a0 > 0.0 && nm / a0 > P.sensor_thr) ? 1 : 0);
      if (post.flag_filt) post.flag_filt[e] = (unsigned char)sh.filt[le];
    }
    __syncthreads();
    filtered = active && sh.filt[le];
    // u_j <- sum_m V[j][m] (lambda_km (V^-1 u)_m), the damped modes staged in sC (every
    // lane has read sC before the barriers above)
    if (filtered && pt) {
#pragma unroll
      for (int k = 0; k < M; ++k) sC[le][s][k][slot] = um[k] * sh.lam[k * NPT + slot];
    }
    __syncthreads();
    if (filtered && pt) {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < NPT; ++m) acc += P.tri_V[slot * NPT + m] * sC[le][s][k][m];
        c[k] = acc;
      }
    }
    __syncthreads();
    if (filtered && pt) {
#pragma unroll
      for (int k = 0; k < M; ++k) sC[le][s][k][slot] = c[k];
    }
  }
  __syncthreads();
  if (!post.limit) return filtered;
  // element means of the four variables (every lane, from LDS)
  double ub[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NPT; ++j) acc += sC[le][v][0][j] * P.tab.swts[j];
    ub[v] = acc;
  }
  const double pb = (P.gamma - 1.0) * (ub[3] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2]) / ub[0]);
  const bool real = ub[0] > 0.0 && pb > 0.0 && isfinite(ub[0]) && isfinite(ub[1]) && isfinite(ub[2]) &&
                    isfinite(ub[3]);
  const double eps = fmin(1e-8, fmin(ub[0], pb));
  // flux-point lanes: interpolate all modes to their flux point
  double a[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double acc = 0.0;
    if (fp) {
#pragma unroll
      for (int j = 0; j < NPT; ++j) acc += P.tri_Lf[slot * NPT + j] * sC[le][s][k][j];
    }
    a[k] = acc;
  }
  // rigorous bounds at the solution point and the flux point of this lane
  auto bound_ok = [&](const double* coef, bool on) {
    double mn = coef[0], vr = 0.0;
#pragma unroll
    for (int k = 1; k < M; ++k) vr += fabs(coef[k]) * P.tab.cmax[k];
    double MN[4], VR[4];
    quad_gather(mn, MN);
    quad_gather(vr, VR);
    if (!on) return true;
    const double rlo = MN[0] - VR[0];
    const double tol_r = 1e-10 * (fabs(MN[0]) + VR[0]);
    if (!(rlo > eps + tol_r)) return false;
    double m2 = 0.0;
#pragma unroll
    for (int v = 1; v < 3; ++v) {
      const double mx = fabs(MN[v]) + VR[v];
      m2 += mx * mx;
    }
    const double ke = 0.5 * m2 / rlo;
    const double elo = MN[3] - VR[3];
    const double plo = (P.gamma - 1.0) * (elo - ke);
    const double tol_p = 1e-10 * (P.gamma - 1.0) * (fabs(MN[3]) + VR[3] + ke);
    return plo > eps + tol_p;
  };
  const bool ok_sp = bound_ok(c, pt && real);
  const bool ok_fp = bound_ok(a, fp && real);
  if (active && real && !(ok_sp && ok_fp)) {
    sh.need[le] = 1;
    sh.any = 1;
  }
  if (active && !real && slot == 0 && s == 0) atomicOr(P.status, kStatusNotRealizable);
  __syncthreads();
  bool act = false;
  if (sh.any) {
    const bool need = active && real && sh.need[le];
    // node-by-node minima of density and pressure over solution and flux points
    double rmin = INFINITY, pmin = INFINITY;
    for (int q = 0; q < NQ; ++q) {
      double vs = 0.0, vf = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double ph = P.tab.PhiT[q * M + k];
        vs += ph * c[k];
        vf += ph * a[k];
      }
      double Us[4], Uf[4];
      quad_gather(vs, Us);
      quad_gather(vf, Uf);
      if (need && pt) {
        rmin = fmin(rmin, Us[0]);
        pmin = fmin(pmin, (P.gamma - 1.0) * (Us[3] - 0.5 * (Us[1] * Us[1] + Us[2] * Us[2]) / Us[0]));
      }
      if (need && fp) {
        rmin = fmin(rmin, Uf[0]);
        pmin = fmin(pmin, (P.gamma - 1.0) * (Uf[3] - 0.5 * (Uf[1] * Uf[1] + Uf[2] * Uf[2]) / Uf[0]));
      }
    }
    if (active) sh.mn[le][rem] = rmin;
    __syncthreads();
    if (active && rem == 0) {
      double r = INFINITY;
      for (int i = 0; i < TPE; ++i) r = fmin(r, sh.mn[le][i]);
      sh.red[le][0][0] = r;
    }
    __syncthreads();
    if (active) sh.mn[le][rem] = pmin;
    __syncthreads();
    if (active && rem == 0) {
      double r = INFINITY;
      for (int i = 0; i < TPE; ++i) r = fmin(r, sh.mn[le][i]);
      sh.red[le][0][1] = r;
    }
    __syncthreads();
    const double Rmin = sh.red[le][0][0], Pmin = sh.red[le][0][1];
    act = need && fmin(Rmin, Pmin) < eps;
    const double beta1 = (Rmin >= eps) ? 1.0 : (ub[0] - eps) / (ub[0] - Rmin);
    // beta2: smallest root over the points whose pressure stays below eps after beta1
    double bmin = 1.0;
    for (int q = 0; q < NQ; ++q) {
      double vs = 0.0, vf = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double ph = P.tab.PhiT[q * M + k];
        vs += ph * c[k];
        vf += ph * a[k];
      }
      double Us[4], Uf[4];
      quad_gather(vs, Us);
      quad_gather(vf, Uf);
      if (act && pt) {
        Us[0] = beta1 * (Us[0] - ub[0]) + ub[0];
        if ((P.gamma - 1.0) * (Us[3] - 0.5 * (Us[1] * Us[1] + Us[2] * Us[2]) / Us[0]) < eps)
          bmin = fmin(bmin, pressure_root<kEuler2>(ub, Us, eps, P.gamma));
      }
      if (act && fp) {
        Uf[0] = beta1 * (Uf[0] - ub[0]) + ub[0];
        if ((P.gamma - 1.0) * (Uf[3] - 0.5 * (Uf[1] * Uf[1] + Uf[2] * Uf[2]) / Uf[0]) < eps)
          bmin = fmin(bmin, pressure_root<kEuler2>(ub, Uf, eps, P.gamma));
      }
    }
    if (active) sh.mn[le][rem] = bmin;
    __syncthreads();
    if (active && rem == 0) {
      double r = 1.0;
      for (int i = 0; i < TPE; ++i) r = fmin(r, sh.mn[le][i]);
      sh.red[le][1][0] = r;
    }
    __syncthreads();
    const double beta2 = sh.red[le][1][0];
    // no lane reads sC past the last barrier: rewrite it in place
    if (act && pt) {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double m0 = (k == 0) ? 1.0 : 0.0;
        double v = c[k];
        if (s == 0) v = beta1 * (v - ub[0] * m0) + ub[0] * m0;
        v = beta2 * (v - pick4(ub, s) * m0) + pick4(ub, s) * m0;
        c[k] = v;
        sC[le][s][k][slot] = v;
      }
    }
  }
  if (active && rem == 0 && post.flag_lim) post.flag_lim[e] = act ? 1 : 0;
  return filtered || act;
}

// Lane layout: lane = 4 slot + s within an element's 4 x SLOTS lanes, so the four
// conserved variables of one point sit in one group of four lanes and trade values
// by DPP instead of LDS.  Per node two barriers: after the nodal values and
// contravariant fluxes (double-buffered by node parity) and after the face jumps.
template <int PD, int M, int NQ>
__global__ void __launch_bounds__(256) k_stage_tri(KParams P, const double* __restrict__ in, const double* u,
                                                   const double* w, double* out, double cu, double cw, int rhs_only,
                                                   const double* __restrict__ Tm, double* __restrict__ Tm_out,
                                                   TriPost post) {
  using Sh = TriShape<PD>;
  constexpr int NPT = Sh::NPT, NFP = Sh::NFP, NF = Sh::NF, EPB = Sh::EPB;
  __shared__ double sU[2][EPB][4][NPT], sFr[2][EPB][4][NPT], sGs[2][EPB][4][NPT];
  __shared__ double sJ[EPB][4][NF];
  __shared__ double sDr[NPT * NPT], sDs[NPT * NPT], sLf[NF * NPT], sLift[NPT * NF];
  __shared__ double sO[EPB][4][M][NPT];  // the output, for the filter, the limiter and its traces
  __shared__ TriPostShared<PD, M> sh;
  for (int i = threadIdx.x; i < NPT * NPT; i += 256) {
    sDr[i] = P.tri_Dr[i];
    sDs[i] = P.tri_Ds[i];
  }
  for (int i = threadIdx.x; i < NF * NPT; i += 256) {
    sLf[i] = P.tri_Lf[i];
    sLift[i] = P.tri_lift[i];
  }
  const int E = P.E;
  const int el = threadIdx.x / Sh::TPE;
  const int rem = threadIdx.x % Sh::TPE;
  const int slot = rem >> 2, s = rem & 3;
  const int e = blockIdx.x * EPB + el;
  const bool active = el < EPB && e < E;
  const int le = active ? el : 0;
  const bool pt = active && slot < NPT;
  const bool fp = active && slot < NF;
  const long EN = (long)E * NPT;

  const double* geo = P.tri_geo + (long)(active ? e : 0) * kTriGeo;
  const double rx = geo[kGeoRx], ry = geo[kGeoRy], sx = geo[kGeoSx], sy = geo[kGeoSy], det = geo[kGeoDet];
  const int f = fp ? slot / NFP : 0, kk = fp ? slot % NFP : 0;
  const double fnx = geo[kGeoN0 + 2 * f], fny = geo[kGeoN0 + 2 * f + 1], fsc = geo[kGeoSc0 + f];
  // F . n from the contravariant fluxes: F = x_r Fr + x_s Gs, G = y_r Fr + y_s Gs
  const double fa = det * (fnx * sy - fny * sx), fb = det * (fny * rx - fnx * ry);
  const int nb = fp ? P.tri_nbr[(long)e * 6 + f] : -1;
  const int g = fp ? P.tri_nbr[(long)e * 6 + 3 + f] : 0;

  double uc[M], tn[M], acc[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    uc[k] = pt ? in[((long)s * M + k) * EN + (long)e * NPT + slot] : 0.0;
    tn[k] = (fp && nb >= 0) ? Tm[(((long)nb * NF + g * NFP + (NFP - 1 - kk)) * 4 + s) * M + k] : 0.0;
    acc[k] = 0.0;
  }
  __syncthreads();

  for (int q = 0; q < NQ; ++q) {
    const int b = q & 1;
    // A: nodal value of state s at point `slot`, the four states by quad exchange,
    // physical flux of state s, stored in contravariant form
    double v = 0.0, vr = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double ph = P.tab.PhiT[q * M + k];  // node-major: wide scalar loads
      v += ph * uc[k];
      vr += ph * tn[k];
    }
    double U[4];
    quad_gather(v, U);
    if (pt) {
      const double ir = rcp2(U[0]);
      const double vx = U[1] * ir, vy = U[2] * ir;
      const double p = (P.gamma - 1.0) * (U[3] - 0.5 * (U[1] * vx + U[2] * vy));
      // component s of F and G as A v + B without branching on s (the four variables
      // of a point sit in neighbouring lanes): s = 0: F = m_x, G = m_y; s = 1: A = m_x,
      // B = (p, 0); s = 2: A = m_y, B = (0, p); s = 3: A = E + p, B = 0
      const double A = (s == 0) ? 0.0 : ((s == 3) ? v + p : v);
      const double Bx = (s == 0) ? U[1] : ((s == 1) ? p : 0.0);
      const double By = (s == 0) ? U[2] : ((s == 2) ? p : 0.0);
      const double Fs = A * vx + Bx, Gs = A * vy + By;
      sU[b][le][s][slot] = v;
      sFr[b][le][s][slot] = rx * Fs + ry * Gs;
      sGs[b][le][s][slot] = sx * Fs + sy * Gs;
    }
    __syncthreads();
    // B: own trace and interpolated normal flux at flux point `slot`; both traces
    // of the four states by quad exchange; interactive flux; jump.  The flux
    // divergence at solution point `slot` reads the same contravariant fluxes, so
    // it is formed here too (one LDS read of each flux value per node)
    double ul = 0.0, fr = 0.0, gs = 0.0, d = 0.0;
    if (fp) {
      const int drow = (slot < NPT ? slot : NPT - 1) * NPT;  // flux-only lanes: any row, d unused
#pragma unroll
      for (int j = 0; j < NPT; ++j) {
        const double l = sLf[slot * NPT + j];
        const double Frj = sFr[b][le][s][j], Gsj = sGs[b][le][s][j];
        ul += l * sU[b][le][s][j];
        fr += l * Frj;
        gs += l * Gsj;
        d += sDr[drow + j] * Frj + sDs[drow + j] * Gsj;
      }
    }
    double L[4], R[4];
    quad_gather(ul, L);
    quad_gather(vr, R);
    if (fp) {
      double Rs = vr;
      if (nb < 0) {  // domain boundary: the ghost state
        ghost_n(P, -1 - nb, L, fnx, fny, R);
        Rs = pick4(R, s);
      }
      sJ[le][s][slot] = (flux_n_comp(P.flux, L, R, fnx, fny, P.gamma, s, ul, Rs) - (fa * fr + fb * gs)) * fsc;
    }
    __syncthreads();
    // C: nodal residual of state s at point `slot`, projected onto the chaos
    if (pt) {
      double c = 0.0;
#pragma unroll
      for (int m = 0; m < NF; ++m) c += sLift[slot * NF + m] * sJ[le][s][m];
      const double Rq = -(d + c);
#pragma unroll
      for (int k = 0; k < M; ++k) acc[k] += P.tab.PWT[q * M + k] * Rq;
    }
  }
  const double dt = rhs_only ? 0.0 : *P.dt;
  const bool do_post = post.filter || post.limit;
  // the stages combine with w == in (uc holds it already) and read u only where cu != 0
  const bool w_in = (w == in), need_u = (cu != 0.0);
  if (pt) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const long idx = ((long)s * M + k) * EN + (long)e * NPT + slot;
      const double wv = w_in ? uc[k] : w[idx];
      const double uv = need_u ? u[idx] : 0.0;
      const double o = rhs_only ? acc[k] : cu * uv + cw * (wv + dt * acc[k]);
      acc[k] = o;
      sO[le][s][k][slot] = o;
      if (!do_post) out[idx] = o;
    }
  }
  // the limiter after the stage, or the end-of-step filter and limiter, on the output
  if (do_post) {
    __syncthreads();
    post_tri<PD, M, NQ>(P, acc, sO, sh, e, le, rem, active, post);
    if (pt) {
#pragma unroll
      for (int k = 0; k < M; ++k) out[((long)s * M + k) * EN + (long)e * NPT + slot] = acc[k];
    }
  }
  if (!Tm_out) return;
  // modal traces of the output at the flux points, for the next stage's neighbours
  __syncthreads();
  if (fp) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < NPT; ++j) t += sLf[slot * NPT + j] * sO[le][s][k][j];
      Tm_out[(((long)e * NF + slot) * 4 + s) * M + k] = t;
    }
  }
}

// CFL maximum of a modal state: (|v| + c) / d_e over solution points and nodes
__global__ void __launch_bounds__(256) k_cfl_tri_modal(KParams P, const double* __restrict__ u) {
  __shared__ double sm[256];
  const int np = P.nsp, E = P.E, M = P.M, Nq = P.Nq;
  const long EN = (long)E * np;
  const long t = blockIdx.x * 256l + threadIdx.x;
  double rate = 0.0;
  if (t < EN) {
    const int e = (int)(t / np);
    const double din = P.tri_geo[(long)e * kTriGeo + kGeoDin];
    for (int q = 0; q < Nq; ++q) {
      double U[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double v = 0.0;
        for (int k = 0; k < M; ++k) v += P.tab.Phi[k * Nq + q] * u[((long)s * M + k) * EN + t];
        U[s] = v;
      }
      const double p = euler2_p(U, P.gamma);
      double r = (sqrt(U[1] * U[1] + U[2] * U[2]) / U[0] + sqrt(P.gamma * p / U[0])) / din;
      if (!(r == r)) r = __longlong_as_double(0x7ff0000000000000ll);
      rate = fmax(rate, r);
    }
  }
  sm[threadIdx.x] = rate;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(P.lam_bits, (unsigned long long)__double_as_longlong(sm[0]));
}

// the same for the (M, N_q) pairs of the fused stage: the thread's coefficients stay in registers
template <int M, int NQ>
__global__ void __launch_bounds__(256) k_cfl_tri_mq(KParams P, const double* __restrict__ u) {
  __shared__ double sm[256];
  const int np = P.nsp;
  const long EN = (long)P.E * np;
  const long t = blockIdx.x * 256l + threadIdx.x;
  double rate = 0.0;
  if (t < EN) {
    const double din = P.tri_geo[(t / np) * kTriGeo + kGeoDin];
    double c[4][M];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < M; ++k) c[s][k] = u[((long)s * M + k) * EN + t];
    for (int q = 0; q < NQ; ++q) {
      double U[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) v += P.tab.PhiT[q * M + k] * c[s][k];
        U[s] = v;
      }
      const double p = euler2_p(U, P.gamma);
      double r = (sqrt(U[1] * U[1] + U[2] * U[2]) / U[0] + sqrt(P.gamma * p / U[0])) / din;
      if (!(r == r)) r = __longlong_as_double(0x7ff0000000000000ll);
      rate = fmax(rate, r);
    }
  }
  sm[threadIdx.x] = rate;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(P.lam_bits, (unsigned long long)__double_as_longlong(sm[0]));
}

// the filter and/or limiter in place on a state, as a pass of its own
template <int PD, int M, int NQ>
__global__ void __launch_bounds__(256) k_limit_tri(KParams P, double* __restrict__ u, TriPost post) {
  using Sh = TriShape<PD>;
  constexpr int NPT = Sh::NPT, EPB = Sh::EPB;
  __shared__ double sC[EPB][4][M][NPT];
  __shared__ TriPostShared<PD, M> sh;
  const int E = P.E;
  const int el = threadIdx.x / Sh::TPE;
  const int rem = threadIdx.x % Sh::TPE;
  const int slot = rem >> 2, s = rem & 3;
  const int e = blockIdx.x * EPB + el;
  const bool active = el < EPB && e < E;
  const int le = active ? el : 0;
  const bool pt = active && slot < NPT;
  const long EN = (long)E * NPT;
  double c[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    c[k] = pt ? u[((long)s * M + k) * EN + (long)e * NPT + slot] : 0.0;
    if (pt) sC[le][s][k][slot] = c[k];
  }
  __syncthreads();
  const bool changed = post_tri<PD, M, NQ>(P, c, sC, sh, e, le, rem, active, post);
  if (changed && pt) {
#pragma unroll
    for (int k = 0; k < M; ++k) u[((long)s * M + k) * EN + (long)e * NPT + slot] = c[k];
  }
}

template <int PD, int M, int NQ>
hipError_t go_stage_tri(const KParams& P, const double* in, const double* u, const double* w, double* out, double cu,
                        double cw, int rhs_only, double* Tm, int traces_ready, double* Tm_out, const TriPost& post,
                        hipStream_t s) {
  using Sh = TriShape<PD>;
  if (!traces_ready) {
    const long nt = 4l * M * P.E;
    hipLaunchKernelGGL((k_trace_tri<PD>), dim3(blocks(nt)), dim3(256), 0, s, P, in, Tm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const unsigned grid = (unsigned)((P.E + Sh::EPB - 1) / Sh::EPB);
  hipLaunchKernelGGL((k_stage_tri<PD, M, NQ>), dim3(grid), dim3(256), 0, s, P, in, u, w, out, cu, cw, rhs_only,
                     (const double*)Tm, Tm_out, post);
  return hipGetLastError();
}

template <int PD>
hipError_t dispatch_mq(const KParams& P, const double* in, const double* u, const double* w, double* out, double cu,
                       double cw, int rhs_only, double* Tm, int traces_ready, double* Tm_out, const TriPost& post,
                       hipStream_t s) {
#define FRSG_TRI_MQ(MM, QQ)                                                                                 \
  if (P.M == MM && P.Nq == QQ)                                                                               \
    return go_stage_tri<PD, MM, QQ>(P, in, u, w, out, cu, cw, rhs_only, Tm, traces_ready, Tm_out, post, s);
  FRSG_TRI_MQ(15, 25) FRSG_TRI_MQ(10, 16) FRSG_TRI_MQ(6, 9) FRSG_TRI_MQ(5, 5) FRSG_TRI_MQ(3, 4)
#undef FRSG_TRI_MQ
  return hipErrorInvalidValue;
}

}  // namespace

template <int PD>
hipError_t dispatch_limit(const KParams& P, double* u, const TriPost& post, hipStream_t s) {
  using Sh = TriShape<PD>;
  const unsigned grid = (unsigned)((P.E + Sh::EPB - 1) / Sh::EPB);
#define FRSG_TRI_LIM(MM, QQ)                                                                        \
  if (P.M == MM && P.Nq == QQ) {                                                                     \
    hipLaunchKernelGGL((k_limit_tri<PD, MM, QQ>), dim3(grid), dim3(256), 0, s, P, u, post);              \
    return hipGetLastError();                                                                        \
  }
  FRSG_TRI_LIM(15, 25) FRSG_TRI_LIM(10, 16) FRSG_TRI_LIM(6, 9) FRSG_TRI_LIM(5, 5) FRSG_TRI_LIM(3, 4)
#undef FRSG_TRI_LIM
  return hipErrorInvalidValue;
}

bool tri_fused_supported(const KParams& P) {
  if (P.eq != FRSG_EULER2D || P.nfp < 2 || P.nfp > 5) return false;
  const int mq[5][2] = {{15, 25}, {10, 16}, {6, 9}, {5, 5}, {3, 4}};
  for (auto& x : mq)
    if (P.M == x[0] && P.Nq == x[1]) return true;
  return false;
}

// one stage: out = cu u + cw (w + dt R(in)), or R(in) with rhs_only, the neighbours' traces
// of `in` from Tm (filled by a trace pass first unless traces_ready); with Tm_out the
// traces of `out` are written there for the next stage
hipError_t launch_stage_tri(const KParams& P, const double* in, const double* u, const double* w, double* out,
                            double cu, double cw, int rhs_only, double* Tm, int traces_ready, double* Tm_out,
                            hipStream_t s, const TriPost& post) {
  if (!tri_fused_supported(P) || (post.filter && P.filter == FRSG_FILTER_LASSO) || (rhs_only && (post.filter || post.limit)))
    return hipErrorInvalidValue;
  switch (P.nfp - 1) {
    case 1: return dispatch_mq<1>(P, in, u, w, out, cu, cw, rhs_only, Tm, traces_ready, Tm_out, post, s);
    case 2: return dispatch_mq<2>(P, in, u, w, out, cu, cw, rhs_only, Tm, traces_ready, Tm_out, post, s);
    case 3: return dispatch_mq<3>(P, in, u, w, out, cu, cw, rhs_only, Tm, traces_ready, Tm_out, post, s);
    case 4: return dispatch_mq<4>(P, in, u, w, out, cu, cw, rhs_only, Tm, traces_ready, Tm_out, post, s);
    default: return hipErrorInvalidValue;
  }
}

// the sensor-gated filter and/or the limiter in place with the fused lane layout (the
// fused (p, M, N_q) set)
hipError_t launch_post_tri(const KParams& P, double* u, const TriPost& post, hipStream_t s) {
  if (!tri_fused_supported(P) || (post.filter && P.filter == FRSG_FILTER_LASSO)) return hipErrorInvalidValue;
  switch (P.nfp - 1) {
    case 1: return dispatch_limit<1>(P, u, post, s);
    case 2: return dispatch_limit<2>(P, u, post, s);
    case 3: return dispatch_limit<3>(P, u, post, s);
    case 4: return dispatch_limit<4>(P, u, post, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_limit_tri(const KParams& P, double* u, unsigned char* flags, hipStream_t s) {
  TriPost post;
  post.limit = 1;
  post.flag_lim = flags;
  return launch_post_tri(P, u, post, s);
}

hipError_t launch_cfl_tri_modal(const KParams& P, const double* u, hipStream_t s) {
  if (P.eq != FRSG_EULER2D) return hipErrorInvalidValue;
  const long n = (long)P.E * P.nsp;
#define FRSG_TRI_CFL(MM, QQ)                                                                    \
  if (P.M == MM && P.Nq == QQ) {                                                                 \
    hipLaunchKernelGGL((k_cfl_tri_mq<MM, QQ>), dim3(blocks(n)), dim3(256), 0, s, P, u);          \
    return hipGetLastError();                                                                    \
  }
  FRSG_TRI_CFL(15, 25) FRSG_TRI_CFL(10, 16) FRSG_TRI_CFL(6, 9) FRSG_TRI_CFL(5, 5) FRSG_TRI_CFL(3, 4)
#undef FRSG_TRI_CFL
  hipLaunchKernelGGL(k_cfl_tri_modal, dim3(blocks(n)), dim3(256), 0, s, P, u);
  return hipGetLastError();
}

}  // namespace frsg
