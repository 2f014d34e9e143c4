// Device helpers shared by the quadrilateral 2D Euler stage kernels: lane
// exchanges inside a 16-lane row that holds the 4 x 4 solution points of an
// element (lane r = a + 4 b), reciprocal and square root in the node loop's
// type, the Lax-Friedrichs and HLL interactive fluxes (Sec. 3.3), LDS record
// types, and raw buffer access to state arrays.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace frsg {
namespace quad {

constexpr int NP = 4;
constexpr int NSP = 16;

// ---------------------------------------------------------------------------
// lane exchange within an element row of 16 lanes, lane r = a + 4 b
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  // all lanes active and every source lane inside the row: bound_ctrl lets the
  // move skip the old-value operand
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

// 1/x to the accuracy of the type: hardware estimate refined by Newton steps
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
// FP32: a pressure the FP64 limiter kept at its small positive floor can round
// below zero in FP32 arithmetic; under a square root it counts as zero
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(fmaxf(x, 0.0f)); }

// value at point ((a + k) & 3, b)
template <int K, typename T>
__device__ __forceinline__ T xrot(T v) {
  if constexpr (K == 0) return v;
  else if constexpr (K == 1) return dpp<0x39>(v);
  else if constexpr (K == 2) return dpp<0x4E>(v);
  else return dpp<0x93>(v);
}
// value at point (a, (b - k) & 3)
template <int K, typename T>
__device__ __forceinline__ T yrot(T v) {
  if constexpr (K == 0) return v;
  else return dpp<0x120 + 4 * K>(v);
}

// sum_c w[c] v(c, b) with wx[k] = w[(a + k) & 3]
template <typename T>
__device__ __forceinline__ T xdot(const T* wx, T v) {
  return wx[0] * v + wx[1] * xrot<1>(v) + wx[2] * xrot<2>(v) + wx[3] * xrot<3>(v);
}
// sum_c w[c] v(a, c) with wy[k] = w[(b - k) & 3]
template <typename T>
__device__ __forceinline__ T ydot(const T* wy, T v) {
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

// Lax-Friedrichs flux of the 2D Euler equations along direction dir (0: x, 1: y)
// between the own trace and the neighbour's; the neighbour is the left state
// when nb_left.  f(L) + f(R) and the jump are formed so that the result does not
// depend on which side computes it.
template <typename T>
__device__ __forceinline__ void rusanov_e2(const T* own, const T* nb, bool nb_left, T* Fs, T g, int dir) {
  T fo[4], fn[4], so, sn;
  auto side = [&](const T* U, T* f, T& sp) {
    const T ir = recip(U[0]);
    const T un = dir == 0 ? U[1] : U[2];
    const T p = (g - T(1)) * (U[3] - T(0.5) * (U[1] * U[1] + U[2] * U[2]) * ir);
    const T vn = un * ir;
    f[0] = un;
    f[1] = U[1] * vn + (dir == 0 ? p : T(0));
    f[2] = U[2] * vn + (dir == 0 ? T(0) : p);
    f[3] = (U[3] + p) * vn;
    sp = fabs(vn) + sqrt_t(g * p * ir);
  };
  side(own, fo, so);
  side(nb, fn, sn);
  // 0.5 (f(L) + f(R)) - 0.5 lam (R - L), with R - L = +-(nb - own)
  const T hl = nb_left ? T(-0.5) * fmax(so, sn) : T(0.5) * fmax(so, sn);
#pragma unroll
  for (int s = 0; s < 4; ++s) Fs[s] = T(0.5) * (fo[s] + fn[s]) - hl * (nb[s] - own[s]);
}

// HLL flux of the 2D Euler equations along direction dir between the own trace
// and the neighbour's (the left state when nb_left): Davis's wave speeds
// S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).  Both
// elements of a face pass the same left and right states, so they get the
// same result.
template <typename T>
__device__ __forceinline__ void hll_e2(const T* own, const T* nb, bool nb_left, T* Fs, T g, int dir) {
  T Lv[4], Rv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    Lv[s] = nb_left ? nb[s] : own[s];
    Rv[s] = nb_left ? own[s] : nb[s];
  }
  T fL[4], fR[4], uL, uR, cL, cR;
  auto side = [&](const T* U, T* f, T& un, T& c) {
    const T ir = recip(U[0]);
    const T mn = dir == 0 ? U[1] : U[2];
    const T p = (g - T(1)) * (U[3] - T(0.5) * (U[1] * U[1] + U[2] * U[2]) * ir);
    const T vn = mn * ir;
    f[0] = mn;
    f[1] = U[1] * vn + (dir == 0 ? p : T(0));
    f[2] = U[2] * vn + (dir == 0 ? T(0) : p);
    f[3] = (U[3] + p) * vn;
    un = vn;
    c = sqrt_t(g * p * ir);
  };
  side(Lv, fL, uL, cL);
  side(Rv, fR, uR, cR);
  const T SL = fmin(uL - cL, uR - cR), SR = fmax(uL + cL, uR + cR);
  const T iw = recip(SR - SL);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const T mid = (SR * fL[s] - SL * fR[s] + (SL * SR) * (Rv[s] - Lv[s])) * iw;
    Fs[s] = (SL >= T(0)) ? fL[s] : (SR <= T(0)) ? fR[s] : mid;
  }
}

// the four conserved variables at one point, stored with one or two LDS accesses
template <typename T>
struct alignas(4 * sizeof(T) > 16 ? 16 : 4 * sizeof(T)) Quad4 {
  T v[4];
};
// two of the four conserved variables at one point: the nodal values, traces
// and interface fluxes of an element are kept as two planes (variables 0-1,
// variables 2-3) so that 16 consecutive points fill whole rows of LDS banks
template <typename T>
struct alignas(2 * sizeof(T)) Half2 {
  T x, y;
};

// Raw buffer access to a state array: one lane offset (VGPR) plus a uniform
// offset per (variable, mode) (SGPR), so no per-coefficient address has to be
// kept in registers.  Out-of-range offsets read 0 and drop stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const double* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, (int)bytes, 0x00020000);
}
// Cache policy: the stage states are streamed (each coefficient is read once by a
// launch and written once), so their loads and every store carry the non-temporal
// hint and leave the L2 to the data that is reused within a launch (the neighbours'
// face traces, the tables); measured 5 % off the FP64 shock-vortex step.
constexpr int kNonTemporal = 2;  // the nt bit of the buffer instructions' cache-policy operand
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ double bload_stream(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kNonTemporal));
}
// stores that the L2 should combine: pieces of a line written by several instructions
__device__ __forceinline__ void bstore_cached(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, kNonTemporal);
}

}  // namespace quad
}  // namespace frsg
