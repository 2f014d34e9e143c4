// Device helpers: physical fluxes, spectral radii, boundary ghosts and the
// Lax-Friedrichs (Rusanov) interface flux (Sec. 3.3), for the conservation
// laws of Sec. 5 (advection, Burgers, 1D/2D Euler with p = (gamma-1)(rho E -
// rho |U|^2 / 2)).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace frsg {

enum : int { kAdvection = FRSG_ADVECTION, kBurgers = FRSG_BURGERS, kEuler1 = FRSG_EULER1D, kEuler2 = FRSG_EULER2D };

template <int EQ>
__host__ __device__ constexpr int nstate() {
  return EQ <= kBurgers ? 1 : (EQ == kEuler1 ? 3 : 4);
}

template <int EQ, typename R>
__device__ __forceinline__ R pressure(const R* U, R gamma) {
  if constexpr (EQ == kEuler1) {
    R kin = R(0.5) * U[1] * U[1] / U[0];
    return (gamma - R(1)) * (U[2] - kin);
  } else {
    R kin = R(0.5) * (U[1] * U[1] + U[2] * U[2]) / U[0];
    return (gamma - R(1)) * (U[3] - kin);
  }
}

// physical flux along direction DIR (0: x, 1: y)
template <int EQ, int DIR, typename R>
__device__ __forceinline__ void flux(const R* U, R* F, R adv, R gamma) {
  if constexpr (EQ == kAdvection) {
    F[0] = adv * U[0];
  } else if constexpr (EQ == kBurgers) {
    F[0] = R(0.5) * U[0] * U[0];
  } else if constexpr (EQ == kEuler1) {
    R v = U[1] / U[0];
    R p = pressure<EQ>(U, gamma);
    F[0] = U[1];
    F[1] = U[1] * v + p;
    F[2] = (U[2] + p) * v;
  } else {
    R p = pressure<EQ>(U, gamma);
    if constexpr (DIR == 0) {
      R vx = U[1] / U[0];
      F[0] = U[1];
      F[1] = U[1] * vx + p;
      F[2] = U[2] * vx;
      F[3] = (U[3] + p) * vx;
    } else {
      R vy = U[2] / U[0];
      F[0] = U[2];
      F[1] = U[1] * vy;
      F[2] = U[2] * vy + p;
      F[3] = (U[3] + p) * vy;
    }
  }
}

// sound speed from gamma p / rho.  In FP32 node loops a pressure that the FP64
// limiter kept at or above its small positive floor can round to a tiny
// negative value (the rounding of the energy exceeds the floor); it counts as
// zero there.  FP64 takes the square root as it is.
template <typename R>
__device__ __forceinline__ R sound_speed(R g_p_over_rho) {
  if constexpr (sizeof(R) == sizeof(float)) return sqrtf(fmaxf(g_p_over_rho, 0.0f));
  else return sqrt(g_p_over_rho);
}

// spectral radius of the flux Jacobian along DIR
template <int EQ, int DIR, typename R>
__device__ __forceinline__ R speed(const R* U, R adv, R gamma) {
  if constexpr (EQ == kAdvection) {
    return fabs(adv);
  } else if constexpr (EQ == kBurgers) {
    return fabs(U[0]);
  } else {
    R p = pressure<EQ>(U, gamma);
    R c = sound_speed(gamma * p / U[0]);
    return fabs(U[1 + DIR] / U[0]) + c;
  }
}

template <int EQ, int DIR, typename R>
__device__ __forceinline__ void rusanov(const R* L, const R* Rt, R* Fs, R adv, R gamma) {
  constexpr int S = nstate<EQ>();
  R fL[S], fR[S];
  flux<EQ, DIR>(L, fL, adv, gamma);
  flux<EQ, DIR>(Rt, fR, adv, gamma);
  R lam = fmax(speed<EQ, DIR>(L, adv, gamma), speed<EQ, DIR>(Rt, adv, gamma));
#pragma unroll
  for (int s = 0; s < S; ++s) Fs[s] = R(0.5) * (fL[s] + fR[s]) - R(0.5) * lam * (Rt[s] - L[s]);
}

// HLL interactive flux (Euler): two waves with Davis's speed estimates bound
// the Riemann fan, one constant state between them conserves it
template <int EQ, int DIR, typename R>
__device__ __forceinline__ void hll(const R* L, const R* Rt, R* Fs, R gamma) {
  constexpr int S = nstate<EQ>();
  R fL[S], fR[S];
  flux<EQ, DIR>(L, fL, R(0), gamma);
  flux<EQ, DIR>(Rt, fR, R(0), gamma);
  const R uL = L[1 + DIR] / L[0], uR = Rt[1 + DIR] / Rt[0];
  const R cL = sound_speed(gamma * pressure<EQ>(L, gamma) / L[0]);
  const R cR = sound_speed(gamma * pressure<EQ>(Rt, gamma) / Rt[0]);
  const R SL = fmin(uL - cL, uR - cR), SR = fmax(uL + cL, uR + cR);
#pragma unroll
  for (int s = 0; s < S; ++s)
    Fs[s] = (SL >= R(0)) ? fL[s]
          : (SR <= R(0)) ? fR[s]
                         : (SR * fL[s] - SL * fR[s] + (SL * SR) * (Rt[s] - L[s])) / (SR - SL);
}

// the configured interactive flux (Sec. 3.3): Lax-Friedrichs, or HLL for Euler
template <int EQ, int DIR, typename R>
__device__ __forceinline__ void interface_flux(int kind, const R* L, const R* Rt, R* Fs, R adv, R gamma) {
  if constexpr (EQ == kEuler1 || EQ == kEuler2) {
    if (kind == FRSG_FLUX_HLL) {
      hll<EQ, DIR>(L, Rt, Fs, gamma);
      return;
    }
  }
  rusanov<EQ, DIR>(L, Rt, Fs, adv, gamma);
}

// ghost trace outside boundary `side` (0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi)
template <int EQ, typename R>
__device__ __forceinline__ void ghost(const KParams& P, int side, const R* in, R* out) {
  constexpr int S = nstate<EQ>();
  const int kind = P.bc[side];
#pragma unroll
  for (int s = 0; s < S; ++s) out[s] = (kind == FRSG_BC_DIRICHLET) ? R(P.bc_state[side][s]) : in[s];
  if (kind == FRSG_BC_REFLECT && S > 1) {
    const int nrm = side < 2 ? 1 : 2;
    out[nrm] = -out[nrm];
  }
}

// root in (0, 1) of p(beta (u* - u_bar) + u_bar) = eps, Sec. 4.3; the
// quadratic rho (E - eps/(gamma-1)) - |m|^2 / 2 = 0 along the segment, solved in
// cancellation-free form.
template <int EQ>
__device__ __forceinline__ double pressure_root(const double* ub, const double* us, double eps, double gamma) {
  constexpr int S = nstate<EQ>();
  const double ep = eps / (gamma - 1.0);
  double d[S];
#pragma unroll
  for (int s = 0; s < S; ++s) d[s] = us[s] - ub[s];
  double dmm = 0.0, mbdm = 0.0, mbmb = 0.0;
#pragma unroll
  for (int s = 1; s < S - 1; ++s) {
    dmm += d[s] * d[s];
    mbdm += ub[s] * d[s];
    mbmb += ub[s] * ub[s];
  }
  const double a = d[S - 1] * d[0] - 0.5 * dmm;
  const double b = d[S - 1] * ub[0] + (ub[S - 1] - ep) * d[0] - mbdm;
  const double c = (ub[S - 1] - ep) * ub[0] - 0.5 * mbmb;
  const double disc = fmax(b * b - 4.0 * a * c, 0.0);
  const double sq = sqrt(disc);
  return (b < 0.0) ? 2.0 * c / (-b + sq) : (-b - sq) / (2.0 * a);
}

// block-wide reductions over blockDim.x <= 256 threads (shared scratch of 256 doubles)
__device__ __forceinline__ double block_reduce_min(double v, double* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  double r = sm[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_reduce_sum(double v, double* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = sm[threadIdx.x] + sm[threadIdx.x + o];
    __syncthreads();
  }
  double r = sm[0];
  __syncthreads();
  return r;
}

}  // namespace frsg
