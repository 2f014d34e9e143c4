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

}  // namespace frsg
