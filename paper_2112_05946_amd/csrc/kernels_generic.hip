// Generic FP64 FR-SG kernels: any equation, FR degree 1..7, any gPC order and
// quadrature size.  One pass per stage:
//
//   nodal     gPC expansion at the random nodes, every solution point (Sec. 2.1
//             Eq. polynomial chaos), physical flux there (Eq. local direct flux);
//             optionally the CFL maximum of the wave speed;
//   faces     traces at the flux points by Lagrange interpolation (Sec. 3.2),
//             Lax-Friedrichs flux per node (Sec. 3.3), minus the interpolated
//             discontinuous flux, stored per element side;
//   resid     nodal total-flux derivative with the Radau corrections (Sec. 3.4,
//             Sec. 3.5 tensor extension), du/dt = -(1/J) df/dr (Eq. fr update);
//   project   Galerkin projection onto the chaos (Eq. discrete expectation value)
//             and the SSP-RK3 stage combination.
//
// Because the projection is linear and acts only on the node index, the
// residual is assembled per node and projected once, instead of projecting the
// flux, the interface flux and the interpolated flux separately; the result is
// the same up to rounding.
//
// Element-wise passes: positivity-preserving limiter (Sec. 4.3) and
// sensor-gated modal filter (Sec. 4.1, 4.2).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace frsg {
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(long n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

// ---------------------------------------------------------------------------
// scalars
// ---------------------------------------------------------------------------
__global__ void k_set_scalars(KParams P, double dt_fixed) {
  *P.lam_bits = 0ull;
  if (dt_fixed > 0.0) *P.dt = dt_fixed;
}

template <int DIM>
__global__ void k_dt(KParams P, double* dt_used) {
  const double lam = __longlong_as_double((long long)*P.lam_bits);
  double dt;
  if (DIM == 1)
    dt = P.cfl * P.dx / (P.np1 * lam);
  else
    dt = P.cfl / (P.np1 * lam);
  if (!(dt > 0.0) || !isfinite(dt)) atomicOr(P.status, kStatusNonFinite);
  *P.dt = dt;
  if (dt_used) *dt_used = dt;
}

__global__ void k_copy_dt(KParams P, double* dt_used) { *dt_used = *P.dt; }

__global__ void k_fill_flags(unsigned char* f, long n) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) f[t] = 0;
}

// ---------------------------------------------------------------------------
// nodal values and fluxes at (node q, element e, solution point j)
// ---------------------------------------------------------------------------
template <int EQ, int DIM>
__global__ void __launch_bounds__(kBlock) k_nodal(KParams P, const double* __restrict__ u, double* __restrict__ Un,
                                                  double* __restrict__ Fn, double* __restrict__ Gn, int do_cfl) {
  constexpr int S = nstate<EQ>();
  __shared__ double sm[kBlock];
  const long EN = (long)P.E * P.nsp;
  const long total = (long)P.Nq * EN;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  double rate = 0.0;
  if (t < total) {
    const int q = (int)(t / EN);
    const long ej = t - (long)q * EN;
    double U[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      for (int k = 0; k < P.M; ++k) acc += u[((long)s * P.M + k) * EN + ej] * P.tab.Phi[k * P.Nq + q];
      U[s] = acc;
    }
    double F[S];
    flux<EQ, 0>(U, F, P.adv, P.gamma);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      Un[(long)s * total + t] = U[s];
      Fn[(long)s * total + t] = F[s];
    }
    if constexpr (DIM == 2) {
      double G[S];
      flux<EQ, 1>(U, G, P.adv, P.gamma);
#pragma unroll
      for (int s = 0; s < S; ++s) Gn[(long)s * total + t] = G[s];
    }
    if (do_cfl) {
      if constexpr (DIM == 1)
        rate = speed<EQ, 0>(U, P.adv, P.gamma);
      else
        rate = speed<EQ, 0>(U, P.adv, P.gamma) / P.dx + speed<EQ, 1>(U, P.adv, P.gamma) / P.dy;
      if (!(rate == rate)) rate = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf, dt -> 0
    }
  }
  if (do_cfl) {
    // max is exact, so the reduction order does not matter
    sm[threadIdx.x] = rate;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(P.lam_bits, (unsigned long long)__double_as_longlong(sm[0]));
  }
}

// ---------------------------------------------------------------------------
// interface fluxes
// ---------------------------------------------------------------------------
// 1D: face f in [0, E] between element f-1 (its r=+1 trace) and f (its r=-1 trace)
template <int EQ>
__global__ void __launch_bounds__(kBlock) k_faces_1d(KParams P, const double* __restrict__ Un,
                                                     const double* __restrict__ Fn, double* __restrict__ Corr) {
  constexpr int S = nstate<EQ>();
  const int E = P.E, n = P.np1, Nq = P.Nq;
  const long total = (long)(E + 1) * Nq;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  if (t >= total) return;
  const int f = (int)(t % (E + 1));
  const int q = (int)(t / (E + 1));
  const bool periodic = P.bc[0] == FRSG_BC_PERIODIC;
  auto trace = [&](const double* src, int e, const double* l, double* out) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      const double* p = src + (((long)s * Nq + q) * E + e) * n;
      for (int j = 0; j < n; ++j) acc += l[j] * p[j];
      out[s] = acc;
    }
  };
  double UL[S], UR[S], tmp[S];
  if (f == 0) {
    if (periodic) {
      trace(Un, E - 1, P.tab.lR, UL);
    } else {
      trace(Un, 0, P.tab.lL, tmp);
      ghost<EQ>(P, 0, tmp, UL);
    }
  } else {
    trace(Un, f - 1, P.tab.lR, UL);
  }
  if (f == E) {
    if (periodic) {
      trace(Un, 0, P.tab.lL, UR);
    } else {
      trace(Un, E - 1, P.tab.lR, tmp);
      ghost<EQ>(P, 1, tmp, UR);
    }
  } else {
    trace(Un, f, P.tab.lL, UR);
  }
  double Fs[S];
  interface_flux<EQ, 0>(P.flux, UL, UR, Fs, P.adv, P.gamma);
  if (f >= 1) {
    trace(Fn, f - 1, P.tab.lR, tmp);
#pragma unroll
    for (int s = 0; s < S; ++s) Corr[(((long)s * Nq + q) * E + (f - 1)) * 2 + 1] = Fs[s] - tmp[s];
  }
  if (f <= E - 1) {
    trace(Fn, f, P.tab.lL, tmp);
#pragma unroll
    for (int s = 0; s < S; ++s) Corr[(((long)s * Nq + q) * E + f) * 2 + 0] = Fs[s] - tmp[s];
  }
}

// 2D: DIR 0 = x-faces (fx in [0, nx], row iy, flux point b),
//     DIR 1 = y-faces (fy in [0, ny], column ix, flux point a).
// Corr[s][q][e][side * n + fp], sides 0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi.
template <int EQ, int DIR>
__global__ void __launch_bounds__(kBlock) k_faces_2d(KParams P, const double* __restrict__ Un,
                                                     const double* __restrict__ Fn, double* __restrict__ Corr) {
  constexpr int S = 4;
  const int n = P.np1, Nq = P.Nq, nx = P.nx, ny = P.ny, E = P.E, nsp = P.nsp;
  const int nfaces = DIR == 0 ? (nx + 1) : (ny + 1);
  const int nlines = DIR == 0 ? ny : nx;
  const long total = (long)Nq * nlines * nfaces * n;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  if (t >= total) return;
  const int fp = (int)(t % n);
  long r = t / n;
  const int f = (int)(r % nfaces);
  r /= nfaces;
  const int line = (int)(r % nlines);
  const int q = (int)(r / nlines);
  const int lo_side = DIR == 0 ? 0 : 2, hi_side = DIR == 0 ? 1 : 3;
  const bool periodic = P.bc[lo_side] == FRSG_BC_PERIODIC;
  const int ncell = DIR == 0 ? nx : ny;
  auto elem = [&](int c) { return DIR == 0 ? (line * nx + c) : (c * nx + line); };
  // trace of element e along DIR at r = +-1 (l = lL or lR), at flux point fp
  auto trace = [&](const double* src, int e, const double* l, double* out) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      const double* p = src + (((long)s * Nq + q) * E + e) * nsp;
      for (int i = 0; i < n; ++i) acc += l[i] * p[DIR == 0 ? (i + n * fp) : (fp + n * i)];
      out[s] = acc;
    }
  };
  double UL[S], UR[S], tmp[S];
  if (f == 0) {
    if (periodic) {
      trace(Un, elem(ncell - 1), P.tab.lR, UL);
    } else {
      trace(Un, elem(0), P.tab.lL, tmp);
      ghost<EQ>(P, lo_side, tmp, UL);
    }
  } else {
    trace(Un, elem(f - 1), P.tab.lR, UL);
  }
  if (f == ncell) {
    if (periodic) {
      trace(Un, elem(0), P.tab.lL, UR);
    } else {
      trace(Un, elem(ncell - 1), P.tab.lR, tmp);
      ghost<EQ>(P, hi_side, tmp, UR);
    }
  } else {
    trace(Un, elem(f), P.tab.lL, UR);
  }
  double Fs[S];
  interface_flux<EQ, DIR>(P.flux, UL, UR, Fs, P.adv, P.gamma);
  const int nface_slots = 4 * n;
  if (f >= 1) {
    const int e = elem(f - 1);
    trace(Fn, e, P.tab.lR, tmp);
#pragma unroll
    for (int s = 0; s < S; ++s) Corr[(((long)s * Nq + q) * E + e) * nface_slots + hi_side * n + fp] = Fs[s] - tmp[s];
  }
  if (f <= ncell - 1) {
    const int e = elem(f);
    trace(Fn, e, P.tab.lL, tmp);
#pragma unroll
    for (int s = 0; s < S; ++s) Corr[(((long)s * Nq + q) * E + e) * nface_slots + lo_side * n + fp] = Fs[s] - tmp[s];
  }
}

// ---------------------------------------------------------------------------
// nodal residual at (q, e, j)
// ---------------------------------------------------------------------------
template <int EQ, int DIM>
__global__ void __launch_bounds__(kBlock) k_resid(KParams P, const double* __restrict__ Fn,
                                                  const double* __restrict__ Gn, const double* __restrict__ Corr,
                                                  double* __restrict__ Rn) {
  constexpr int S = nstate<EQ>();
  const int n = P.np1, nsp = P.nsp;
  const long EN = (long)P.E * nsp;
  const long total = (long)P.Nq * EN;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  if (t >= total) return;
  const long qe = t / nsp;  // q * E + e
  const int j = (int)(t - qe * nsp);
  const double* D = P.tab.D;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const long base = (long)s * total + qe * nsp;
    if constexpr (DIM == 1) {
      double acc = 0.0;
      for (int l = 0; l < n; ++l) acc += D[j * n + l] * Fn[base + l];
      const double* C = Corr + ((long)s * total / nsp + qe) * 2;
      acc = acc + C[0] * P.tab.dhL[j] + C[1] * P.tab.dhR[j];
      Rn[base + j] = -acc / P.Jx;
    } else {
      const int a = j % n, b = j / n;
      double ax = 0.0, ay = 0.0;
      for (int c = 0; c < n; ++c) ax += D[a * n + c] * Fn[base + c + n * b];
      for (int c = 0; c < n; ++c) ay += D[b * n + c] * Gn[base + a + n * c];
      const double* C = Corr + ((long)s * (total / nsp) + qe) * (4 * n);
      ax = ax + C[0 * n + b] * P.tab.dhL[a] + C[1 * n + b] * P.tab.dhR[a];
      ay = ay + C[2 * n + a] * P.tab.dhL[b] + C[3 * n + a] * P.tab.dhR[b];
      Rn[base + j] = -ax / P.Jx - ay / P.Jy;
    }
  }
}

// ---------------------------------------------------------------------------
// projection and stage combination at (k, e, j)
// ---------------------------------------------------------------------------
template <int EQ>
__global__ void __launch_bounds__(kBlock) k_project(KParams P, const double* __restrict__ Rn,
                                                    const double* __restrict__ u, const double* __restrict__ w,
                                                    double* out, double cu, double cw, int rhs_only) {
  constexpr int S = nstate<EQ>();
  const long EN = (long)P.E * P.nsp;
  const long total = (long)P.M * EN;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  if (t >= total) return;
  const int k = (int)(t / EN);
  const long ej = t - (long)k * EN;
  const long ntot = (long)P.Nq * EN;
  const double dt = rhs_only ? 0.0 : *P.dt;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double acc = 0.0;
    const double* R = Rn + (long)s * ntot + ej;
    for (int q = 0; q < P.Nq; ++q) acc += P.tab.PW[k * P.Nq + q] * R[(long)q * EN];
    const long idx = ((long)s * P.M + k) * EN + ej;
    if (rhs_only)
      out[idx] = acc;
    else
      out[idx] = cu * u[idx] + cw * (w[idx] + dt * acc);
  }
}

template <int EQ>
__global__ void __launch_bounds__(kBlock) k_project_ic(KParams P, const double* __restrict__ U0,
                                                       double* __restrict__ out) {
  constexpr int S = nstate<EQ>();
  const long EN = (long)P.E * P.nsp;
  const long total = (long)P.M * EN;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  if (t >= total) return;
  const int k = (int)(t / EN);
  const long ej = t - (long)k * EN;
  const long ntot = (long)P.Nq * EN;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double acc = 0.0;
    for (int q = 0; q < P.Nq; ++q) acc += P.tab.PW[k * P.Nq + q] * U0[(long)s * ntot + (long)q * EN + ej];
    out[((long)s * P.M + k) * EN + ej] = acc;
  }
}

// ---------------------------------------------------------------------------
// positivity-preserving limiter, one block per element (Sec. 4.3)
// ---------------------------------------------------------------------------
constexpr int kElemBlock = 128;

// The element's coefficients c(s, k, j) = C[(s * M + k) * cs + j]: staged in LDS
// (cs = nsp) when they fit, else read in place from the state (cs = E * nsp).
// nodal state at limiter point `pt` (solution points first, then face points)
template <int EQ, int DIM>
__device__ __forceinline__ void limiter_point(const KParams& P, const double* C, long cs, int pt, int q, double* U) {
  constexpr int S = nstate<EQ>();
  const int n = P.np1, nsp = P.nsp, M = P.M, Nq = P.Nq;
  auto at_sp = [&](int s, int j) {
    double acc = 0.0;
    for (int k = 0; k < M; ++k) acc += C[((long)s * M + k) * cs + j] * P.tab.Phi[k * Nq + q];
    return acc;
  };
  if (pt < nsp) {
#pragma unroll
    for (int s = 0; s < S; ++s) U[s] = at_sp(s, pt);
    return;
  }
  const int f = pt - nsp;
  if constexpr (DIM == 3) {
    // triangle flux point f: interpolation row of the face table
    const double* l = P.tri_Lf + (long)f * nsp;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      for (int j = 0; j < nsp; ++j) acc += l[j] * at_sp(s, j);
      U[s] = acc;
    }
  } else if constexpr (DIM == 1) {
    const double* l = (f == 0) ? P.tab.lL : P.tab.lR;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += l[j] * at_sp(s, j);
      U[s] = acc;
    }
  } else {
    const int side = f / n, i = f % n;
    const double* l = (side == 0 || side == 2) ? P.tab.lL : P.tab.lR;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      for (int c = 0; c < n; ++c) acc += l[c] * at_sp(s, side < 2 ? (c + n * i) : (i + n * c));
      U[s] = acc;
    }
  }
}

template <int EQ, int DIM>
__global__ void __launch_bounds__(kElemBlock) k_limiter(KParams P, double* __restrict__ u,
                                                        unsigned char* __restrict__ flags, int staged) {
  constexpr int S = nstate<EQ>();
  extern __shared__ double sc[];  // [S][M][nsp] when staged
  __shared__ double sm[kElemBlock];
  const int e = blockIdx.x;
  const int nsp = P.nsp, M = P.M, Nq = P.Nq;
  const long EN = (long)P.E * nsp;
  if (staged) {
    for (int it = threadIdx.x; it < S * M * nsp; it += kElemBlock) {
      const int sk = it / nsp, j = it - sk * nsp;
      sc[it] = u[(long)sk * EN + (long)e * nsp + j];
    }
    __syncthreads();
  }
  const double* C = staged ? sc : u + (long)e * nsp;
  const long cs = staged ? nsp : EN;
  double ub[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double acc = 0.0;
    for (int j = 0; j < nsp; ++j) acc += C[((long)s * M) * cs + j] * P.tab.swts[j];
    ub[s] = acc;
  }
  const double pb = pressure<EQ>(ub, P.gamma);
  bool finite = true;
#pragma unroll
  for (int s = 0; s < S; ++s) finite = finite && isfinite(ub[s]);
  if (!(ub[0] > 0.0 && pb > 0.0 && finite)) {
    if (threadIdx.x == 0) {
      atomicOr(P.status, kStatusNotRealizable);
      if (flags) flags[e] = 0;
    }
    return;
  }
  const double eps = fmin(1e-8, fmin(ub[0], pb));
  const int nfp = DIM == 1 ? 2 : (DIM == 2 ? 4 * P.np1 : 3 * P.nfp);
  const int items = (nsp + nfp) * Nq;

  // Decision from rigorous bounds first: at point pt the value at any node is
  // a_0 + sum_{k>=1} a_k Phi_k(z_q), a_k the interpolated mode k, |Phi_k(z_q)|
  // <= cmax_k.  If density and pressure bounds clear eps (with a relative
  // margin for the rounding of the bounds) at every point, the node-by-node
  // minimum clears it too and the element is left unchanged.
  {
    const int n = P.np1;
    double safe = 1.0;
    for (int pt = threadIdx.x; pt < nsp + nfp; pt += kElemBlock) {
      double mn[S], vr[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        double mean = 0.0, var = 0.0;
        for (int k = 0; k < M; ++k) {
          const double* ck = C + ((long)s * M + k) * cs;
          double a;
          if (pt < nsp) {
            a = ck[pt];
          } else {
            const int f = pt - nsp;
            a = 0.0;
            if constexpr (DIM == 3) {
              const double* l = P.tri_Lf + (long)f * nsp;
              for (int j = 0; j < nsp; ++j) a += l[j] * ck[j];
            } else if constexpr (DIM == 1) {
              const double* l = (f == 0) ? P.tab.lL : P.tab.lR;
              for (int j = 0; j < n; ++j) a += l[j] * ck[j];
            } else {
              const int side = f / n, i = f % n;
              const double* l = (side == 0 || side == 2) ? P.tab.lL : P.tab.lR;
              for (int c = 0; c < n; ++c) a += l[c] * ck[side < 2 ? (c + n * i) : (i + n * c)];
            }
          }
          if (k == 0)
            mean = a;
          else
            var += fabs(a) * P.tab.cmax[k];
        }
        mn[s] = mean;
        vr[s] = var;
      }
      const double rlo = mn[0] - vr[0];
      const double tol_r = 1e-10 * (fabs(mn[0]) + vr[0]);
      bool ok = rlo > eps + tol_r;
      if (ok) {
        double m2 = 0.0, ke = 0.0;
#pragma unroll
        for (int s = 1; s < S - 1; ++s) {
          const double mx = fabs(mn[s]) + vr[s];
          m2 += mx * mx;
        }
        ke = 0.5 * m2 / rlo;
        const double elo = mn[S - 1] - vr[S - 1];
        const double plo = (P.gamma - 1.0) * (elo - ke);
        const double tol_p = 1e-10 * (P.gamma - 1.0) * (fabs(mn[S - 1]) + vr[S - 1] + ke);
        ok = plo > eps + tol_p;
      }
      if (!ok) safe = 0.0;
    }
    if (block_reduce_min(safe, sm) > 0.5) {
      if (threadIdx.x == 0 && flags) flags[e] = 0;
      return;
    }
  }
  // node-by-node test: the solution-point values at every node first go to an
  // LDS table (all threads busy), face values interpolate from it
  double* sN = sc + S * M * nsp;  // [S][nsp][Nq] when staged == 2
  if (staged == 2) {
    for (int it = threadIdx.x; it < S * nsp * Nq; it += kElemBlock) {
      const int s = it / (nsp * Nq), rem = it - s * nsp * Nq;
      const int j = rem / Nq, q = rem - j * Nq;
      double acc = 0.0;
      for (int k = 0; k < M; ++k) acc += C[((long)s * M + k) * cs + j] * P.tab.Phi[k * Nq + q];
      sN[it] = acc;
    }
    __syncthreads();
  }
  auto point = [&](int pt, int q, double* U) {
    if (staged != 2) {
      limiter_point<EQ, DIM>(P, C, cs, pt, q, U);
      return;
    }
    const int n = P.np1;
    if (pt < nsp) {
#pragma unroll
      for (int s = 0; s < S; ++s) U[s] = sN[((long)s * nsp + pt) * Nq + q];
      return;
    }
    const int f = pt - nsp;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      if constexpr (DIM == 3) {
        const double* l = P.tri_Lf + (long)f * nsp;
        for (int j = 0; j < nsp; ++j) acc += l[j] * sN[((long)s * nsp + j) * Nq + q];
      } else if constexpr (DIM == 1) {
        const double* l = (f == 0) ? P.tab.lL : P.tab.lR;
        for (int j = 0; j < n; ++j) acc += l[j] * sN[((long)s * nsp + j) * Nq + q];
      } else {
        const int side = f / n, i = f % n;
        const double* l = (side == 0 || side == 2) ? P.tab.lL : P.tab.lR;
        for (int c = 0; c < n; ++c) acc += l[c] * sN[((long)s * nsp + (side < 2 ? (c + n * i) : (i + n * c))) * Nq + q];
      }
      U[s] = acc;
    }
  };
  double rmin = INFINITY, pmin = INFINITY;
  for (int it = threadIdx.x; it < items; it += kElemBlock) {
    double U[S];
    point(it / Nq, it % Nq, U);
    rmin = fmin(rmin, U[0]);
    pmin = fmin(pmin, pressure<EQ>(U, P.gamma));
  }
  rmin = block_reduce_min(rmin, sm);
  pmin = block_reduce_min(pmin, sm);
  if (!(fmin(rmin, pmin) < eps)) {
    if (threadIdx.x == 0 && flags) flags[e] = 0;
    return;
  }
  const double beta1 = (rmin >= eps) ? 1.0 : (ub[0] - eps) / (ub[0] - rmin);
  double bmin = 1.0;
  for (int it = threadIdx.x; it < items; it += kElemBlock) {
    double U[S];
    point(it / Nq, it % Nq, U);
    U[0] = beta1 * (U[0] - ub[0]) + ub[0];
    if (pressure<EQ>(U, P.gamma) < eps) bmin = fmin(bmin, pressure_root<EQ>(ub, U, eps, P.gamma));
  }
  const double beta2 = block_reduce_min(bmin, sm);
  // all threads have read u; update the modal coefficients in place
  for (int it = threadIdx.x; it < S * M * nsp; it += kElemBlock) {
    const int j = it % nsp;
    const int k = (it / nsp) % M;
    const int s = it / (nsp * M);
    const long idx = ((long)s * M + k) * EN + (long)e * nsp + j;
    const double m0 = (k == 0) ? 1.0 : 0.0;
    double v = staged ? sc[it] : u[idx];
    if (s == 0) v = beta1 * (v - ub[0] * m0) + ub[0] * m0;
    v = beta2 * (v - ub[s] * m0) + ub[s] * m0;
    u[idx] = v;
  }
  if (threadIdx.x == 0 && flags) flags[e] = 1;
}

// ---------------------------------------------------------------------------
// sensor + filter, one block per element (Sec. 4.1, 4.2)
// ---------------------------------------------------------------------------
template <int EQ, int DIM>
__global__ void __launch_bounds__(kElemBlock) k_sensor_filter(KParams P, double* __restrict__ u,
                                                              unsigned char* __restrict__ flags) {
  constexpr int S = nstate<EQ>();
  extern __shared__ double ut[];  // [S][M][nsp] spatial modal coefficients
  __shared__ double sm[kElemBlock];
  const int e = blockIdx.x;
  const int n = P.np1, nsp = P.nsp, M = P.M;
  const long EN = (long)P.E * nsp;
  const double* Vinv = P.tab.Vinv;
  const double* V = P.tab.V;
  for (int it = threadIdx.x; it < S * M * nsp; it += kElemBlock) {
    const int m = it % nsp;
    const int sk = it / nsp;
    const double* src = u + (long)sk * EN + (long)e * nsp;
    double acc = 0.0;
    if constexpr (DIM == 3) {
      for (int l = 0; l < nsp; ++l) acc += P.tri_Vinv[m * nsp + l] * src[l];
    } else if constexpr (DIM == 1) {
      for (int l = 0; l < n; ++l) acc += Vinv[m * n + l] * src[l];
    } else {
      const int ma = m % n, mb = m / n;
      for (int d = 0; d < n; ++d) {
        double row = 0.0;
        for (int c = 0; c < n; ++c) row += Vinv[ma * n + c] * src[c + n * d];
        acc += Vinv[mb * n + d] * row;
      }
    }
    ut[it] = acc;
  }
  __syncthreads();
  bool flag = true;
  if (P.sensor == FRSG_SENSOR_DETECTOR) {
    double num = 0.0, den = 0.0;
    for (int it = threadIdx.x; it < M * nsp; it += kElemBlock) {
      const double e2 = ut[it] * ut[it];
      num += e2 * P.tab.shell[it];
      den += e2;
    }
    num = block_reduce_sum(num, sm);
    den = block_reduce_sum(den, sm);
    flag = (den > 0.0) && (num / den > P.sensor_thr);
  }
  if (!flag) {
    if (threadIdx.x == 0 && flags) flags[e] = 0;
    return;
  }
  const double dt = *P.dt;
  for (int it = threadIdx.x; it < S * M * nsp; it += kElemBlock) {
    const int j = it % nsp;
    const int sk = it / nsp;
    const int k = sk % M;
    const double* src = ut + (long)sk * nsp;
    auto lam = [&](int m) {
      const double f = P.tab.filt[k * nsp + m];
      if (P.filter == FRSG_FILTER_LASSO) {
        // Eq. LassoFilterFunction with the strengths of Eq. fStrength (one
        // physical and one random dimension); f = ||Psi_m Phi_k||_1
        const int s = sk / M;
        const double a1 = fabs(ut[(long)s * M * nsp + n - 1]) / ((double)(n * (n - 1)) * P.tab.filt[n - 1]);
        const double a2 =
            M > 1 ? fabs(ut[((long)s * M + M - 1) * nsp]) / ((double)((M - 1) * M) * P.tab.filt[(M - 1) * nsp])
                  : 0.0;
        const double pen = (a1 * (double)(m * (m + 1)) + a2 * (double)(k * (k + 1))) * f;
        const double au = fabs(src[m]);
        const double g = au > 0.0 ? 1.0 - pen / au : 0.0;
        return g > 0.0 ? g : 0.0;
      }
      return P.filter == FRSG_FILTER_EXP ? exp(-P.alpha * dt * f) : f;
    };
    double acc = 0.0;
    if constexpr (DIM == 3) {
      for (int m = 0; m < nsp; ++m) acc += P.tri_V[j * nsp + m] * (src[m] * lam(m));
    } else if constexpr (DIM == 1) {
      for (int m = 0; m < n; ++m) acc += V[j * n + m] * (src[m] * lam(m));
    } else {
      const int a = j % n, b = j / n;
      for (int d = 0; d < n; ++d) {
        double row = 0.0;
        for (int c = 0; c < n; ++c) row += V[a * n + c] * (src[c + n * d] * lam(c + n * d));
        acc += V[b * n + d] * row;
      }
    }
    u[(long)sk * EN + (long)e * nsp + j] = acc;
  }
  if (threadIdx.x == 0 && flags) flags[e] = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define FRSG_DISPATCH_EQ(EQV, BODY)               \
  switch (EQV) {                                  \
    case kAdvection: { constexpr int EQ = kAdvection; BODY; } break; \
    case kBurgers: { constexpr int EQ = kBurgers; BODY; } break;     \
    case kEuler1: { constexpr int EQ = kEuler1; BODY; } break;       \
    default: { constexpr int EQ = kEuler2; BODY; } break;            \
  }

hipError_t launch_set_scalars(const KParams& P, double dt_fixed, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(1), 0, s, P, dt_fixed);
  return hipGetLastError();
}

hipError_t launch_dt(const KParams& P, int dim, double* dt_used, hipStream_t s) {
  if (dim == 1)
    hipLaunchKernelGGL(k_dt<1>, dim3(1), dim3(1), 0, s, P, dt_used);
  else
    hipLaunchKernelGGL(k_dt<2>, dim3(1), dim3(1), 0, s, P, dt_used);
  return hipGetLastError();
}

hipError_t launch_copy_dt(const KParams& P, double* dt_used, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_dt, dim3(1), dim3(1), 0, s, P, dt_used);
  return hipGetLastError();
}

hipError_t launch_fill_flags(unsigned char* flags, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_flags, dim3(grid_for(n)), dim3(kBlock), 0, s, flags, n);
  return hipGetLastError();
}

hipError_t launch_nodal(const KParams& P, const double* u, double* Un, double* Fn, double* Gn, int do_cfl,
                        hipStream_t s) {
  const long total = (long)P.Nq * P.E * P.nsp;
  FRSG_DISPATCH_EQ(P.eq, {
    constexpr int DIM = EQ == kEuler2 ? 2 : 1;
    hipLaunchKernelGGL((k_nodal<EQ, DIM>), dim3(grid_for(total)), dim3(kBlock), 0, s, P, u, Un, Fn, Gn, do_cfl);
  });
  return hipGetLastError();
}

hipError_t launch_faces(const KParams& P, const double* Un, const double* Fn, const double* Gn, double* Corr,
                        hipStream_t s) {
  if (P.dim == 1) {
    const long total = (long)(P.E + 1) * P.Nq;
    FRSG_DISPATCH_EQ(P.eq, {
      if constexpr (EQ != kEuler2)
        hipLaunchKernelGGL((k_faces_1d<EQ>), dim3(grid_for(total)), dim3(kBlock), 0, s, P, Un, Fn, Corr);
    });
  } else {
    const long tx = (long)P.Nq * P.ny * (P.nx + 1) * P.np1;
    const long ty = (long)P.Nq * P.nx * (P.ny + 1) * P.np1;
    hipLaunchKernelGGL((k_faces_2d<kEuler2, 0>), dim3(grid_for(tx)), dim3(kBlock), 0, s, P, Un, Fn, Corr);
    hipLaunchKernelGGL((k_faces_2d<kEuler2, 1>), dim3(grid_for(ty)), dim3(kBlock), 0, s, P, Un, Gn, Corr);
  }
  return hipGetLastError();
}

hipError_t launch_resid(const KParams& P, const double* Fn, const double* Gn, const double* Corr, double* Rn,
                        hipStream_t s) {
  const long total = (long)P.Nq * P.E * P.nsp;
  FRSG_DISPATCH_EQ(P.eq, {
    constexpr int DIM = EQ == kEuler2 ? 2 : 1;
    hipLaunchKernelGGL((k_resid<EQ, DIM>), dim3(grid_for(total)), dim3(kBlock), 0, s, P, Fn, Gn, Corr, Rn);
  });
  return hipGetLastError();
}

hipError_t launch_project_stage(const KParams& P, const double* Rn, const double* u, const double* w, double* out,
                                double cu, double cw, int rhs_only, hipStream_t s) {
  const long total = (long)P.M * P.E * P.nsp;
  FRSG_DISPATCH_EQ(P.eq, {
    hipLaunchKernelGGL((k_project<EQ>), dim3(grid_for(total)), dim3(kBlock), 0, s, P, Rn, u, w, out, cu, cw,
                       rhs_only);
  });
  return hipGetLastError();
}

hipError_t launch_project_ic(const KParams& P, const double* U0, double* u, hipStream_t s) {
  const long total = (long)P.M * P.E * P.nsp;
  FRSG_DISPATCH_EQ(P.eq, {
    hipLaunchKernelGGL((k_project_ic<EQ>), dim3(grid_for(total)), dim3(kBlock), 0, s, P, U0, u);
  });
  return hipGetLastError();
}

hipError_t launch_limiter(const KParams& P, double* u, unsigned char* flags, hipStream_t s) {
  // stage the element's coefficients in LDS when they fit in 32 KB (staged = 1),
  // with the nodal table of the solution points as well when both fit in 48 KB (2)
  const size_t bytes = sizeof(double) * (size_t)P.S * P.M * P.nsp;
  const size_t nodal = sizeof(double) * (size_t)P.S * P.nsp * P.Nq;
  const int staged = bytes + nodal <= 48 * 1024 ? 2 : (bytes <= 32 * 1024 ? 1 : 0);
  const size_t shmem = staged == 2 ? bytes + nodal : (staged ? bytes : 0);
  if (P.eq == kEuler1)
    hipLaunchKernelGGL((k_limiter<kEuler1, 1>), dim3(P.E), dim3(kElemBlock), shmem, s, P, u, flags, staged);
  else if (P.eq == kEuler2 && P.tri)
    hipLaunchKernelGGL((k_limiter<kEuler2, 3>), dim3(P.E), dim3(kElemBlock), shmem, s, P, u, flags, staged);
  else if (P.eq == kEuler2)
    hipLaunchKernelGGL((k_limiter<kEuler2, 2>), dim3(P.E), dim3(kElemBlock), shmem, s, P, u, flags, staged);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sensor_filter(const KParams& P, double* u, unsigned char* flags, hipStream_t s) {
  const size_t shmem = sizeof(double) * (size_t)P.S * P.M * P.nsp;
  if (P.tri) {
    if (P.eq != kEuler2) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sensor_filter<kEuler2, 3>), dim3(P.E), dim3(kElemBlock), shmem, s, P, u, flags);
    return hipGetLastError();
  }
  FRSG_DISPATCH_EQ(P.eq, {
    constexpr int DIM = EQ == kEuler2 ? 2 : 1;
    hipLaunchKernelGGL((k_sensor_filter<EQ, DIM>), dim3(P.E), dim3(kElemBlock), shmem, s, P, u, flags);
  });
  return hipGetLastError();
}

}  // namespace frsg
