// Fused FR-SG stage kernel for the 1D equations (linear advection, Burgers,
// Euler): one launch computes the whole right-hand side of a block of elements
// (Sec. 2.1 chaos expansion and Galerkin projection, Sec. 3.2-3.4 flux
// reconstruction with Lax-Friedrichs interface fluxes per random node) and the
// SSP-RK3 stage combination.  The limiter and the detector-switched filter stay
// separate element-wise passes.
//
// A workgroup owns EB consecutive elements plus one neighbour on each side:
//   1. the modal coefficients of the EB + 2 elements are staged in LDS
//      (coalesced);
//   2. thread (element, node q) expands its element at node q, evaluates the
//      flux at the solution points and the two traces, and publishes the traces
//      in LDS;
//   3. thread (element, q) forms the Lax-Friedrichs fluxes at both faces (ghost
//      traces at non-periodic boundaries) and the nodal residual
//        R_q[j] = -(1/J) ( sum_l Dt[j,l] f_q[l] + F*_L h_L'(r_j) + F*_R h_R'(r_j) ),
//      Dt = D - h_L' l(-1)^T - h_R' l(+1)^T, into LDS;
//   4. thread (element, variable, mode, point) projects, sum_q PW[k,q] R_q[j],
//      and writes cu u + cw (w + dt R) (or R alone for a right-hand side).
// Element counts that are not a multiple of EB leave the last workgroup partly idle.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace frsg {
namespace {

constexpr int kBlock1 = 256;
constexpr int kMaxN = 8;  // FR degree <= 7

struct Stage1DArgs {
  const double* in;   // state the right-hand side is taken of
  const double* u;    // u^n for the combination (may equal in)
  const double* w;    // w for the combination
  double* out;
  double cu, cw;
  int rhs_only;
  unsigned char* clear_flags;  // per element, set to 0 (no limiter); may be null
  int EB;                      // elements per workgroup
};

template <int EQ, int N>
__global__ void __launch_bounds__(kBlock1) k_stage1d(KParams P, Stage1DArgs A) {
  constexpr int S = nstate<EQ>();
  constexpr int n = N;
  extern __shared__ double smem[];
  const int E = P.E, M = P.M, Nq = P.Nq, EB = A.EB;
  const int e0 = blockIdx.x * EB;
  const int nloc = min(EB, E - e0);           // elements owned by this workgroup
  const int ncoef = S * M * n;                 // coefficients per element
  const long EN = (long)E * n;
  double* sC = smem;                           // [EB + 2][S][M][n]
  double* sTr = sC + (EB + 2) * ncoef;         // [EB + 2][Nq][2][S] traces at r = -1, +1
  double* sR = sTr + (EB + 2) * Nq * 2 * S;    // [EB][S][n][Nq] nodal residual
  const bool periodic = P.bc[0] == FRSG_BC_PERIODIC;
  const int tid = threadIdx.x;

  // 1. stage coefficients: local slot ls = 0 .. nloc + 1 holds element e0 - 1 + ls
  // (variable, mode) outer, so consecutive threads read consecutive addresses
  const int span = (nloc + 2) * n;
  for (int it = tid; it < S * M * span; it += kBlock1) {
    const int sk = it / span, rem = it - sk * span;  // sk = s * M + k
    const int ls = rem / n, j = rem - ls * n;
    int e = e0 - 1 + ls;
    if (e < 0) e = periodic ? E - 1 : 0;         // non-periodic: replaced by ghosts below
    if (e >= E) e = periodic ? 0 : E - 1;
    sC[ls * ncoef + sk * n + j] = A.in[(long)sk * EN + (long)e * n + j];
  }
  __syncthreads();

  // 2. expansion at node q, flux, traces
  const int ls = tid / Nq, q = tid - ls * Nq;
  const bool active = ls < nloc + 2;
  double F[S][N];
  if (active) {
    double U[S][N];
    const double* C = sC + ls * ncoef;
#pragma unroll
    for (int j = 0; j < n; ++j) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) acc += C[(s * M + k) * n + j] * P.tab.Phi[k * Nq + q];
        U[s][j] = acc;
      }
    }
    double tm[S], tp[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        a += P.tab.lL[j] * U[s][j];
        b += P.tab.lR[j] * U[s][j];
      }
      tm[s] = a;
      tp[s] = b;
    }
#pragma unroll
    for (int j = 0; j < n; ++j) {
      double Uj[S], Fj[S];
#pragma unroll
      for (int s = 0; s < S; ++s) Uj[s] = U[s][j];
      flux<EQ, 0>(Uj, Fj, P.adv, P.gamma);
#pragma unroll
      for (int s = 0; s < S; ++s) F[s][j] = Fj[s];
    }
    double* T = sTr + ((long)ls * Nq + q) * 2 * S;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      T[s] = tm[s];
      T[S + s] = tp[s];
    }
  }
  __syncthreads();

  // 3. interface fluxes at both faces and the nodal residual (owned elements)
  if (active && ls >= 1 && ls <= nloc) {
    const int e = e0 + ls - 1;
    const double* Tl = sTr + ((long)(ls - 1) * Nq + q) * 2 * S;  // left neighbour
    const double* Tc = sTr + ((long)ls * Nq + q) * 2 * S;
    const double* Tr = sTr + ((long)(ls + 1) * Nq + q) * 2 * S;  // right neighbour
    double UL[S], UR[S], FL[S], FR[S];
    // left face: left state = neighbour's r = +1 trace, or the ghost of our r = -1 trace
    if (e == 0 && !periodic) {
      ghost<EQ>(P, 0, Tc, UL);
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) UL[s] = Tl[S + s];
    }
    rusanov<EQ, 0>(UL, Tc, FL, P.adv, P.gamma);
    // right face: right state = neighbour's r = -1 trace, or the ghost of our r = +1 trace
    if (e == E - 1 && !periodic) {
      ghost<EQ>(P, 1, Tc + S, UR);
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) UR[s] = Tr[s];
    }
    rusanov<EQ, 0>(Tc + S, UR, FR, P.adv, P.gamma);
    const double iJ = 1.0 / P.Jx;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // f^D at the faces enters through Dt; the interface fluxes through h'
      double fdl = 0.0, fdr = 0.0;
#pragma unroll
      for (int l = 0; l < n; ++l) {
        fdl += P.tab.lL[l] * F[s][l];
        fdr += P.tab.lR[l] * F[s][l];
      }
#pragma unroll
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < n; ++l) acc += P.tab.D[j * n + l] * F[s][l];
        acc = acc + (FL[s] - fdl) * P.tab.dhL[j] + (FR[s] - fdr) * P.tab.dhR[j];
        sR[(((long)(ls - 1) * S + s) * n + j) * Nq + q] = -acc * iJ;
      }
    }
  }
  __syncthreads();

  // 4. projection and stage combination
  const double dt = A.rhs_only ? 0.0 : *P.dt;
  const int ospan = nloc * n;
  for (int it = tid; it < S * M * ospan; it += kBlock1) {
    const int sk = it / ospan, rem = it - sk * ospan;
    const int le = rem / n, j = rem - le * n;
    const int s = sk / M, k = sk - s * M;
    const double* Rq = sR + (((long)le * S + s) * n + j) * Nq;
    double acc = 0.0;
    for (int qq = 0; qq < Nq; ++qq) acc += P.tab.PW[k * Nq + qq] * Rq[qq];
    const long idx = (long)sk * EN + (long)(e0 + le) * n + j;
    A.out[idx] = A.rhs_only ? acc : A.cu * A.u[idx] + A.cw * (A.w[idx] + dt * acc);
  }
  if (A.clear_flags)
    for (int it = tid; it < nloc; it += kBlock1) A.clear_flags[e0 + it] = 0;
}

// CFL maximum of a 1D state: a workgroup stages the coefficients of 256 / Nq
// elements in LDS; thread (element, node q) takes the maximum over the points
template <int EQ>
__global__ void __launch_bounds__(kBlock1) k_cfl1d(KParams P, const double* __restrict__ u, int EB) {
  constexpr int S = nstate<EQ>();
  extern __shared__ double sC[];  // [EB][S][M][n]
  __shared__ double sm[kBlock1];
  const int E = P.E, n = P.np1, M = P.M, Nq = P.Nq;
  const long EN = (long)E * n;
  const int e0 = blockIdx.x * EB, nloc = min(EB, E - e0);
  const int ncoef = S * M * n, span = nloc * n;
  for (int it = threadIdx.x; it < S * M * span; it += kBlock1) {
    const int sk = it / span, rem = it - sk * span;
    const int le = rem / n, j = rem - le * n;
    sC[le * ncoef + sk * n + j] = u[(long)sk * EN + (long)(e0 + le) * n + j];
  }
  __syncthreads();
  const int le = threadIdx.x / Nq, q = threadIdx.x - le * Nq;
  double rate = 0.0;
  if (le < nloc) {
    const double* C = sC + le * ncoef;
    for (int j = 0; j < n; ++j) {
      double U[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) acc += C[(s * M + k) * n + j] * P.tab.Phi[k * Nq + q];
        U[s] = acc;
      }
      double r = speed<EQ, 0>(U, P.adv, P.gamma);
      if (!(r == r)) r = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf, dt -> 0
      rate = fmax(rate, r);
    }
  }
  sm[threadIdx.x] = rate;
  __syncthreads();
  for (int o = kBlock1 / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(P.lam_bits, (unsigned long long)__double_as_longlong(sm[0]));
}

}  // namespace

// elements per workgroup and LDS bytes; EB = 0 when the node count does not fit
static void fr1d_shape(const KParams& P, int& EB, size_t& shmem) {
  EB = kBlock1 / P.Nq - 2;
  if (EB < 1 || P.np1 > kMaxN) {
    EB = 0;
    shmem = 0;
    return;
  }
  const size_t ncoef = (size_t)P.S * P.M * P.np1;
  shmem = sizeof(double) * ((EB + 2) * ncoef + (size_t)(EB + 2) * P.Nq * 2 * P.S + (size_t)EB * P.S * P.np1 * P.Nq);
  if (shmem > 64 * 1024) {
    EB = 0;
    shmem = 0;
  }
}

bool fr1d_supported(const KParams& P) {
  if (P.dim != 1) return false;
  int EB;
  size_t sh;
  fr1d_shape(P, EB, sh);
  return EB > 0;
}

hipError_t launch_stage1d(const KParams& P, const double* in, const double* u, const double* w, double* out, double cu,
                          double cw, int rhs_only, unsigned char* clear_flags, hipStream_t s) {
  int EB;
  size_t shmem;
  fr1d_shape(P, EB, shmem);
  if (EB == 0) return hipErrorInvalidValue;
  Stage1DArgs A{in, u, w, out, cu, cw, rhs_only, clear_flags, EB};
  const unsigned grid = (unsigned)((P.E + EB - 1) / EB);
  auto go = [&](auto eq_tag) -> hipError_t {
    constexpr int EQ = decltype(eq_tag)::value;
    switch (P.np1) {
#define FRSG_N(NN) \
  case NN: hipLaunchKernelGGL((k_stage1d<EQ, NN>), dim3(grid), dim3(kBlock1), shmem, s, P, A); break;
      FRSG_N(2) FRSG_N(3) FRSG_N(4) FRSG_N(5) FRSG_N(6) FRSG_N(7) FRSG_N(8)
#undef FRSG_N
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  switch (P.eq) {
    case kAdvection: return go(std::integral_constant<int, kAdvection>{});
    case kBurgers: return go(std::integral_constant<int, kBurgers>{});
    case kEuler1: return go(std::integral_constant<int, kEuler1>{});
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cfl1d(const KParams& P, const double* u, hipStream_t s) {
  const int EB = kBlock1 / P.Nq;  // >= 1 wherever the fused 1D path runs
  if (EB < 1) return hipErrorInvalidValue;
  const size_t shmem = sizeof(double) * (size_t)EB * P.S * P.M * P.np1;
  const unsigned grid = (unsigned)((P.E + EB - 1) / EB);
  switch (P.eq) {
    case kAdvection: hipLaunchKernelGGL(k_cfl1d<kAdvection>, dim3(grid), dim3(kBlock1), shmem, s, P, u, EB); break;
    case kBurgers: hipLaunchKernelGGL(k_cfl1d<kBurgers>, dim3(grid), dim3(kBlock1), shmem, s, P, u, EB); break;
    case kEuler1: hipLaunchKernelGGL(k_cfl1d<kEuler1>, dim3(grid), dim3(kBlock1), shmem, s, P, u, EB); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace frsg
