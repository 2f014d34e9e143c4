// Discrete adjoint of the FR-SG step for the scalar 1D equations (linear
// advection, Burgers): the transpose of the right-hand side at a given state,
// applied to an adjoint vector, and the transpose of the detector-switched
// modal filter at frozen flags.
//
// The forward right-hand side (Sec. 3.2-3.4, evaluated per random node and
// Galerkin-projected, Sec. 2.1 Eq. discrete expectation value) is
//
//   R_k = sum_q PW[k,q] Rn_q,
//   Rn_q[j] = -(1/J) ( sum_l Dt[j,l] f(U_q[l]) + F*_L,q h_L'(r_j) + F*_R,q h_R'(r_j) ),
//   U_q[j] = sum_k Phi[k,q] u_k[j],   Dt = D - h_L' l(-1)^T - h_R' l(+1)^T,
//
// with F* the Lax-Friedrichs flux of the two traces at each face and node.
// Its transpose applied to g is assembled in three passes:
//
//   adj_node  (q, e):   gR = PW^T g, d = -gR / J;  GL = h_L'.d, GR = h_R'.d
//                       (adjoints of the element's left / right interface flux),
//                       GU[l] = f'(U[l]) sum_j Dt[j,l] d[j];
//   adj_face  (q, e):   transposed Lax-Friedrichs flux at the element's two faces
//                       (adjoint of the face flux = GL of the element on the right
//                       plus GR of the element on the left), giving the adjoints
//                       gTm, gTp of the element's traces at r = -1, +1;
//   adj_project (k, e, j): g_u = sum_q Phi[k,q] (GU + l_j(-1) gTm + l_j(+1) gTp),
//                       combined with up to three vectors for the SSP-RK3 chain.
//
// The dissipation speed max(|f'(L)|, |f'(R)|) is differentiated through the
// side attaining it (the left one on a tie).  The derivative with respect to the
// advection speed is reduced per block and added, scaled, into one scalar.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace frsg {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxNp = 8;  // FR degree <= 7

inline unsigned grid_for(long n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

template <typename T>
__device__ __forceinline__ T sgn(T x) { return (T)((x > T(0)) - (x < T(0))); }

// f'(U) of the scalar flux
template <int EQ, typename T>
__device__ __forceinline__ T dflux(T U, T adv) {
  if constexpr (EQ == kAdvection) return adv;
  else return U;
}

// transpose of F = (f(L) + f(R))/2 - lam (R - L)/2 applied to g; also d/da of g F
template <int EQ, typename T>
__device__ __forceinline__ void rusanov_adj(T L, T R, T g, T adv, T& gL, T& gR, T& da) {
  const T h = T(0.5);
  if constexpr (EQ == kAdvection) {
    const T aa = fabs(adv);
    gL = h * adv * g + h * aa * g;
    gR = h * adv * g - h * aa * g;
    da = g * (h * (L + R) - h * sgn(adv) * (R - L));
  } else {
    const T sL = fabs(L), sR = fabs(R);
    const T lam = fmax(sL, sR);
    const T dlam = -h * (R - L) * g;
    gL = h * L * g + h * lam * g;
    gR = h * R * g - h * lam * g;
    if (sL >= sR)
      gL += sgn(L) * dlam;
    else
      gR += sgn(R) * dlam;
    da = T(0);
  }
}

// transpose of the ghost trace of a boundary side (outflow: copy, Dirichlet: constant)
template <typename T>
__device__ __forceinline__ T ghost_adj(const KParams& P, int side, T g) {
  return P.bc[side] == FRSG_BC_OUTFLOW ? g : T(0);
}

// ghost value of a boundary side for a scalar interior trace
template <typename T>
__device__ __forceinline__ T ghost_val(const KParams& P, int side, T t) {
  return P.bc[side] == FRSG_BC_DIRICHLET ? (T)P.bc_state[side][0] : t;
}

// ---------------------------------------------------------------------------
// (q, e): nodal adjoint of the residual
// ---------------------------------------------------------------------------
template <int EQ>
__global__ void __launch_bounds__(kBlock) k_adj_node(KParams P, const double* __restrict__ Un,
                                                     const double* __restrict__ g, double* __restrict__ GU,
                                                     double* __restrict__ Gside, double* __restrict__ part) {
  __shared__ double sm[kBlock];
  const int E = P.E, n = P.np1, Nq = P.Nq, M = P.M;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  double pa = 0.0;
  if (t < (long)Nq * E) {
    const int q = (int)(t / E), e = (int)(t - (long)q * E);
    const long EN = (long)E * n;
    double d[kMaxNp];
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < M; ++k) acc += P.tab.PW[k * Nq + q] * g[(long)k * EN + (long)e * n + j];
      d[j] = -acc / P.Jx;
    }
    double GL = 0.0, GR = 0.0;
    for (int j = 0; j < n; ++j) {
      GL += P.tab.dhL[j] * d[j];
      GR += P.tab.dhR[j] * d[j];
    }
    const double* U = Un + ((long)q * E + e) * n;
    double* out = GU + ((long)q * E + e) * n;
    for (int l = 0; l < n; ++l) {
      double gF = 0.0;
      for (int j = 0; j < n; ++j) gF += P.tab.D[j * n + l] * d[j];
      gF = gF - P.tab.lL[l] * GL - P.tab.lR[l] * GR;
      out[l] = dflux<EQ>(U[l], P.adv) * gF;
      if constexpr (EQ == kAdvection) pa += gF * U[l];
    }
    Gside[((long)q * E + e) * 2 + 0] = GL;
    Gside[((long)q * E + e) * 2 + 1] = GR;
  }
  if (part) {
    const double s = block_reduce_sum(pa, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// (q, e): transposed interface fluxes at the element's two faces
// ---------------------------------------------------------------------------
template <int EQ>
__global__ void __launch_bounds__(kBlock) k_adj_face(KParams P, const double* __restrict__ Un,
                                                     const double* __restrict__ Gside, double* __restrict__ gT,
                                                     double* __restrict__ part) {
  __shared__ double sm[kBlock];
  const int E = P.E, n = P.np1, Nq = P.Nq;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  double pa = 0.0;
  if (t < (long)Nq * E) {
    const int q = (int)(t / E), e = (int)(t - (long)q * E);
    const bool periodic = P.bc[0] == FRSG_BC_PERIODIC;
    auto tr = [&](int el, const double* l) {
      const double* U = Un + ((long)q * E + el) * n;
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += l[j] * U[j];
      return acc;
    };
    auto side = [&](int el, int s) { return Gside[((long)q * E + el) * 2 + s]; };
    const double Tm = tr(e, P.tab.lL), Tp = tr(e, P.tab.lR);
    double gTm, gTp;
    {  // left face of e
      const bool interior = e > 0 || periodic;
      const int el = e > 0 ? e - 1 : E - 1;
      const double UL = interior ? tr(el, P.tab.lR) : ghost_val(P, 0, Tm);
      const double gF = side(e, 0) + (interior ? side(el, 1) : 0.0);
      double gL, gR, da;
      rusanov_adj<EQ>(UL, Tm, gF, P.adv, gL, gR, da);
      gTm = gR + (interior ? 0.0 : ghost_adj(P, 0, gL));
      pa += da;
    }
    {  // right face of e
      const bool interior = e < E - 1 || periodic;
      const int er = e < E - 1 ? e + 1 : 0;
      const double UR = interior ? tr(er, P.tab.lL) : ghost_val(P, 1, Tp);
      const double gF = side(e, 1) + (interior ? side(er, 0) : 0.0);
      double gL, gR, da;
      rusanov_adj<EQ>(Tp, UR, gF, P.adv, gL, gR, da);
      gTp = gL + (interior ? 0.0 : ghost_adj(P, 1, gR));
      if (!interior) pa += da;  // the last face of a non-periodic mesh has no element on its right
    }
    gT[((long)q * E + e) * 2 + 0] = gTm;
    gT[((long)q * E + e) * 2 + 1] = gTp;
  }
  if (part) {
    const double s = block_reduce_sum(pa, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// (k, e, j): back to the modes, combined with the SSP-RK3 chain
//   out = c0 x0 + c1 x1 + c2 x2 + cg * (dR/du)^T g
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_adj_project(KParams P, const double* __restrict__ GU,
                                                        const double* __restrict__ gT, const double* x0,
                                                        const double* x1, const double* x2, double* out, double c0,
                                                        double c1, double c2, double cg) {
  const int E = P.E, n = P.np1, Nq = P.Nq, M = P.M;
  const long EN = (long)E * n;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  if (t >= (long)M * EN) return;
  const int k = (int)(t / EN);
  const long ej = t - (long)k * EN;
  const int e = (int)(ej / n), j = (int)(ej - (long)e * n);
  const double lLj = P.tab.lL[j], lRj = P.tab.lR[j];
  double acc = 0.0;
  for (int q = 0; q < Nq; ++q) {
    const long qe = (long)q * E + e;
    acc += P.tab.Phi[k * Nq + q] * (GU[qe * n + j] + lLj * gT[qe * 2 + 0] + lRj * gT[qe * 2 + 1]);
  }
  double v = cg * acc;
  if (x0) v += c0 * x0[t];
  if (x1) v += c1 * x1[t];
  if (x2) v += c2 * x2[t];
  out[t] = v;
}

// dparam[0] += scale * (sum of the partial sums), one thread, fixed order
__global__ void k_adj_param(const double* __restrict__ part, int n, double scale, double* dparam) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  dparam[0] += scale * s;
}

// ---------------------------------------------------------------------------
// transposed filter on the flagged elements, identity elsewhere (Sec. 4.1 at
// frozen switches): out = V^-T diag(Lambda) V^T g per chaos mode
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_filter_adj(KParams P, const double* __restrict__ g,
                                                       const unsigned char* __restrict__ flags, double* out) {
  const int E = P.E, n = P.np1, M = P.M;
  const long EN = (long)E * n;
  const long t = blockIdx.x * (long)kBlock + threadIdx.x;
  if (t >= (long)M * E) return;
  const int k = (int)(t / E), e = (int)(t - (long)k * E);
  const double* src = g + (long)k * EN + (long)e * n;
  double* dst = out + (long)k * EN + (long)e * n;
  if (!flags[e]) {
    for (int j = 0; j < n; ++j) dst[j] = src[j];
    return;
  }
  const double dt = *P.dt;
  double x[kMaxNp];
  for (int l = 0; l < n; ++l) {  // Lambda (V^T g)
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += P.tab.V[j * n + l] * src[j];
    const double f = P.tab.filt[k * n + l];
    x[l] = acc * (P.filter == FRSG_FILTER_EXP ? exp(-P.alpha * dt * f) : f);
  }
  for (int l = 0; l < n; ++l) {  // V^-T x
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += P.tab.Vinv[m * n + l] * x[m];
    dst[l] = acc;
  }
}

// ---------------------------------------------------------------------------
// fused transposed right-hand side for a block of EB elements (the same three
// steps as k_adj_node / k_adj_face / k_adj_project, with the state and adjoint
// coefficients of the block and one neighbour on each side staged in LDS)
//   out = c0 x0 + c1 x1 + c2 x2 + cg (dR/dw)^T g
// FP32-mixed (R = float): the node and face steps and the projection of the
// modes k >= 1 in FP32 on the FP64 inputs and tables rounded to FP32; mode 0 is
// projected in FP64, and the combination is FP64.
// ---------------------------------------------------------------------------
constexpr int kBlockA = 256;

struct AdjStageArgs {
  const double* w;  // state the right-hand side is linearised at
  const double* g;  // adjoint vector
  const double* x0;
  const double* x1;
  const double* x2;
  double* out;
  double c0, c1, c2, cg;
  double* part;     // per-workgroup partial sums of d<g, R>/da (advection), or null
  int EB;
};

template <int EQ, int N, typename R>
__global__ void __launch_bounds__(kBlockA) k_adj_stage1d(KParams P, AdjStageArgs A) {
  constexpr int n = N;
  extern __shared__ double smem[];
  __shared__ double sm[kBlockA];
  const int E = P.E, M = P.M, Nq = P.Nq, EB = A.EB;
  const int e0 = blockIdx.x * EB;
  const int nloc = min(EB, E - e0);
  const int nc = M * n;
  const long EN = (long)E * n;
  double* sW = smem;                         // [EB + 2][M][n]
  double* sGc = sW + (EB + 2) * nc;          // [EB + 2][M][n]
  double* sT = sGc + (EB + 2) * nc;          // [EB + 2][Nq][2] traces at r = -1, +1
  double* sS = sT + (EB + 2) * Nq * 2;       // [EB + 2][Nq][2] adjoints of the left / right face fluxes
  double* sU = sS + (EB + 2) * Nq * 2;       // [EB][n][Nq] nodal adjoint of the state
  const bool periodic = P.bc[0] == FRSG_BC_PERIODIC;
  const int tid = threadIdx.x;

  const int span = (nloc + 2) * n;
  // unrolled so that a thread's loads of both arrays are in flight together
#pragma unroll 3
  for (int it = tid; it < M * span; it += kBlockA) {
    const int k = it / span, rem = it - k * span;
    const int ls = rem / n, j = rem - ls * n;
    int e = e0 - 1 + ls;
    if (e < 0) e = periodic ? E - 1 : 0;
    if (e >= E) e = periodic ? 0 : E - 1;
    const long src = (long)k * EN + (long)e * n + j;
    sW[ls * nc + k * n + j] = A.w[src];
    sGc[ls * nc + k * n + j] = A.g[src];
  }
  __syncthreads();

  const int ls = tid / Nq, q = tid - ls * Nq;
  const bool active = ls < nloc + 2;
  const bool owned = active && ls >= 1 && ls <= nloc;
  const R adv = (R)P.adv;
  R U[n], GU[n];
  R pa = R(0);
  R tm = R(0), tp = R(0);
  if (active) {
    const double* W = sW + ls * nc;
    const double* Gc = sGc + ls * nc;
    const R Jx = (R)P.Jx;
    R d[n], gr[n];
#pragma unroll
    for (int j = 0; j < n; ++j) U[j] = gr[j] = R(0);
    // mode by mode into every point's sums: each sum takes the modes in order,
    // and the 2 n chains are independent
    for (int k = 0; k < M; ++k) {
      const R phi = (R)P.tab.Phi[k * Nq + q], pw = (R)P.tab.PW[k * Nq + q];
#pragma unroll
      for (int j = 0; j < n; ++j) {
        U[j] += (R)W[k * n + j] * phi;
        gr[j] += pw * (R)Gc[k * n + j];
      }
    }
#pragma unroll
    for (int j = 0; j < n; ++j) d[j] = -gr[j] / Jx;
    R GL = R(0), GR = R(0);
#pragma unroll
    for (int j = 0; j < n; ++j) {
      GL += (R)P.tab.dhL[j] * d[j];
      GR += (R)P.tab.dhR[j] * d[j];
      tm += (R)P.tab.lL[j] * U[j];
      tp += (R)P.tab.lR[j] * U[j];
    }
#pragma unroll
    for (int l = 0; l < n; ++l) {
      R gF = R(0);
#pragma unroll
      for (int j = 0; j < n; ++j) gF += (R)P.tab.D[j * n + l] * d[j];
      gF = gF - (R)P.tab.lL[l] * GL - (R)P.tab.lR[l] * GR;
      GU[l] = dflux<EQ>(U[l], adv) * gF;
      if constexpr (EQ == kAdvection)
        if (owned) pa += gF * U[l];
    }
    double* T = sT + ((long)ls * Nq + q) * 2;
    T[0] = tm;
    T[1] = tp;
    double* G2 = sS + ((long)ls * Nq + q) * 2;
    G2[0] = GL;
    G2[1] = GR;
  }
  __syncthreads();

  if (owned) {
    const int e = e0 + ls - 1;
    const double* Tl = sT + ((long)(ls - 1) * Nq + q) * 2;
    const double* Tr = sT + ((long)(ls + 1) * Nq + q) * 2;
    const double* Sl = sS + ((long)(ls - 1) * Nq + q) * 2;
    const double* Sc = sS + ((long)ls * Nq + q) * 2;
    const double* Sr = sS + ((long)(ls + 1) * Nq + q) * 2;
    R gTm, gTp;
    {  // left face
      const bool interior = e > 0 || periodic;
      const R UL = interior ? (R)Tl[1] : ghost_val(P, 0, tm);
      const R gF = (R)Sc[0] + (interior ? (R)Sl[1] : R(0));
      R gL, gR, da;
      rusanov_adj<EQ>(UL, tm, gF, adv, gL, gR, da);
      gTm = gR + (interior ? R(0) : ghost_adj(P, 0, gL));
      pa += da;
    }
    {  // right face
      const bool interior = e < E - 1 || periodic;
      const R UR = interior ? (R)Tr[0] : ghost_val(P, 1, tp);
      const R gF = (R)Sc[1] + (interior ? (R)Sr[0] : R(0));
      R gL, gR, da;
      rusanov_adj<EQ>(tp, UR, gF, adv, gL, gR, da);
      gTp = gL + (interior ? R(0) : ghost_adj(P, 1, gR));
      if (!interior) pa += da;
    }
#pragma unroll
    for (int j = 0; j < n; ++j)
      sU[((long)(ls - 1) * n + j) * Nq + q] = (double)(GU[j] + (R)P.tab.lL[j] * gTm + (R)P.tab.lR[j] * gTp);
  }
  if (A.part) {
    const double sum = block_reduce_sum((double)pa, sm);
    if (tid == 0) A.part[blockIdx.x] = sum;
  } else {
    __syncthreads();
  }

  // thread (block of KB modes, element, point): one pass over the nodal adjoint
  // feeds KB independent sums, each taking the nodes in order
  constexpr int KB = 4;
  const int nkb = (M + KB - 1) / KB;
  const int ospan = nloc * n;
  for (int it = tid; it < nkb * ospan; it += kBlockA) {
    const int kb = it / ospan, rem = it - kb * ospan;
    const int le = rem / n, j = rem - le * n;
    const int k0 = kb * KB;
    const double* Gq = sU + ((long)le * n + j) * Nq;
    const double* Phk[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) Phk[i] = P.tab.Phi + min(k0 + i, M - 1) * Nq;  // clamped: past M unused
    double ad[KB];
    R ar[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      ad[i] = 0.0;
      ar[i] = R(0);
    }
    for (int qq = 0; qq < Nq; ++qq) {
      const double gq = Gq[qq];
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        if (std::is_same<R, double>::value || k0 + i == 0)
          ad[i] += Phk[i][qq] * gq;  // FP64 (the mean mode in every precision)
        else
          ar[i] += (R)Phk[i][qq] * (R)gq;
      }
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      const int k = k0 + i;
      if (k >= M) continue;
      const double acc = (std::is_same<R, double>::value || k == 0) ? ad[i] : (double)ar[i];
      const long idx = (long)k * EN + (long)(e0 + le) * n + j;
      double v = A.cg * acc;
      if (A.x0) v += A.c0 * A.x0[idx];
      if (A.x1) v += A.c1 * A.x1[idx];
      if (A.x2) v += A.c2 * A.x2[idx];
      A.out[idx] = v;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static void adj1d_shape(const KParams& P, int& EB, size_t& shmem) {
  EB = kBlockA / P.Nq - 2;
  if (EB < 1 || P.np1 > kMaxNp || P.S != 1 || P.dim != 1) {
    EB = 0;
    shmem = 0;
    return;
  }
  const size_t nc = (size_t)P.M * P.np1;
  shmem = sizeof(double) * (2 * (EB + 2) * nc + 4 * (size_t)(EB + 2) * P.Nq + (size_t)EB * P.np1 * P.Nq);
  if (shmem > 48 * 1024) {
    EB = 0;
    shmem = 0;
  }
}

bool adj1d_fused_supported(const KParams& P) {
  int EB;
  size_t sh;
  adj1d_shape(P, EB, sh);
  return EB > 0;
}

long adj1d_partials(const KParams& P) {
  int EB;
  size_t sh;
  adj1d_shape(P, EB, sh);
  return EB > 0 ? (P.E + EB - 1) / EB : 0;
}

hipError_t launch_adj_stage1d(const KParams& P, const double* w, const double* g, const double* x0, const double* x1,
                              const double* x2, double* out, double c0, double c1, double c2, double cg, double* part,
                              double param_scale, double* dparam, hipStream_t s) {
  int EB;
  size_t shmem;
  adj1d_shape(P, EB, shmem);
  if (EB == 0) return hipErrorInvalidValue;
  const bool want = P.eq == kAdvection && dparam && part;
  AdjStageArgs A{w, g, x0, x1, x2, out, c0, c1, c2, cg, want ? part : nullptr, EB};
  const unsigned grid = (unsigned)((P.E + EB - 1) / EB);
  auto go = [&](auto eq_tag) -> hipError_t {
    constexpr int EQ = decltype(eq_tag)::value;
    if (P.fp32) {
      switch (P.np1) {
#define FRSG_N(NN) \
  case NN: hipLaunchKernelGGL((k_adj_stage1d<EQ, NN, float>), dim3(grid), dim3(kBlockA), shmem, s, P, A); break;
        FRSG_N(2) FRSG_N(3) FRSG_N(4) FRSG_N(5) FRSG_N(6) FRSG_N(7) FRSG_N(8)
#undef FRSG_N
        default: return hipErrorInvalidValue;
      }
    } else {
      switch (P.np1) {
#define FRSG_N(NN) \
  case NN: hipLaunchKernelGGL((k_adj_stage1d<EQ, NN, double>), dim3(grid), dim3(kBlockA), shmem, s, P, A); break;
        FRSG_N(2) FRSG_N(3) FRSG_N(4) FRSG_N(5) FRSG_N(6) FRSG_N(7) FRSG_N(8)
#undef FRSG_N
        default: return hipErrorInvalidValue;
      }
    }
    return hipGetLastError();
  };
  hipError_t e;
  if (P.eq == kAdvection)
    e = go(std::integral_constant<int, kAdvection>{});
  else if (P.eq == kBurgers)
    e = go(std::integral_constant<int, kBurgers>{});
  else
    return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  if (want) hipLaunchKernelGGL(k_adj_param, dim3(1), dim3(64), 0, s, part, (int)grid, param_scale, dparam);
  return hipGetLastError();
}
long adjoint_partials(const KParams& P) { return 2 * (long)grid_for((long)P.Nq * P.E); }

hipError_t launch_rhs_adjoint(const KParams& P, const double* Un, const double* g, double* GU, double* Gside,
                              double* gT, const double* x0, const double* x1, const double* x2, double* out,
                              double c0, double c1, double c2, double cg, double* part, double param_scale,
                              double* dparam, hipStream_t s) {
  const long nqe = (long)P.Nq * P.E;
  const unsigned gq = grid_for(nqe);
  const bool want = P.eq == kAdvection && dparam && part;
  double* p0 = want ? part : nullptr;
  double* p1 = want ? part + gq : nullptr;
  if (P.eq == kAdvection) {
    hipLaunchKernelGGL(k_adj_node<kAdvection>, dim3(gq), dim3(kBlock), 0, s, P, Un, g, GU, Gside, p0);
    hipLaunchKernelGGL(k_adj_face<kAdvection>, dim3(gq), dim3(kBlock), 0, s, P, Un, Gside, gT, p1);
  } else if (P.eq == kBurgers) {
    hipLaunchKernelGGL(k_adj_node<kBurgers>, dim3(gq), dim3(kBlock), 0, s, P, Un, g, GU, Gside, nullptr);
    hipLaunchKernelGGL(k_adj_face<kBurgers>, dim3(gq), dim3(kBlock), 0, s, P, Un, Gside, gT, nullptr);
  } else {
    return hipErrorInvalidValue;
  }
  const long total = (long)P.M * P.E * P.np1;
  hipLaunchKernelGGL(k_adj_project, dim3(grid_for(total)), dim3(kBlock), 0, s, P, GU, gT, x0, x1, x2, out, c0, c1,
                     c2, cg);
  if (want) hipLaunchKernelGGL(k_adj_param, dim3(1), dim3(64), 0, s, part, (int)(2 * gq), param_scale, dparam);
  return hipGetLastError();
}

hipError_t launch_filter_adjoint(const KParams& P, const double* g, const unsigned char* flags, double* out,
                                 hipStream_t s) {
  const long total = (long)P.M * P.E;
  hipLaunchKernelGGL(k_filter_adj, dim3(grid_for(total)), dim3(kBlock), 0, s, P, g, flags, out);
  return hipGetLastError();
}

}  // namespace frsg
