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
//
// FP32-mixed precision (R = float): steps 2 and 3 and the projection of the
// modes k >= 1 run in FP32 on the FP64 coefficients and tables rounded to FP32;
// the mean mode k = 0 is projected in FP64 (of the FP32 nodal residual), and the
// stage combination, the filter, the limiter and the CFL maximum stay in FP64.
// Both sides of a face read the same trace from LDS, so the interface flux is
// single-valued.
//
// BF16-split precision (XF = 1, R = float): the two random-space transforms are
// dense contractions and run on the matrix cores.  The chaos expansion of step 2
// is one product per 16 rows (element, variable, solution point) and 16 nodes,
// [rows x modes] x [modes x nodes], and the projection of step 4 one product per
// 16 rows, [rows x nodes] x [nodes x modes] accumulated over the blocks of 16
// nodes; both with each operand split into bfloat16 high and low parts and FP32
// accumulation.  The fluxes and residual are FP32 as above; the mean mode is
// projected in FP64, and the epilogue is FP64.  M <= 16 (one block of modes).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"
#include "mfma_bf16.hpp"

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
  int limit;                   // apply the positivity limiter to the output (Euler)
  int end_of_step;             // detector-switched filter before the limiter, CFL maximum after
  unsigned char* flag_lim;     // per element: limiter acted (may be null)
  unsigned char* flag_filt;    // per element: filter acted (may be null)
  int cfl_out;                   // end of step: take the CFL maximum of the output
  unsigned long long* lam_next;  // accumulator the maximum is merged into (may be null)
  // Butcher-row form (tab > 0) instead of cu u + cw (w + dt R): out = u + dt (sum_j ka[j]
  // kk[j] + ka_cur R) over the nt earlier stage right-hand sides with nonzero
  // coefficients, in stage order, R last (skipped when ka_cur is 0); R itself is stored
  // in k_out when that is not null
  int tab;
  int nt;
  const double* kk[kRkMaxTerms];
  double ka[kRkMaxTerms];
  double ka_cur;
  double* k_out;
  int flag_or;                   // limiter flags OR-ed into flag_lim (set only where it acts)
  // time step: dt_source 0 reads *P.dt; 1 takes dt_fixed; 2 computes it from the
  // CFL accumulator lam_in.  With 1 or 2, workgroup 0 also stores it in *P.dt and
  // dt_used, zeroes lam_reset and latches a non-finite or non-positive dt.  3 takes
  // dt_fixed and leaves all of that to the caller.
  int dt_source;
  double dt_fixed;
  const unsigned long long* lam_in;
  unsigned long long* lam_reset;
  double* dt_used;
};

// padded sizes of the matrix-core operands: rows of 16, nodes in blocks of 16
__host__ __device__ inline int pad16(int x) { return (x + 15) & ~15; }

// One stage over the elements of workgroup blk, run by BS threads.  Returns the
// CFL maximum of the workgroup's output (every thread) when it is asked for
// (end of step and cfl_out), else 0.
template <int EQ, int N, typename R, int XF, int BS>
__device__ __forceinline__ double stage1d_block(const KParams& P, const Stage1DArgs& A, int blk) {
  // products fuse with the sum of the same expression only, so every kernel that
  // runs this code (one launch per stage, or several steps in one launch) rounds
  // alike whatever it knows of the arguments at compile time
#pragma clang fp contract(on)
  constexpr int S = nstate<EQ>();
  constexpr int n = N;
  extern __shared__ double smem[];
  const int E = P.E, M = P.M, Nq = P.Nq, EB = A.EB;
  const int e0 = blk * EB;
  const int nloc = min(EB, E - e0);           // elements owned by this workgroup
  const int ncoef = S * M * n;                 // coefficients per element
  const long EN = (long)E * n;
  double* sC = smem;                           // [EB + 2][S][M][n]
  double* sTr = sC + (EB + 2) * ncoef;         // [EB + 2][Nq][2][S] traces at r = -1, +1
  double* sR = sTr + (EB + 2) * Nq * 2 * S;    // [EB][S][n][Nq] nodal residual
  // matrix-core transforms: projected mean mode (FP64), nodal values, projected modes
  const int NQP = pad16(Nq);
  double* sP0 = sR + (long)EB * S * n * Nq;             // [EB S n]
  float* sU = reinterpret_cast<float*>(sP0 + EB * S * n);  // [pad16((EB + 2) S n)][NQP]
  float* sPk = sU + (long)pad16((EB + 2) * S * n) * NQP;  // [pad16(EB S n)][16]
  const bool periodic = P.bc[0] == FRSG_BC_PERIODIC;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, li = tid & 15, lc = (tid >> 4) & 3;

  // 1. stage coefficients: local slot ls = 0 .. nloc + 1 holds element e0 - 1 + ls
  // (variable, mode) outer, so consecutive threads read consecutive addresses
  const int span = (nloc + 2) * n;
  auto stage_in = [&](int it) {
    const int sk = it / span, rem = it - sk * span;  // sk = s * M + k
    const int ls = rem / n, j = rem - ls * n;
    int e = e0 - 1 + ls;
    if (e < 0) e = periodic ? E - 1 : 0;         // non-periodic: replaced by ghosts below
    if (e >= E) e = periodic ? 0 : E - 1;
    sC[ls * ncoef + sk * n + j] = A.in[(long)sk * EN + (long)e * n + j];
  };
  if constexpr (S > 1) {
    // several loads in flight per thread: a system's workgroup stages several
    // values per thread (the Euler problem with 11 modes: 5-6); the scalar
    // equations' 1-3 per thread gain nothing from it
#pragma unroll 4
    for (int it = tid; it < S * M * span; it += BS) stage_in(it);
  } else {
    for (int it = tid; it < S * M * span; it += BS) stage_in(it);
  }
  __syncthreads();

  // 1b. matrix cores: nodal values of every (element slot, variable, point) row at
  // every node, 16 rows x 16 nodes per product (whole waves, rows and nodes past
  // the end padded with zeros)
  if constexpr (XF) {
    const int xrows = (nloc + 2) * S * n;
    const int RT = (xrows + 15) >> 4, NT = NQP >> 4;
    for (int t = wave; t < RT * NT; t += BS / 64) {
      const int rt = t / NT, nt = t - rt * NT;
      const int r = 16 * rt + li, qq = 16 * nt + li;
      const int lsr = r / (S * n), rr = r - lsr * S * n, sr = rr / n, jr = rr - sr * n;
      float a[4], b[4];
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int k = 4 * lc + it;
        a[it] = (r < xrows && k < M) ? (float)sC[lsr * ncoef + (sr * M + k) * n + jr] : 0.0f;
        b[it] = (k < M && qq < Nq) ? (float)P.tab.Phi[k * Nq + qq] : 0.0f;
      }
      v4s ah, al, bh, bl;
      split4(a, ah, al);
      split4(b, bh, bl);
      const v4f z = {0.0f, 0.0f, 0.0f, 0.0f};
      const v4f d = mfma_split(ah, al, bh, bl, z);
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) sU[(long)(16 * rt + 4 * lc + reg) * NQP + qq] = d[reg];
    }
    __syncthreads();
  }

  // 2. expansion at node q, flux, traces
  const int ls = tid / Nq, q = tid - ls * Nq;
  const bool active = ls < nloc + 2;
  const R adv = (R)P.adv, gam = (R)P.gamma;
  R F[S][N];
  if (active) {
    R U[S][N];
    const double* C = sC + ls * ncoef;
    if constexpr (XF) {
#pragma unroll
      for (int j = 0; j < n; ++j)
#pragma unroll
        for (int s = 0; s < S; ++s) U[s][j] = (R)sU[(long)((ls * S + s) * n + j) * NQP + q];
    } else {
      // mode by mode into every (variable, point) sum: each sum takes its terms in
      // mode order, and the S n chains are independent
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int j = 0; j < n; ++j) U[s][j] = R(0);
      for (int k = 0; k < M; ++k) {
        const R phi = (R)P.tab.Phi[k * Nq + q];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int j = 0; j < n; ++j) U[s][j] += (R)C[(s * M + k) * n + j] * phi;
      }
    }
    R tm[S], tp[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      R a = R(0), b = R(0);
#pragma unroll
      for (int j = 0; j < n; ++j) {
        a += (R)P.tab.lL[j] * U[s][j];
        b += (R)P.tab.lR[j] * U[s][j];
      }
      tm[s] = a;
      tp[s] = b;
    }
#pragma unroll
    for (int j = 0; j < n; ++j) {
      R Uj[S], Fj[S];
#pragma unroll
      for (int s = 0; s < S; ++s) Uj[s] = U[s][j];
      flux<EQ, 0>(Uj, Fj, adv, gam);
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
    // traces in the arithmetic of the node loop (exact: LDS holds the values it wrote)
    R TL[S], TC[S], TCp[S], TR[S], UL[S], UR[S], FL[S], FR[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      TL[s] = (R)Tl[S + s];
      TC[s] = (R)Tc[s];
      TCp[s] = (R)Tc[S + s];
      TR[s] = (R)Tr[s];
    }
    // left face: left state = neighbour's r = +1 trace, or the ghost of our r = -1 trace
    if (e == 0 && !periodic) {
      ghost<EQ>(P, 0, TC, UL);
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) UL[s] = TL[s];
    }
    interface_flux<EQ, 0>(P.flux, UL, TC, FL, adv, gam);
    // right face: right state = neighbour's r = -1 trace, or the ghost of our r = +1 trace
    if (e == E - 1 && !periodic) {
      ghost<EQ>(P, 1, TCp, UR);
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) UR[s] = TR[s];
    }
    interface_flux<EQ, 0>(P.flux, TCp, UR, FR, adv, gam);
    const R iJ = (R)(1.0 / P.Jx);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // f^D at the faces enters through Dt; the interface fluxes through h'
      R fdl = R(0), fdr = R(0);
#pragma unroll
      for (int l = 0; l < n; ++l) {
        fdl += (R)P.tab.lL[l] * F[s][l];
        fdr += (R)P.tab.lR[l] * F[s][l];
      }
#pragma unroll
      for (int j = 0; j < n; ++j) {
        R acc = R(0);
#pragma unroll
        for (int l = 0; l < n; ++l) acc += (R)P.tab.D[j * n + l] * F[s][l];
        acc = acc + (FL[s] - fdl) * (R)P.tab.dhL[j] + (FR[s] - fdr) * (R)P.tab.dhR[j];
        sR[(((long)(ls - 1) * S + s) * n + j) * Nq + q] = (double)(-acc * iJ);
      }
    }
  }
  __syncthreads();

  // 4. projection and stage combination; with an epilogue the output stays in
  // LDS (over the staged input, no longer needed) until the epilogue is done
  double dt;
  if (A.rhs_only) {
    dt = 0.0;
  } else if (A.dt_source == 0) {
    dt = *P.dt;
  } else if (A.dt_source == 3) {
    dt = A.dt_fixed;  // checked and published by the caller
  } else {
    // dt = CFL dx / ((p+1) lambda_max) from the accumulated wave-speed maximum
    dt = A.dt_source == 1 ? A.dt_fixed
                          : P.cfl * P.dx / (P.np1 * __longlong_as_double((long long)*A.lam_in));
    if (blk == 0 && tid == 0) {
      if (!(dt > 0.0) || !isfinite(dt)) atomicOr(P.status, kStatusNonFinite);
      *P.dt = dt;
      if (A.dt_used) *A.dt_used = dt;
      if (A.lam_reset) *A.lam_reset = 0ull;
    }
  }
  // matrix cores: projection of the nodal residual rows (owned element, variable,
  // point) onto the modes, 16 rows x 16 modes per product accumulated over the node
  // blocks; the mean mode in FP64 by one thread per row
  if constexpr (XF) {
    const int prows = nloc * S * n;
    const int RT = (prows + 15) >> 4, KS = NQP >> 4;
    for (int rt = wave; rt < RT; rt += BS / 64) {
      const int r = 16 * rt + li;
      v4f d = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int ks = 0; ks < KS; ++ks) {
        float a[4], b[4];
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int qq = 16 * ks + 4 * lc + it;
          a[it] = (r < prows && qq < Nq) ? (float)sR[(long)r * Nq + qq] : 0.0f;
          b[it] = (li < M && qq < Nq) ? (float)P.tab.PW[li * Nq + qq] : 0.0f;
        }
        v4s ah, al, bh, bl;
        split4(a, ah, al);
        split4(b, bh, bl);
        d = mfma_split(ah, al, bh, bl, d);
      }
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) sPk[(long)(16 * rt + 4 * lc + reg) * 16 + li] = d[reg];
    }
    for (int r = tid; r < prows; r += BS) {
      double a0 = 0.0;
      for (int qq = 0; qq < Nq; ++qq) a0 += P.tab.PW[qq] * sR[(long)r * Nq + qq];
      sP0[r] = a0;
    }
    __syncthreads();
  }
  const bool epi = A.limit || A.end_of_step;
  double* sO = sC;  // [EB][S][M][n] output coefficients
  const int ospan = nloc * n;
  // the combination of the projected residual into the stage output
  auto state_index = [&](int sk, int le, int j) { return (long)sk * EN + (long)(e0 + le) * n + j; };
  auto combine = [&](int sk, int le, int j, double acc, double uv, double wv) {
    double v;
    if (BS < 1024 && A.tab) {  // (the one-workgroup kernel runs SSP-RK3 stages only)
      const long idx = state_index(sk, le, j);
      if (A.k_out) A.k_out[idx] = acc;
      double t = 0.0;
      for (int m = 0; m < A.nt; ++m) t = t + A.ka[m] * A.kk[m][idx];
      if (A.ka_cur != 0.0) t = t + A.ka_cur * acc;
      v = uv + dt * t;
    } else {
      v = A.rhs_only ? acc : A.cu * uv + A.cw * (wv + dt * acc);
    }
    if (epi)
      sO[le * ncoef + sk * n + j] = v;
    else
      A.out[state_index(sk, le, j)] = v;
  };
  if constexpr (XF) {
    for (int it = tid; it < S * M * ospan; it += BS) {
      const int sk = it / ospan, rem = it - sk * ospan;
      const int le = rem / n, j = rem - le * n;
      const int s = sk / M, k = sk - s * M;
      const int r = (le * S + s) * n + j;
      const long idx = state_index(sk, le, j);
      combine(sk, le, j, (k == 0) ? sP0[r] : (double)sPk[(long)r * 16 + k], A.rhs_only ? 0.0 : A.u[idx],
              A.rhs_only ? 0.0 : A.w[idx]);
    }
  } else {
    // thread (variable, block of KB modes, element, point): one pass over the
    // nodal residual feeds KB independent sums, each taking the nodes in order
    // (so every KB gives the same sums; the one-workgroup kernel, at 128
    // registers per lane, keeps one mode per thread)
    auto project = [&](auto kb_tag) {
      constexpr int KB = decltype(kb_tag)::value;
      const int nkb = (M + KB - 1) / KB;
      for (int it = tid; it < S * nkb * ospan; it += BS) {
        const int skb = it / ospan, rem = it - skb * ospan;
        const int le = rem / n, j = rem - le * n;
        const int s = skb / nkb, k0 = (skb - s * nkb) * KB;
        const double* Rq = sR + (((long)le * S + s) * n + j) * Nq;
        const double* PWk[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) PWk[i] = P.tab.PW + min(k0 + i, M - 1) * Nq;  // clamped: past M unused
        double ad[KB];
        R ar[KB];
        // the combination's inputs, loaded before the sums so that their latency overlaps them
        double uv[KB], wv[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
          ad[i] = 0.0;
          ar[i] = R(0);
          const long idx = state_index(s * M + min(k0 + i, M - 1), le, j);
          uv[i] = A.rhs_only ? 0.0 : A.u[idx];
          wv[i] = A.rhs_only ? 0.0 : A.w[idx];
        }
        for (int qq = 0; qq < Nq; ++qq) {
          const double r = Rq[qq];
#pragma unroll
          for (int i = 0; i < KB; ++i) {
            if (std::is_same<R, double>::value || k0 + i == 0)
              ad[i] += PWk[i][qq] * r;  // FP64 (the mean mode in every precision)
            else
              ar[i] += (R)PWk[i][qq] * (R)r;
          }
        }
#pragma unroll
        for (int i = 0; i < KB; ++i)
          if (k0 + i < M)
            combine(s * M + k0 + i, le, j, (std::is_same<R, double>::value || k0 + i == 0) ? ad[i] : (double)ar[i],
                    uv[i], wv[i]);
      }
    };
    // systems take blocks of six modes where blocks of four would leave part of
    // the tasks to a second pass of the workgroup's threads (the Euler problem
    // with 11 modes and 8 elements per workgroup: 288 tasks of four modes, 192 of
    // six, for 256 threads)
    if constexpr (BS >= 1024)
      project(std::integral_constant<int, 1>{});
    else if constexpr (S == 1)
      project(std::integral_constant<int, 4>{});
    else if (S * ((M + 3) / 4) * ospan > BS && S * ((M + 5) / 6) * ospan <= BS)
      project(std::integral_constant<int, 6>{});
    else
      project(std::integral_constant<int, 4>{});
  }
  if (A.clear_flags)
    for (int it = tid; it < nloc; it += BS) A.clear_flags[e0 + it] = 0;
  if (!epi) return 0.0;
  __syncthreads();

  // 5. element epilogue: thread (owned element le, node q); per-(element, node)
  // partial results go to sP (the trace buffer, free now) and are combined by
  // every thread of the element in the same order
  const bool own = active && ls >= 1 && ls <= nloc;
  const int le = ls - 1;
  double* O = sO + (own ? le : 0) * ncoef;
  constexpr int PS = 2 * S;  // slots per (element, node) in the trace buffer
  double* sP = sTr;          // [EB + 2][Nq][PS]
  double* myP = sP + ((long)ls * Nq + q) * PS;
  auto elemP = [&](int slot, int qq) { return sP[((long)ls * Nq + qq) * PS + slot]; };

  // 5a. detector and modal filter (Sec. 4.2, 4.1): thread q owns chaos mode k = q
  if (A.end_of_step && P.filter != FRSG_FILTER_NONE) {
    const int k = q;
    double ut[S][N];
    double num = 0.0, den = 0.0;
    if (own && k < M) {
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int m = 0; m < n; ++m) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < n; ++j) acc += P.tab.Vinv[m * n + j] * O[(s * M + k) * n + j];
          ut[s][m] = acc;
        }
#pragma unroll
      for (int m = 0; m < n; ++m) {
        const double e2 = ut[0][m] * ut[0][m];
        num += e2 * P.tab.shell[k * n + m];
        den += e2;
      }
    }
    // Lasso strengths (Eq. fStrength) need |u~| of the highest pure spatial
    // mode (owned by thread k = 0) and of the highest chaos mode at spatial
    // mode 0 (thread k = M - 1); they pass through sR, free since step 4
    double* la = sR + (long)(own ? le : 0) * 2 * S;
    if (P.filter == FRSG_FILTER_LASSO && own) {
      if (k == 0)
#pragma unroll
        for (int s = 0; s < S; ++s) la[s] = fabs(ut[s][n - 1]);
      if (k == M - 1)
#pragma unroll
        for (int s = 0; s < S; ++s) la[S + s] = fabs(ut[s][0]);
    }
    if (own) {
      myP[0] = num;
      myP[1] = den;
    }
    __syncthreads();
    bool flag = false;
    if (own) {
      double tn = 0.0, td = 0.0;
      for (int qq = 0; qq < M; ++qq) {
        tn += elemP(0, qq);
        td += elemP(1, qq);
      }
      flag = (P.sensor == FRSG_SENSOR_ALWAYS) || (td > 0.0 && tn / td > P.sensor_thr);
      if (flag && k < M) {
        if (P.filter == FRSG_FILTER_LASSO) {
          // Eq. LassoFilterFunction: soft threshold of every (spatial, chaos)
          // coefficient; filt holds ||Psi_m Phi_k||_1
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const double a1 = la[s] / ((double)(n * (n - 1)) * P.tab.filt[n - 1]);
            const double a2 = (M > 1) ? la[S + s] / ((double)((M - 1) * M) * P.tab.filt[(M - 1) * n]) : 0.0;
#pragma unroll
            for (int m = 0; m < n; ++m) {
              const double pen = (a1 * (double)(m * (m + 1)) + a2 * (double)(k * (k + 1))) * P.tab.filt[k * n + m];
              const double au = fabs(ut[s][m]);
              const double f = (au > 0.0) ? 1.0 - pen / au : 0.0;
              ut[s][m] = (f > 0.0 ? f : 0.0) * ut[s][m];
            }
#pragma unroll
            for (int j = 0; j < n; ++j) {
              double acc = 0.0;
#pragma unroll
              for (int m = 0; m < n; ++m) acc += P.tab.V[j * n + m] * ut[s][m];
              O[(s * M + k) * n + j] = acc;
            }
          }
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < n; ++j) {
              double acc = 0.0;
#pragma unroll
              for (int m = 0; m < n; ++m) {
                const double f = P.tab.filt[k * n + m];
                const double lam = (P.filter == FRSG_FILTER_EXP) ? exp(-P.alpha * dt * f) : f;
                acc += P.tab.V[j * n + m] * (ut[s][m] * lam);
              }
              O[(s * M + k) * n + j] = acc;
            }
        }
      }
      if (q == 0 && A.flag_filt) A.flag_filt[e0 + le] = flag ? 1 : 0;
    }
    __syncthreads();
  } else if (A.end_of_step && A.flag_filt) {
    if (own && q == 0) A.flag_filt[e0 + le] = 0;
  }

  // nodal values of the output at node q: the limiter forms them, and the CFL
  // maximum takes them where the limiter left the element as it was (the same
  // sums in the same order as its own expansion)
  double Usp[S][N];
  bool usp_ok = false;

  // 5b. positivity limiter (Sec. 4.3): minimum of density and pressure over the
  // solution and face points at node q, then over the element's nodes
  if constexpr (S > 1) {
    if (A.limit) {
      const double g = P.gamma;
      double ub[S];
      bool realizable = false;
      double eps = 0.0;
      // values at node q: the n solution points, then the two faces by interpolation
      double Ufc[S][2];
      auto point = [&](int pt, double* U) {  // pt < n: solution point; n, n+1: faces
#pragma unroll
        for (int s = 0; s < S; ++s) U[s] = pt < n ? Usp[s][pt] : Ufc[s][pt - n];
      };
      if (own) {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int j = 0; j < n; ++j) Usp[s][j] = 0.0;
        for (int k = 0; k < M; ++k) {
          const double phi = P.tab.Phi[k * Nq + q];
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < n; ++j) Usp[s][j] += O[(s * M + k) * n + j] * phi;
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
          double a = 0.0, b = 0.0;
#pragma unroll
          for (int j = 0; j < n; ++j) {
            a += P.tab.lL[j] * Usp[s][j];
            b += P.tab.lR[j] * Usp[s][j];
          }
          Ufc[s][0] = a;
          Ufc[s][1] = b;
        }
      }
      if (own) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < n; ++j) acc += O[(s * M) * n + j] * P.tab.swts[j];
          ub[s] = acc;
        }
        const double pb = pressure<EQ>(ub, g);
        bool finite = true;
#pragma unroll
        for (int s = 0; s < S; ++s) finite = finite && isfinite(ub[s]);
        realizable = ub[0] > 0.0 && pb > 0.0 && finite;
        if (!realizable && q == 0) atomicOr(P.status, kStatusNotRealizable);
        eps = fmin(1e-8, fmin(ub[0], pb));
        double rmin = INFINITY, pmin = INFINITY;
        if (realizable)
#pragma unroll
          for (int pt = 0; pt < n + 2; ++pt) {
            double U[S];
            point(pt, U);
            rmin = fmin(rmin, U[0]);
            pmin = fmin(pmin, pressure<EQ>(U, g));
          }
        myP[0] = rmin;
        myP[1] = pmin;
      }
      __syncthreads();
      bool on = false;
      double beta1 = 1.0;
      if (own && realizable) {
        double rmin = INFINITY, pmin = INFINITY;
        for (int qq = 0; qq < Nq; ++qq) {
          rmin = fmin(rmin, elemP(0, qq));
          pmin = fmin(pmin, elemP(1, qq));
        }
        on = fmin(rmin, pmin) < eps;
        if (on) {
          beta1 = (rmin >= eps) ? 1.0 : (ub[0] - eps) / (ub[0] - rmin);
          double bmin = 1.0;
#pragma unroll
          for (int pt = 0; pt < n + 2; ++pt) {
            double U[S];
            point(pt, U);
            U[0] = beta1 * (U[0] - ub[0]) + ub[0];
            if (pressure<EQ>(U, g) < eps) bmin = fmin(bmin, pressure_root<EQ>(ub, U, eps, g));
          }
          myP[2] = bmin;
        }
      }
      __syncthreads();
      if (own && on) {
        double beta2 = 1.0;
        for (int qq = 0; qq < Nq; ++qq) beta2 = fmin(beta2, elemP(2, qq));
        for (int it = q; it < S * M * n; it += Nq) {
          const int s = it / (M * n), k = (it / n) % M;
          const double m0 = (k == 0) ? 1.0 : 0.0;
          double v = O[it];
          if (s == 0) v = beta1 * (v - ub[0] * m0) + ub[0] * m0;
          O[it] = beta2 * (v - ub[s] * m0) + ub[s] * m0;
        }
      }
      if (own && q == 0 && A.flag_lim && !(A.flag_or && !on)) A.flag_lim[e0 + le] = on ? 1 : 0;
      usp_ok = own && !on;
      __syncthreads();
    }
  }

  // 5c. CFL maximum of the output for the next step
  double lam_out = 0.0;
  if (A.end_of_step && A.cfl_out) {
    __shared__ double sm[BS / 64];
    double rate = 0.0;
    if (own) {
      if (!usp_ok) {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int j = 0; j < n; ++j) Usp[s][j] = 0.0;
        for (int k = 0; k < M; ++k) {
          const double phi = P.tab.Phi[k * Nq + q];
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < n; ++j) Usp[s][j] += O[(s * M + k) * n + j] * phi;
        }
      }
#pragma unroll
      for (int j = 0; j < n; ++j) {
        double U[S];
#pragma unroll
        for (int s = 0; s < S; ++s) U[s] = Usp[s][j];
        double r = speed<EQ, 0>(U, P.adv, P.gamma);
        if (!(r == r)) r = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf, dt -> 0
        rate = fmax(rate, r);
      }
    }
    // the maximum over the wave, then over the waves (exact in any order: no NaN)
    for (int o = 32; o > 0; o >>= 1) rate = fmax(rate, __shfl_xor(rate, o));
    if ((tid & 63) == 0) sm[tid >> 6] = rate;
    __syncthreads();
    lam_out = sm[0];
    for (int w = 1; w < BS / 64; ++w) lam_out = fmax(lam_out, sm[w]);
    if (tid == 0 && A.lam_next) atomicMax(A.lam_next, (unsigned long long)__double_as_longlong(lam_out));
  }

  // 6. output
  for (int it = tid; it < S * M * ospan; it += BS) {
    const int sk = it / ospan, rem = it - sk * ospan;
    const int le2 = rem / n, j = rem - le2 * n;
    A.out[(long)sk * EN + (long)(e0 + le2) * n + j] = sO[le2 * ncoef + sk * n + j];
  }
  return lam_out;
}

template <int EQ, int N, typename R, int XF>
__global__ void __launch_bounds__(kBlock1) k_stage1d(KParams P, Stage1DArgs A) {
  stage1d_block<EQ, N, R, XF, kBlock1>(P, A, blockIdx.x);
}


// CFL maximum of a 1D state: a workgroup stages the coefficients of 256 / Nq
// elements in LDS; thread (element, node q) takes the maximum over the points
template <int EQ>
__global__ void __launch_bounds__(kBlock1) k_cfl1d(KParams P, const double* __restrict__ u, int EB,
                                                   unsigned long long* lam) {
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
  if (threadIdx.x == 0) atomicMax(lam, (unsigned long long)__double_as_longlong(sm[0]));
}

__global__ void k_zero_lam(unsigned long long* lam) { *lam = 0ull; }

// Several SSP-RK3 steps of a small 1D problem in one launch.  One workgroup of
// kBlockRes threads covers every element ((E + 2) element slots x N_q nodes <=
// kBlockRes) and runs the three stages of each step back to back with the
// stage code of k_stage1d, the stages separated by workgroup barriers.  Where
// they fit, the state and the two stage states live in LDS for the whole call
// (u is read once at the start and written once at the end); otherwise a stage
// writes its output to global memory and the next stage, on the same compute
// unit, reads it after the barrier.  The CFL maximum of each step's output stays
// in the workgroup and sets the next step's dt.  Per element the arithmetic, and
// so the result, is that of the three launches per step.
constexpr int kBlockRes = 1024;

struct Resident1DArgs {
  double* u;                         // state, advanced in place
  double* w1;                        // first and second stage states (global variant)
  double* w2;
  int nsteps;
  int limit;                         // positivity limiter on every stage output
  unsigned char* flags;              // [nsteps][4][E] or null
  double* dt_used;                   // [nsteps] or null
  const unsigned long long* lam_in;  // CFL maximum of u on entry
  unsigned long long* lam_out;       // CFL maximum of the final state
  long lds_tab;                      // offset in doubles of the LDS copies of Phi and PW
  long lds_state;                    // > 0: offset in doubles of the three states in LDS
  long nstate;                       // doubles per state
};

template <int EQ, int N>
__global__ void __launch_bounds__(kBlockRes) k_steps1d_resident(KParams P0, Resident1DArgs RA) {
  extern __shared__ double smem_res[];
  // the chaos tables are read with per-thread indices inside loops over the
  // modes and nodes: one workgroup cannot hide their cache latency, so they are
  // read from LDS copies
  KParams P = P0;
  {
    double* sPhi = smem_res + RA.lds_tab;
    double* sPW = sPhi + P.M * P.Nq;
    for (int i = threadIdx.x; i < P.M * P.Nq; i += kBlockRes) {
      sPhi[i] = P0.tab.Phi[i];
      sPW[i] = P0.tab.PW[i];
    }
    P.tab.Phi = sPhi;
    P.tab.PW = sPW;
  }
  double *u = RA.u, *w1 = RA.w1, *w2 = RA.w2;
  if (RA.lds_state > 0) {
    double* base = smem_res + RA.lds_state;
    for (long i = threadIdx.x; i < RA.nstate; i += kBlockRes) base[i] = RA.u[i];
    u = base;
    w1 = base + RA.nstate;
    w2 = base + 2 * RA.nstate;
  }
  __syncthreads();
  // the steps' dt collect in LDS and go out kRing at a time: a global store from
  // inside a stage would hold the next workgroup barrier until it completes
  constexpr int kRing = 256;
  __shared__ double sdt[kRing];
  double lam = __longlong_as_double((long long)*RA.lam_in);
  double dt = 0.0;
  const long fl = 4l * P.E;
  const bool clear = !RA.limit;
  for (int step = 0; step < RA.nsteps; ++step) {
    // the expression of the stage kernel's CFL time step
    dt = P.cfl * P.dx / (P.np1 * lam);
    if (threadIdx.x == 0) {
      if (!(dt > 0.0) || !isfinite(dt)) atomicOr(P.status, kStatusNonFinite);
      sdt[step % kRing] = dt;
    }
    unsigned char* f = RA.flags ? RA.flags + step * fl : nullptr;
    for (int st = 0; st < 3; ++st) {
      Stage1DArgs A{};
      A.u = u;
      A.EB = P.E;
      A.limit = RA.limit;
      A.dt_source = 3;
      A.dt_fixed = dt;
      unsigned char* fs = f ? f + (st == 2 ? 3 : st) * (long)P.E : nullptr;
      A.clear_flags = clear ? fs : nullptr;
      A.flag_lim = fs;
      if (st == 0) {
        A.in = u, A.w = u, A.out = w1, A.cu = 0.0, A.cw = 1.0;
      } else if (st == 1) {
        A.in = w1, A.w = w1, A.out = w2, A.cu = 0.75, A.cw = 0.25;
      } else {
        A.in = w2, A.w = w2, A.out = u, A.cu = 1.0 / 3.0, A.cw = 2.0 / 3.0;
        A.end_of_step = 1;
        A.cfl_out = 1;
        A.flag_filt = f ? f + 2 * (long)P.E : nullptr;
      }
      const double r = stage1d_block<EQ, N, double, 0, kBlockRes>(P, A, 0);
      if (st == 2) lam = r;
      __syncthreads();
    }
    if (step % kRing == kRing - 1 || step == RA.nsteps - 1) {
      const int first = step - step % kRing;
      if (RA.dt_used && (int)threadIdx.x <= step - first) RA.dt_used[first + threadIdx.x] = sdt[threadIdx.x];
      __syncthreads();
    }
  }
  if (RA.lds_state > 0)
    for (long i = threadIdx.x; i < RA.nstate; i += kBlockRes) RA.u[i] = u[i];
  if (threadIdx.x == 0) {
    if (RA.nsteps > 0) *P.dt = dt;
    *RA.lam_out = (unsigned long long)__double_as_longlong(lam);
  }
}

}  // namespace

// elements per workgroup and LDS bytes; EB = 0 when the node count does not fit
// LDS of a stage over EB elements (plus one neighbour on each side)
static size_t fr1d_lds(const KParams& P, int EB) {
  const size_t ncoef = (size_t)P.S * P.M * P.np1;
  size_t shmem =
      sizeof(double) * ((EB + 2) * ncoef + (size_t)(EB + 2) * P.Nq * 2 * P.S + (size_t)EB * P.S * P.np1 * P.Nq);
  if (P.bf16) {  // matrix-core operands: one block of 16 modes
    const int rows = P.S * P.np1;
    shmem += sizeof(double) * (size_t)EB * rows +
             sizeof(float) * ((size_t)pad16((EB + 2) * rows) * pad16(P.Nq) + (size_t)pad16(EB * rows) * 16);
    if (P.M > 16) shmem = ~(size_t)0;
  }
  return shmem;
}

static void fr1d_shape(const KParams& P, int& EB, size_t& shmem) {
  EB = kBlock1 / P.Nq - 2;
  if (EB < 1 || P.np1 > kMaxN) {
    EB = 0;
    shmem = 0;
    return;
  }
  shmem = fr1d_lds(P, EB);
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

static hipError_t go_stage1d(const KParams& P, Stage1DArgs A, hipStream_t s);

hipError_t launch_stage1d(const KParams& P, const double* in, const double* u, const double* w, double* out, double cu,
                          double cw, int rhs_only, unsigned char* clear_flags, hipStream_t s, int limit,
                          int end_of_step, unsigned char* flag_lim, unsigned char* flag_filt,
                          unsigned long long* lam_next, int dt_source, double dt_fixed,
                          const unsigned long long* lam_in, unsigned long long* lam_reset, double* dt_used) {
  Stage1DArgs A{};
  A.in = in, A.u = u, A.w = w, A.out = out, A.cu = cu, A.cw = cw, A.rhs_only = rhs_only;
  A.clear_flags = clear_flags, A.limit = limit, A.end_of_step = end_of_step;
  A.flag_lim = flag_lim, A.flag_filt = flag_filt, A.cfl_out = lam_next != nullptr, A.lam_next = lam_next;
  A.dt_source = dt_source, A.dt_fixed = dt_fixed, A.lam_in = lam_in, A.lam_reset = lam_reset, A.dt_used = dt_used;
  return go_stage1d(P, A, s);
}

hipError_t launch_stage1d_tab(const KParams& P, const double* in, const double* u, double* out, double* k_out,
                              const RkTerms& T, double ka_cur, hipStream_t s, int limit, int end_of_step,
                              unsigned char* flag_lim, unsigned char* flag_filt, unsigned long long* lam_next,
                              int dt_source, double dt_fixed, const unsigned long long* lam_in,
                              unsigned long long* lam_reset, double* dt_used) {
  if (T.n < 0 || T.n > kRkMaxTerms) return hipErrorInvalidValue;
  Stage1DArgs A{};
  A.in = in, A.u = u, A.w = u, A.out = out;
  A.tab = 1, A.nt = T.n, A.ka_cur = ka_cur, A.k_out = k_out;
  for (int m = 0; m < T.n; ++m) A.kk[m] = T.K[m], A.ka[m] = T.a[m];
  A.limit = limit, A.end_of_step = end_of_step, A.flag_lim = flag_lim, A.flag_or = 1, A.flag_filt = flag_filt;
  A.cfl_out = lam_next != nullptr, A.lam_next = lam_next;
  A.dt_source = dt_source, A.dt_fixed = dt_fixed, A.lam_in = lam_in, A.lam_reset = lam_reset, A.dt_used = dt_used;
  return go_stage1d(P, A, s);
}

static hipError_t go_stage1d(const KParams& P, Stage1DArgs A, hipStream_t s) {
  int EB;
  size_t shmem;
  fr1d_shape(P, EB, shmem);
  if (EB == 0) return hipErrorInvalidValue;
  A.EB = EB;
  const unsigned grid = (unsigned)((P.E + EB - 1) / EB);
  auto go = [&](auto eq_tag) -> hipError_t {
    constexpr int EQ = decltype(eq_tag)::value;
    if (P.bf16) {
      switch (P.np1) {
#define FRSG_N(NN) \
  case NN: hipLaunchKernelGGL((k_stage1d<EQ, NN, float, 1>), dim3(grid), dim3(kBlock1), shmem, s, P, A); break;
        FRSG_N(2) FRSG_N(3) FRSG_N(4) FRSG_N(5) FRSG_N(6) FRSG_N(7) FRSG_N(8)
#undef FRSG_N
        default: return hipErrorInvalidValue;
      }
    } else if (P.fp32) {
      switch (P.np1) {
#define FRSG_N(NN) \
  case NN: hipLaunchKernelGGL((k_stage1d<EQ, NN, float, 0>), dim3(grid), dim3(kBlock1), shmem, s, P, A); break;
        FRSG_N(2) FRSG_N(3) FRSG_N(4) FRSG_N(5) FRSG_N(6) FRSG_N(7) FRSG_N(8)
#undef FRSG_N
        default: return hipErrorInvalidValue;
      }
    } else {
      switch (P.np1) {
#define FRSG_N(NN) \
  case NN: hipLaunchKernelGGL((k_stage1d<EQ, NN, double, 0>), dim3(grid), dim3(kBlock1), shmem, s, P, A); break;
        FRSG_N(2) FRSG_N(3) FRSG_N(4) FRSG_N(5) FRSG_N(6) FRSG_N(7) FRSG_N(8)
#undef FRSG_N
        default: return hipErrorInvalidValue;
      }
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

// the one-workgroup multi-step kernel: FP64 scalar equations of FR degree <= 3
// (at 1024 threads a lane has 128 registers; the Euler and higher-degree
// instances would spill), every element and its neighbours in one workgroup, the
// stage LDS plus the CFL reduction's within 64 KB; the three states join them in
// LDS where that stays within 64 KB
constexpr int kMaxNRes = 4;
constexpr size_t kLdsRes = 64 * 1024;
static size_t fr1d_state_bytes(const KParams& P) { return sizeof(double) * (size_t)P.S * P.M * P.np1 * P.E; }
// stage LDS, the chaos tables' copies, the CFL reduction and the ring of time steps
static size_t fr1d_resident_lds(const KParams& P) {
  return fr1d_lds(P, P.E) + sizeof(double) * (2 * (size_t)P.M * P.Nq + kBlockRes / 64 + 256);
}
bool fr1d_resident_fits(const KParams& P) {
  if (P.dim != 1 || P.fp32 || P.bf16 || P.eq == kEuler1 || P.np1 < 2 || P.np1 > kMaxNRes) return false;
  if ((long)(P.E + 2) * P.Nq > kBlockRes) return false;
  return fr1d_resident_lds(P) <= kLdsRes;
}
bool fr1d_resident_lds_state(const KParams& P) {
  return fr1d_resident_fits(P) && fr1d_resident_lds(P) + 3 * fr1d_state_bytes(P) <= kLdsRes;
}

template <int EQ, int N>
static hipError_t go_resident(const KParams& P, const Resident1DArgs& RA, size_t shmem, hipStream_t s,
                              bool check_only) {
  if (check_only) {
    hipFuncAttributes fa;
    const hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_steps1d_resident<EQ, N>));
    if (e != hipSuccess) return e;
    return fa.localSizeBytes == 0 ? hipSuccess : hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((k_steps1d_resident<EQ, N>), dim3(1), dim3(kBlockRes), shmem, s, P, RA);
  return hipGetLastError();
}

// with u == nullptr only checks that the instance for P runs without register
// spills (hipErrorInvalidValue otherwise)
hipError_t launch_steps1d_resident(const KParams& P, double* u, double* w1, double* w2, int nsteps, int limit,
                                   unsigned char* flags, double* dt_used, const unsigned long long* lam_in,
                                   unsigned long long* lam_out, hipStream_t s) {
  if (!fr1d_resident_fits(P)) return hipErrorInvalidValue;
  const bool check_only = u == nullptr;
  const bool in_lds = fr1d_resident_lds_state(P);
  const long stage = (long)(fr1d_lds(P, P.E) / sizeof(double)), tab = 2l * P.M * P.Nq;
  const Resident1DArgs RA{u,      w1,     w2,      nsteps, limit, flags, dt_used, lam_in, lam_out, stage,
                          in_lds ? stage + tab : 0l, (long)(fr1d_state_bytes(P) / sizeof(double))};
  const size_t shmem = sizeof(double) * (stage + tab) + (in_lds ? 3 * fr1d_state_bytes(P) : 0);
  auto go = [&](auto eq_tag) -> hipError_t {
    constexpr int EQ = decltype(eq_tag)::value;
    switch (P.np1) {
      case 2: return go_resident<EQ, 2>(P, RA, shmem, s, check_only);
      case 3: return go_resident<EQ, 3>(P, RA, shmem, s, check_only);
      case 4: return go_resident<EQ, 4>(P, RA, shmem, s, check_only);
      default: return hipErrorInvalidValue;
    }
  };
  switch (P.eq) {
    case kAdvection: return go(std::integral_constant<int, kAdvection>{});
    case kBurgers: return go(std::integral_constant<int, kBurgers>{});
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cfl1d(const KParams& P, const double* u, unsigned long long* lam, hipStream_t s) {
  const int EB = kBlock1 / P.Nq;  // >= 1 wherever the fused 1D path runs
  if (EB < 1) return hipErrorInvalidValue;
  const size_t shmem = sizeof(double) * (size_t)EB * P.S * P.M * P.np1;
  const unsigned grid = (unsigned)((P.E + EB - 1) / EB);
  hipLaunchKernelGGL(k_zero_lam, dim3(1), dim3(1), 0, s, lam);
  switch (P.eq) {
    case kAdvection: hipLaunchKernelGGL(k_cfl1d<kAdvection>, dim3(grid), dim3(kBlock1), shmem, s, P, u, EB, lam); break;
    case kBurgers: hipLaunchKernelGGL(k_cfl1d<kBurgers>, dim3(grid), dim3(kBlock1), shmem, s, P, u, EB, lam); break;
    case kEuler1: hipLaunchKernelGGL(k_cfl1d<kEuler1>, dim3(grid), dim3(kBlock1), shmem, s, P, u, EB, lam); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace frsg
