// C ABI of the FR-SG hot path: problem validation, tables, workspace and the
// orchestration of the HIP passes for the right-hand side and the SSP-RK3 step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"

using namespace frsg;

namespace {

thread_local std::string g_init_error;

#define FRSG_TRY_HIP(expr, ctx)                                        \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess) {                                            \
      (ctx)->err = std::string("HIP error: ") + hipGetErrorString(e_); \
      return FRSG_EDEVICE;                                             \
    }                                                                  \
  } while (0)

int nstates(int eq) { return eq <= FRSG_BURGERS ? 1 : (eq == FRSG_EULER1D ? 3 : 4); }

// Explicit Runge-Kutta tableaux of the paper's integrators (RK4, Table 1;
// Tsitouras 5(4), Table 4; Bogacki-Shampine 3(2), Tables 5, 6), used at the
// CFL step: the propagating weights only (the first-same-as-last stage of the
// embedded pairs serves the error estimate and is left out).
struct Tableau {
  int s;
  double A[kRkMaxTerms][kRkMaxTerms];
  double b[kRkMaxTerms];
};
const Tableau kRK4 = {4,
                      {{0}, {0.5}, {0.0, 0.5}, {0.0, 0.0, 1.0}},
                      {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}};
const Tableau kBS3 = {3, {{0}, {0.5}, {0.0, 0.75}}, {2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0}};
const Tableau kTsit5 = {6,
                        {{0},
                         {0.161},
                         {-0.008480655492356989, 0.335480655492357},
                         {2.897153057105493, -6.359448489975075, 4.3622954328695815},
                         {5.325864828439257, -11.748883564062828, 7.4955393428898365, -0.09249506636175525},
                         {5.86145544294642, -12.92096931784711, 8.159367898576159, -0.071584973281401,
                          -0.028269050394068383}},
                        {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742, -3.290069515436081,
                         2.324710524099774}};
const Tableau* tableau_of(int integrator) {
  switch (integrator) {
    case FRSG_RK4: return &kRK4;
    case FRSG_RK_BS3: return &kBS3;
    case FRSG_RK_TSIT5: return &kTsit5;
    default: return nullptr;
  }
}

fr_sg_status validate(const fr_sg_problem& P, std::string& err) {
  if (P.abi_version != FRSG_ABI_VERSION) {
    err = "abi_version mismatch";
    return FRSG_EABI;
  }
  if (P.equation < FRSG_ADVECTION || P.equation > FRSG_EULER2D) {
    err = "unknown equation";
    return FRSG_EINVAL;
  }
  const int dim = P.equation == FRSG_EULER2D ? 2 : 1;
  if (P.fr_degree < 1 || P.fr_degree > kMaxNp1 - 1) {
    err = "fr_degree must be in 1..7";
    return P.fr_degree < 1 ? FRSG_EINVAL : FRSG_EUNSUPPORTED;
  }
  if (P.element != FRSG_ELEM_QUAD && P.element != FRSG_ELEM_TRI) {
    err = "unknown element shape";
    return FRSG_EINVAL;
  }
  const bool tri = P.element == FRSG_ELEM_TRI;
  if (tri) {
    if (P.equation != FRSG_EULER2D) {
      err = "triangles carry the 2D Euler equations";
      return FRSG_EUNSUPPORTED;
    }
    if (P.n_tri < 1 || !P.tri_xy || !P.tri_nbr || !P.tri_nbr_face) {
      err = "a triangle mesh needs n_tri >= 1 and its vertex and neighbour arrays";
      return FRSG_EINVAL;
    }
    if (P.fr_degree > kTriMaxDeg) {
      err = "fr_degree must be in 1..4 on triangles";
      return FRSG_EUNSUPPORTED;
    }
    if (P.precision != FRSG_FP64) {
      err = "triangles run in FP64 only (no FP32-mixed or BF16-split)";
      return FRSG_EUNSUPPORTED;
    }
  } else {
    if (P.nx < 1 || (dim == 2 && P.ny < 1)) {
      err = "element counts must be positive";
      return FRSG_EINVAL;
    }
    if (!(P.xhi > P.xlo) || (dim == 2 && !(P.yhi > P.ylo))) {
      err = "empty domain";
      return FRSG_EINVAL;
    }
  }
  if (P.rdim != 1 && P.rdim != 2) {
    err = "rdim must be 1 or 2";
    return FRSG_EINVAL;
  }
  if (P.gpc_order < 0 || P.nq1d < P.gpc_order + 1) {
    err = "need gpc_order >= 0 and nq1d >= gpc_order + 1";
    return FRSG_EINVAL;
  }
  const long M = P.rdim == 1 ? P.gpc_order + 1 : (long)(P.gpc_order + 1) * (P.gpc_order + 2) / 2;
  const long Nq = P.rdim == 1 ? P.nq1d : (long)P.nq1d * P.nq1d;
  if (M > kMaxModes || Nq > kMaxNodes) {
    err = "too many gPC modes or random nodes";
    return FRSG_EUNSUPPORTED;
  }
  const long E = tri ? (long)P.n_tri : (long)P.nx * (dim == 2 ? P.ny : 1);
  const long nsp = tri ? (long)(P.fr_degree + 1) * (P.fr_degree + 2) / 2
                       : (dim == 2 ? (long)(P.fr_degree + 1) * (P.fr_degree + 1) : P.fr_degree + 1);
  if (E * nsp * Nq > (1l << 31) / 4) {
    err = "problem too large for 32-bit node indexing";
    return FRSG_EUNSUPPORTED;
  }
  for (int side = 0; side < 2 * dim; ++side) {
    const int k = P.bc[side];
    if (k < FRSG_BC_PERIODIC || k > FRSG_BC_REFLECT) {
      err = "unknown boundary kind";
      return FRSG_EINVAL;
    }
    if (k == FRSG_BC_REFLECT && P.equation < FRSG_EULER1D) {
      err = "reflecting boundaries need the Euler equations";
      return FRSG_EUNSUPPORTED;
    }
  }
  for (int d = 0; d < (tri ? 0 : dim); ++d)
    if ((P.bc[2 * d] == FRSG_BC_PERIODIC) != (P.bc[2 * d + 1] == FRSG_BC_PERIODIC)) {
      err = "periodic boundaries must be paired";
      return FRSG_EINVAL;
    }
  if (P.integrator < FRSG_SSPRK3 || P.integrator > FRSG_RK_TSIT5) {
    err = "unknown integrator";
    return FRSG_EINVAL;
  }
  if (P.flux != FRSG_FLUX_RUSANOV && P.flux != FRSG_FLUX_HLL) {
    err = "unknown interactive flux";
    return FRSG_EINVAL;
  }
  if (P.flux == FRSG_FLUX_HLL && P.equation < FRSG_EULER1D) {
    err = "the HLL flux is available for the Euler equations";
    return FRSG_EUNSUPPORTED;
  }
  if (P.filter < FRSG_FILTER_NONE || P.filter > FRSG_FILTER_LASSO) {
    err = "unknown filter";
    return FRSG_EINVAL;
  }
  if (P.filter == FRSG_FILTER_LASSO && (dim != 1 || P.rdim != 1)) {
    err = "the Lasso filter is available for one physical and one random dimension";
    return FRSG_EUNSUPPORTED;
  }
  if (P.filter == FRSG_FILTER_EXP && !(P.alpha >= 0.0 && P.s > 0.0)) {
    err = "exponential filter needs alpha >= 0 and s > 0";
    return FRSG_EINVAL;
  }
  if (P.filter == FRSG_FILTER_EXP &&
      !(P.nstar >= 0.0 && P.nstar < P.fr_degree && (P.gpc_order == 0 || P.nstar < P.gpc_order))) {
    err = "exponential filter cutoff needs 0 <= nstar < p and nstar < gpc_order";
    return FRSG_EINVAL;
  }
  if (P.filter == FRSG_FILTER_L2 && !(P.eps1 > 0.0 && P.eps2 > 0.0)) {
    err = "L2 filter needs eps1, eps2 > 0";
    return FRSG_EINVAL;
  }
  if (P.sensor != FRSG_SENSOR_ALWAYS && P.sensor != FRSG_SENSOR_DETECTOR) {
    err = "unknown sensor";
    return FRSG_EINVAL;
  }
  if (P.sensor == FRSG_SENSOR_DETECTOR && !(P.kappa > 0.0)) {
    err = "detector needs kappa > 0";
    return FRSG_EINVAL;
  }
  if (P.limiter != 0 && P.limiter != 1) {
    err = "limiter must be 0 or 1";
    return FRSG_EINVAL;
  }
  if (P.limiter && P.equation < FRSG_EULER1D) {
    err = "the positivity limiter applies to the Euler equations only";
    return FRSG_EUNSUPPORTED;
  }
  if (P.equation >= FRSG_EULER1D && !(P.gamma > 1.0)) {
    err = "gamma must exceed 1";
    return FRSG_EINVAL;
  }
  if (!(P.cfl > 0.0)) {
    err = "cfl must be positive";
    return FRSG_EINVAL;
  }
  if (P.precision != FRSG_FP64 && P.precision != FRSG_FP32_MIXED && P.precision != FRSG_BF16_SPLIT) {
    err = "unknown precision";
    return FRSG_EINVAL;
  }
  return FRSG_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

int take_event(fr_sg_ctx* c) {
  if (c->events_used == (int)c->events.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return -1;
    c->events.push_back(ev);
  }
  return c->events_used++;
}

// Launch one pass; when timing is on, bracket it with events on the stream.
fr_sg_status timed(fr_sg_ctx* c, const char* name, double alg_bytes, const std::function<hipError_t()>& launch) {
  int e0 = -1, e1 = -1;
  if (c->timing) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 < 0 || e1 < 0 || hipEventRecord(c->events[e0], c->stream) != hipSuccess) {
      c->err = "event creation/record failed";
      return FRSG_EDEVICE;
    }
  }
  hipError_t e = launch();
  if (e != hipSuccess) {
    c->err = std::string(name) + ": " + hipGetErrorString(e);
    return FRSG_EDEVICE;
  }
  if (c->timing) {
    if (hipEventRecord(c->events[e1], c->stream) != hipSuccess) {
      c->err = "event record failed";
      return FRSG_EDEVICE;
    }
    c->pending.push_back({name, alg_bytes, e0, e1});
  }
  return FRSG_OK;
}

double state_bytes(const fr_sg_ctx* c) { return 8.0 * c->S * c->T.M * (double)c->E * c->nsp; }

int fp32(const fr_sg_ctx* c) { return c->prob.precision == FRSG_FP32_MIXED ? 1 : 0; }

}  // namespace

// Host-side preparation shared by fr_sg_workspace_size and fr_sg_init: validate
// the problem, build the operator tables, choose the kernel path and lay out the
// caller's workspace.  Makes no HIP call.
static fr_sg_status prepare(const fr_sg_problem& problem, fr_sg_ctx* c, std::string& err) {
  fr_sg_status st = validate(problem, err);
  if (st != FRSG_OK) return st;
  c->prob = problem;
  if (!build_host_tables(c->prob, c->T, err)) return FRSG_EINVAL;
  const fr_sg_problem& P = c->prob;
  c->is_tri = P.element == FRSG_ELEM_TRI;
  if (c->is_tri && !build_tri_tables(P, c->tri, err)) return FRSG_EINVAL;
  if (c->is_tri) tri_filter_tables(P, c->tri, c->T);
  // the mesh arrays are the caller's and are read during this call only
  c->prob.tri_xy = nullptr;
  c->prob.tri_nbr = nullptr;
  c->prob.tri_nbr_face = nullptr;
  c->dim = P.equation == FRSG_EULER2D ? 2 : 1;
  c->S = nstates(P.equation);
  c->E = c->is_tri ? P.n_tri : P.nx * (c->dim == 2 ? P.ny : 1);
  const int n = P.fr_degree + 1;
  c->nsp = c->is_tri ? c->tri.np : (c->dim == 2 ? n * n : n);
  const HostTables& T = c->T;

  // every operator table in one double array (uploaded into the workspace by init)
  std::vector<double>& blob = c->host_tab;
  blob.clear();
  c->tab_off.clear();
  if (c->dim == 2 && !c->is_tri) build_quad_fragments(c->T);
  for (const std::vector<double>* v : {&T.r, &T.w, &T.D, &T.lL, &T.lR, &T.dhL, &T.dhR, &T.V, &T.Vinv, &T.Phi, &T.PW,
                                       &T.filt, &T.shell, &T.swts, &T.Dt, &T.cmax, &T.PhiT, &T.PWT, &T.qfrag}) {
    c->tab_off.push_back(blob.size());
    blob.insert(blob.end(), v->begin(), v->end());
  }

  // kernel parameters without device pointers (filled in by init)
  KParams& K = c->kp;
  std::memset(&K, 0, sizeof(K));
  K.eq = P.equation;
  K.dim = c->dim;
  K.E = c->E;
  K.nx = c->is_tri ? 1 : P.nx;
  K.ny = (c->dim == 2 && !c->is_tri) ? P.ny : 1;
  K.nsp = c->nsp;
  K.M = T.M;
  K.Nq = T.Nq;
  K.S = c->S;
  K.np1 = n;
  K.dx = c->is_tri ? 1.0 : (P.xhi - P.xlo) / P.nx;
  K.dy = (c->dim == 2 && !c->is_tri) ? (P.yhi - P.ylo) / P.ny : 1.0;
  K.Jx = K.dx / 2.0;
  K.Jy = K.dy / 2.0;
  K.adv = P.adv_speed;
  K.gamma = P.gamma;
  for (int i = 0; i < 4; ++i) {
    K.bc[i] = P.bc[i];
    for (int s = 0; s < 4; ++s) K.bc_state[i][s] = P.bc_state[i][s];
  }
  if (c->dim == 1) K.bc[2] = K.bc[3] = FRSG_BC_PERIODIC;
  K.cfl = P.cfl;
  K.filter = P.filter;
  K.flux = P.flux;
  K.sensor = P.sensor;
  K.limiter = P.limiter;
  K.alpha = P.alpha;
  K.sensor_thr = std::pow(10.0, P.s0 - (2.0 * P.kappa / M_PI) * std::asin(0.98));
  if (c->is_tri) {
    K.tri = 1;
    K.nfp = c->tri.nfp;
  }
  K.fp32 = P.precision == FRSG_FP32_MIXED ? 1 : 0;
  K.bf16 = (P.precision == FRSG_BF16_SPLIT && c->dim == 1) ? 1 : 0;
  c->fused = !c->is_tri && fused2d_supported(K);
  // the matrix-core kernel takes the BF16-split steps of the 2D quadrilateral path (and the
  // FP64 ones where the VALU kernel does not apply)
  c->quad = !c->is_tri && quad_mfma_supported(K) &&
            (P.precision == FRSG_BF16_SPLIT || (P.precision == FRSG_FP64 && !c->fused));
  c->fused_tri = c->is_tri && tri_fused_supported(K);
  c->fused1d = c->dim == 1 && fr1d_supported(K);
  if (P.precision == FRSG_FP32_MIXED && !c->fused && !c->fused1d) {
    err = "FRSG_FP32_MIXED runs on the fused 1D path (FR degree <= 7, Nq <= 85, one block's LDS within "
          "64 KiB) and the fused 2D Euler path (FR degree 3, nx % 4 == 0, ny % 2 == 0, a compiled (M, Nq) pair)";
    return FRSG_EUNSUPPORTED;
  }
  if (P.precision == FRSG_BF16_SPLIT && !c->quad && !(c->dim == 1 && c->fused1d)) {
    err = "FRSG_BF16_SPLIT runs on the matrix-core paths: the 1D stage kernel (at most 16 gPC modes, FR degree "
          "<= 7, Nq <= 85, one block's LDS within 64 KiB) and the 2D Euler quadrilateral kernel (FR degree 3, "
          "nx and ny even, a compiled (M, Nq) pair)";
    return FRSG_EUNSUPPORTED;
  }
  // triangle operators and geometry: one double array and the neighbour table
  c->host_tri.clear();
  if (c->is_tri) {
    const TriTables& R = c->tri;
    for (const std::vector<double>* v : {&R.Dr, &R.Ds, &R.Lf, &R.lift, &R.geo, &R.V, &R.Vinv})
      c->host_tri.insert(c->host_tri.end(), v->begin(), v->end());
  }
  // FP32 copies of the node-major chaos tables (fused 2D path)
  c->host_f32.clear();
  if (c->fused) {
    c->host_f32.resize(2 * T.PhiT.size());
    for (size_t i = 0; i < T.PhiT.size(); ++i) {
      c->host_f32[i] = (float)T.PhiT[i];
      c->host_f32[T.PhiT.size() + i] = (float)T.PWT[i];
    }
  }

  // workspace layout, every sub-array aligned to 256 bytes
  Layout& L = c->lay;
  L = Layout();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t state = (size_t)c->S * T.M * c->E * c->nsp;
  const bool no_nodal = c->fused || c->quad || c->fused_tri;
  const size_t nodal = no_nodal ? 0 : (size_t)c->S * T.Nq * c->E * c->nsp;
  const size_t corr = no_nodal ? 0
                      : (size_t)c->S * T.Nq * c->E * (c->is_tri ? 3 * c->tri.nfp : (c->dim == 2 ? 4 * n : 2));
  const size_t ntm = c->fused_tri ? (size_t)c->S * T.M * c->E * 3 * c->tri.nfp : 0;
  const bool adj = c->dim == 1 && c->S == 1;
  const size_t nadj_part = adj ? (size_t)std::max(adjoint_partials(K), adj1d_partials(K)) : 0;
  const size_t ntr = c->quad ? quad_trace_count(P.nx, P.ny, T.M) : c->fused ? fused2d_trace_count(P.nx, P.ny, T.M) : 0;
  const Tableau* tab_rk = tableau_of(P.integrator);
  const int nrk = tab_rk ? tab_rk->s : 0;
  L.sc = take(256);
  L.tab = take(blob.size() * sizeof(double));
  L.f32 = take(c->host_f32.size() * sizeof(float));
  L.tri = take(c->host_tri.size() * sizeof(double));
  L.nbr = take(c->is_tri ? c->tri.nbr.size() * sizeof(int) : 0);
  L.w1 = take(state * 8);
  L.w2 = take(state * 8);
  L.un = take(nodal * 8);
  L.fn = take(nodal * 8);
  L.gn = take(c->dim == 2 ? nodal * 8 : 0);
  L.co = take(corr * 8);
  L.avb = take(adj ? state * 8 : 0);
  L.ab2 = take(adj ? state * 8 : 0);
  L.ab1 = take(adj ? state * 8 : 0);
  L.agt = take(adj ? (size_t)T.Nq * c->E * 2 * 8 : 0);
  L.apt = take(nadj_part * 8);
  L.tr0 = take(ntr * 8);
  L.tr1 = take(ntr * 8);
  for (int i = 0; i < nrk; ++i) L.rk[i] = take(state * 8);
  L.nrk = nrk;
  L.tm0 = take(ntm * 8);
  L.tm1 = take(ntm * 8);
  L.adj = adj;
  L.has_tr = ntr > 0;
  L.has_tm = ntm > 0;
  L.total = o;
  return FRSG_OK;
}

extern "C" {

fr_sg_status fr_sg_workspace_size(const fr_sg_problem* problem, int64_t* bytes) {
  if (!problem || !bytes) {
    g_init_error = "problem and bytes must not be NULL";
    return FRSG_EINVAL;
  }
  *bytes = 0;
  fr_sg_ctx* c = new (std::nothrow) fr_sg_ctx();
  if (!c) {
    g_init_error = "out of host memory";
    return FRSG_EDEVICE;
  }
  std::string err;
  const fr_sg_status st = prepare(*problem, c, err);
  if (st == FRSG_OK)
    *bytes = (int64_t)c->lay.total;
  else
    g_init_error = err;
  delete c;
  return st;
}

fr_sg_status fr_sg_init(const fr_sg_problem* problem, void* hip_stream, void* workspace, int64_t workspace_bytes,
                        fr_sg_ctx** out) {
  return frsg::init_with_workspace(problem, hip_stream, workspace, workspace_bytes, out, true);
}

}  // extern "C"

void frsg::set_init_error(const std::string& msg) { g_init_error = msg; }

// fr_sg_init on a given workspace (the caller's, or the library's static array)
fr_sg_status frsg::init_with_workspace(const fr_sg_problem* problem, void* hip_stream, void* workspace,
                                       int64_t workspace_bytes, fr_sg_ctx** out, bool check_device) {
  if (!out) {
    g_init_error = "out is NULL";
    return FRSG_EINVAL;
  }
  *out = nullptr;
  if (!problem) {
    g_init_error = "problem is NULL";
    return FRSG_EINVAL;
  }
  fr_sg_ctx* c = new (std::nothrow) fr_sg_ctx();
  if (!c) {
    g_init_error = "out of host memory";
    return FRSG_EDEVICE;
  }
  std::string err;
  fr_sg_status st = prepare(*problem, c, err);
  if (st != FRSG_OK) {
    g_init_error = err;
    delete c;
    return st;
  }
  const Layout& L = c->lay;
  if (!workspace || workspace_bytes < (int64_t)L.total || ((uintptr_t)workspace & 255u) != 0) {
    g_init_error = "workspace must be a 256-byte aligned device buffer of at least " + std::to_string(L.total) +
                   " bytes (fr_sg_workspace_size)";
    delete c;
    return FRSG_EINVAL;
  }
  if (check_device) {
    hipPointerAttribute_t attr;
    const hipError_t pe = hipPointerGetAttributes(&attr, workspace);
    (void)hipGetLastError();  // do not leave the query's status for a later launch check
    if (pe != hipSuccess || attr.type != hipMemoryTypeDevice) {
      g_init_error = "workspace is not device memory";
      delete c;
      return FRSG_EINVAL;
    }
  }
  c->stream = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  // upload the tables into the workspace and clear the device scalars; the host
  // copies stay alive until the stream has finished with them
  hipError_t he = hipMemsetAsync(ws + L.sc, 0, 256, c->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(ws + L.tab, c->host_tab.data(), c->host_tab.size() * sizeof(double), hipMemcpyHostToDevice,
                        c->stream);
  if (he == hipSuccess && !c->host_f32.empty())
    he = hipMemcpyAsync(ws + L.f32, c->host_f32.data(), c->host_f32.size() * sizeof(float), hipMemcpyHostToDevice,
                        c->stream);
  if (he == hipSuccess && !c->host_tri.empty())
    he = hipMemcpyAsync(ws + L.tri, c->host_tri.data(), c->host_tri.size() * sizeof(double), hipMemcpyHostToDevice,
                        c->stream);
  if (he == hipSuccess && c->is_tri)
    he = hipMemcpyAsync(ws + L.nbr, c->tri.nbr.data(), c->tri.nbr.size() * sizeof(int), hipMemcpyHostToDevice,
                        c->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  if (he != hipSuccess) {
    g_init_error = std::string("HIP error: ") + hipGetErrorString(he);
    delete c;
    return FRSG_EDEVICE;
  }
  c->host_tab.clear();
  c->host_tab.shrink_to_fit();
  c->host_f32.clear();
  c->host_f32.shrink_to_fit();
  c->host_tri.clear();
  c->host_tri.shrink_to_fit();

  // device views of the tables
  const double* b = (const double*)(ws + L.tab);
  const std::vector<size_t>& off = c->tab_off;
  DevTab tab;
  tab.r = b + off[0];
  tab.w = b + off[1];
  tab.D = b + off[2];
  tab.lL = b + off[3];
  tab.lR = b + off[4];
  tab.dhL = b + off[5];
  tab.dhR = b + off[6];
  tab.V = b + off[7];
  tab.Vinv = b + off[8];
  tab.Phi = b + off[9];
  tab.PW = b + off[10];
  tab.filt = b + off[11];
  tab.shell = b + off[12];
  tab.swts = b + off[13];
  c->dDt = b + off[14];
  c->dcmax = b + off[15];
  tab.cmax = c->dcmax;
  c->dPhiT = b + off[16];
  c->dPWT = b + off[17];
  tab.PhiT = c->dPhiT;
  tab.PWT = c->dPWT;
  c->dfrag = b + off[18];
  if (c->fused) {
    c->dPhiT32 = (const float*)(ws + L.f32);
    c->dPWT32 = c->dPhiT32 + c->T.PhiT.size();
  }
  KParams& K = c->kp;
  K.tab = tab;
  if (c->is_tri) {
    const TriTables& R = c->tri;
    const double* b2 = (const double*)(ws + L.tri);
    K.tri_Dr = b2;
    K.tri_Ds = K.tri_Dr + R.Dr.size();
    K.tri_Lf = K.tri_Ds + R.Ds.size();
    K.tri_lift = K.tri_Lf + R.Lf.size();
    K.tri_geo = K.tri_lift + R.lift.size();
    K.tri_V = K.tri_geo + R.geo.size();
    K.tri_Vinv = K.tri_V + R.V.size();
    K.tri_nbr = (const int*)(ws + L.nbr);
  }
  Workspace& W = c->ws;
  W.scal = (double*)(ws + L.sc);
  W.w1 = (double*)(ws + L.w1);
  W.w2 = (double*)(ws + L.w2);
  W.Un = (double*)(ws + L.un);
  W.Fn = (double*)(ws + L.fn);
  W.Gn = c->dim == 2 ? (double*)(ws + L.gn) : nullptr;
  W.Corr = (double*)(ws + L.co);
  if (L.adj) {
    W.avb = (double*)(ws + L.avb);
    W.ab2 = (double*)(ws + L.ab2);
    W.ab1 = (double*)(ws + L.ab1);
    W.agT = (double*)(ws + L.agt);
    W.apart = (double*)(ws + L.apt);
  }
  for (int i = 0; i < L.nrk; ++i) W.rk[i] = (double*)(ws + L.rk[i]);
  if (L.has_tm) {
    W.Tm[0] = (double*)(ws + L.tm0);
    W.Tm[1] = (double*)(ws + L.tm1);
  }
  if (L.has_tr) {
    W.tr[0] = (double*)(ws + L.tr0);
    W.tr[1] = (double*)(ws + L.tr1);
  }
  W.bytes = L.total;
  K.dt = W.scal;
  K.lam_bits = (unsigned long long*)(W.scal + 1);
  K.status = (unsigned*)(W.scal + 2);  // scal[3] is the second CFL accumulator
  // small 1D problems run the steps of an fr_sg_steps call in one launch of one
  // workgroup, where the kernel instance needs no register spills
  c->resident1d = c->fused1d && c->prob.integrator == FRSG_SSPRK3 &&
                  launch_steps1d_resident(K, nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr,
                                          c->stream) == hipSuccess;
  (void)hipGetLastError();  // a failed attribute query leaves nothing for a later launch check
  *out = c;
  return FRSG_OK;
}

extern "C" {

fr_sg_status fr_sg_query(const fr_sg_ctx* ctx, fr_sg_info* out) {
  if (!ctx || !out) return FRSG_EINVAL;
  out->n_elem = ctx->E;
  out->nsp = ctx->nsp;
  out->n_modes = ctx->T.M;
  out->n_nodes = ctx->T.Nq;
  out->n_states = ctx->S;
  out->n_dof = (int64_t)ctx->S * ctx->T.M * ctx->E * ctx->nsp;
  out->state_bytes = out->n_dof * 8;
  out->flags_len = 4 * (int64_t)ctx->E;
  out->workspace_bytes = (int64_t)ctx->ws.bytes;
  return FRSG_OK;
}

fr_sg_status fr_sg_set_stream(fr_sg_ctx* ctx, void* hip_stream) {
  if (!ctx) return FRSG_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return FRSG_OK;
}

fr_sg_status fr_sg_points(const fr_sg_ctx* ctx, double* x, double* y, double* z) {
  if (!ctx) return FRSG_EINVAL;
  const KParams& K = ctx->kp;
  const int n = K.np1;
  const fr_sg_problem& P = ctx->prob;
  if (ctx->is_tri) {
    // physical coordinates of the solution points, computed at init (Sec. 3.1 map)
    const TriTables& R = ctx->tri;
    for (int e = 0; e < K.E; ++e)
      for (int j = 0; j < R.np; ++j) {
        if (x) x[(long)e * R.np + j] = R.xy_pts[((long)e * R.np + j) * 2];
        if (y) y[(long)e * R.np + j] = R.xy_pts[((long)e * R.np + j) * 2 + 1];
      }
    if (z)
      for (size_t i = 0; i < ctx->T.z.size(); ++i) z[i] = ctx->T.z[i];
    return FRSG_OK;
  }
  for (int e = 0; e < K.E; ++e) {
    const int ix = e % K.nx, iy = e / K.nx;
    const double xc = P.xlo + (ix + 0.5) * K.dx;
    const double yc = P.ylo + (iy + 0.5) * K.dy;
    for (int j = 0; j < K.nsp; ++j) {
      const int a = j % n, b = j / n;
      if (x) x[(long)e * K.nsp + j] = xc + 0.5 * K.dx * ctx->T.r[a];
      if (y) y[(long)e * K.nsp + j] = ctx->dim == 2 ? yc + 0.5 * K.dy * ctx->T.r[b] : 0.0;
    }
  }
  if (z)
    for (size_t i = 0; i < ctx->T.z.size(); ++i) z[i] = ctx->T.z[i];
  return FRSG_OK;
}

fr_sg_status fr_sg_project(fr_sg_ctx* ctx, const double* u0_nodal, double* u) {
  if (!ctx) return FRSG_EINVAL;
  if (!u0_nodal || !u) {
    ctx->err = "null pointer";
    return FRSG_EINVAL;
  }
  FRSG_TRY_HIP(launch_project_ic(ctx->kp, u0_nodal, u, ctx->stream), ctx);
  return FRSG_OK;
}

fr_sg_status fr_sg_limit(fr_sg_ctx* ctx, double* u, uint8_t* flags) {
  if (!ctx) return FRSG_EINVAL;
  if (!u) {
    ctx->err = "null pointer";
    return FRSG_EINVAL;
  }
  if (ctx->prob.limiter && ctx->fused)
    return timed(ctx, "limiter", 2 * state_bytes(ctx), [&] {
      return launch_fused_post(ctx->kp, ctx->dPhiT, ctx->dcmax, u, 0, 1, nullptr, flags, ctx->stream);
    });
  if (ctx->prob.limiter && ctx->fused_tri)
    return timed(ctx, "limiter", 2 * state_bytes(ctx),
                 [&] { return launch_limit_tri(ctx->kp, u, flags, ctx->stream); });
  if (ctx->prob.limiter)
    return timed(ctx, "limiter", 2 * state_bytes(ctx), [&] { return launch_limiter(ctx->kp, u, flags, ctx->stream); });
  if (flags) FRSG_TRY_HIP(launch_fill_flags(flags, ctx->E, ctx->stream), ctx);
  return FRSG_OK;
}

static fr_sg_status rhs_passes(fr_sg_ctx* ctx, const double* in, int do_cfl) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  fr_sg_status st;
  if (ctx->is_tri) {
    if ((st = timed(ctx, "nodal", state_bytes(ctx), [&] { return launch_nodal(K, in, W.Un, W.Fn, W.Gn, 0, s); })))
      return st;
    if (do_cfl && (st = timed(ctx, "cfl", 0.0, [&] { return launch_cfl_tri(K, W.Un, s); }))) return st;
    if ((st = timed(ctx, "faces", 0.0, [&] { return launch_faces_tri(K, W.Un, W.Fn, W.Gn, W.Corr, s); })))
      return st;
    return timed(ctx, "resid", 0.0, [&] { return launch_resid_tri(K, W.Fn, W.Gn, W.Corr, W.Un, s); });
  }
  if ((st = timed(ctx, "nodal", state_bytes(ctx), [&] { return launch_nodal(K, in, W.Un, W.Fn, W.Gn, do_cfl, s); })))
    return st;
  if ((st = timed(ctx, "faces", 0.0, [&] { return launch_faces(K, W.Un, W.Fn, W.Gn, W.Corr, s); }))) return st;
  return timed(ctx, "resid", 0.0, [&] { return launch_resid(K, W.Fn, W.Gn, W.Corr, W.Un, s); });
}

static fr_sg_status rhs_into(fr_sg_ctx* ctx, const double* u, double* dudt);

fr_sg_status fr_sg_rhs(fr_sg_ctx* ctx, const double* u, double* dudt) {
  if (!ctx) return FRSG_EINVAL;
  if (!u || !dudt || u == dudt) {
    ctx->err = "u and dudt must be distinct device pointers";
    return FRSG_EINVAL;
  }
  return rhs_into(ctx, u, dudt);
}

// the right-hand side of u into dudt with the path's kernels (no CFL maximum)
static fr_sg_status rhs_into(fr_sg_ctx* ctx, const double* u, double* dudt) {
  if (ctx->fused_tri)
    return timed(ctx, "stage_rhs", 2 * state_bytes(ctx), [&] {
      return launch_stage_tri(ctx->kp, u, u, u, dudt, 0.0, 1.0, 1, ctx->ws.Tm[0], 0, nullptr, ctx->stream);
    });
  if (ctx->quad) {
    fr_sg_status st = timed(ctx, "traces", 0.0, [&] { return launch_quad_traces(ctx->kp, u, ctx->ws.tr[0], ctx->stream); });
    if (st != FRSG_OK) return st;
    QuadStage S{u, u, dudt, 0.0, 1.0, 0, nullptr, nullptr, nullptr, ctx->dDt, ctx->dcmax, ctx->dfrag,
                ctx->prob.precision == FRSG_BF16_SPLIT ? 1 : 0, ctx->ws.tr[0], nullptr};
    return timed(ctx, "stage_rhs", 2 * state_bytes(ctx), [&] { return launch_quad_stage(ctx->kp, S, ctx->stream); });
  }
  if (ctx->fused) {
    FusedStage S{u,          u,          dudt,         0.0,         1.0,           0,
                 nullptr,    nullptr,    nullptr,      ctx->dDt,    ctx->dcmax,    ctx->dPhiT,
                 ctx->dPWT,  fp32(ctx),  ctx->dPhiT32, ctx->dPWT32};
    return timed(ctx, "stage_rhs", 2 * state_bytes(ctx), [&] { return launch_fused_stage(ctx->kp, S, ctx->stream); });
  }
  if (ctx->fused1d)
    return timed(ctx, "stage_rhs", 2 * state_bytes(ctx), [&] {
      return launch_stage1d(ctx->kp, u, u, u, dudt, 0.0, 1.0, 1, nullptr, ctx->stream);
    });
  fr_sg_status st = rhs_passes(ctx, u, 0);
  if (st != FRSG_OK) return st;
  return timed(ctx, "project_rhs", state_bytes(ctx),
               [&] { return launch_project_stage(ctx->kp, ctx->ws.Un, u, u, dudt, 0.0, 1.0, 1, ctx->stream); });
}

static fr_sg_status step_generic(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags,
                                 bool chained = false) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const int E = ctx->E;
  const bool cfl = !(dt > 0.0);
  uint8_t* f0 = flags ? flags : nullptr;
  uint8_t* f1 = flags ? flags + E : nullptr;
  uint8_t* f2 = flags ? flags + 2 * E : nullptr;
  uint8_t* f3 = flags ? flags + 3 * E : nullptr;
  fr_sg_status st;

  FRSG_TRY_HIP(launch_set_scalars(K, cfl ? 0.0 : dt, s), ctx);
  const double sb = state_bytes(ctx);
  if (ctx->fused_tri) {
    // triangles: one fused launch per stage, which also runs the limiter on its output
    // (stages 1 and 2) or the sensor-gated filter and then the limiter (stage 3).  Each
    // stage writes the modal traces of its final output into the trace buffer its
    // input's traces are not in, so only the first step of a call runs a trace pass over
    // u (chained: u is the previous step's result)
    if (cfl) {
      if ((st = timed(ctx, "cfl", sb, [&] { return launch_cfl_tri_modal(K, u, s); }))) return st;
      FRSG_TRY_HIP(launch_dt(K, ctx->dim, nullptr, s), ctx);
    }
    const int c0 = chained ? ctx->tm_cur : 0, c1 = c0 ^ 1;
    double* T0 = W.Tm[c0];
    double* T1 = W.Tm[c1];
    const bool lim = ctx->prob.limiter != 0, filt = ctx->prob.filter != FRSG_FILTER_NONE;
    for (uint8_t* f : {f0, f1, f3})
      if (!lim && f) FRSG_TRY_HIP(launch_fill_flags(f, E, s), ctx);
    if (!filt && f2) FRSG_TRY_HIP(launch_fill_flags(f2, E, s), ctx);
    TriPost p1, p2, p3;
    p1.limit = p2.limit = p3.limit = lim ? 1 : 0;
    p1.flag_lim = lim ? f0 : nullptr;
    p2.flag_lim = lim ? f1 : nullptr;
    p3.flag_lim = lim ? f3 : nullptr;
    p3.filter = filt ? 1 : 0;
    p3.flag_filt = filt ? f2 : nullptr;
    if ((st = timed(ctx, "stage1", 2 * sb, [&] {
           return launch_stage_tri(K, u, u, u, W.w1, 0.0, 1.0, 0, T0, chained ? 1 : 0, T1, s, p1);
         })))
      return st;
    if ((st = timed(ctx, "stage2", 3 * sb,
                    [&] { return launch_stage_tri(K, W.w1, u, W.w1, W.w2, 0.75, 0.25, 0, T1, 1, T0, s, p2); })))
      return st;
    if ((st = timed(ctx, "stage3", 3 * sb, [&] {
           return launch_stage_tri(K, W.w2, u, W.w2, u, 1.0 / 3.0, 2.0 / 3.0, 0, T0, 1, T1, s, p3);
         })))
      return st;
    ctx->tm_cur = c1;
    if (dt_used) FRSG_TRY_HIP(launch_copy_dt(K, dt_used, s), ctx);
    return FRSG_OK;
  }
  // stage 1: w1 = Lim(u + dt R(u)); the CFL maximum is taken in the same pass over u
  if ((st = rhs_passes(ctx, u, cfl ? 1 : 0)) != FRSG_OK) return st;
  if (cfl) FRSG_TRY_HIP(launch_dt(K, ctx->dim, nullptr, s), ctx);
  if ((st = timed(ctx, "project_stage1", 2 * sb,
                  [&] { return launch_project_stage(K, W.Un, u, u, W.w1, 0.0, 1.0, 0, s); })))
    return st;
  if ((st = fr_sg_limit(ctx, W.w1, f0)) != FRSG_OK) return st;
  // stage 2: w2 = Lim(3/4 u + 1/4 (w1 + dt R(w1)))
  if ((st = rhs_passes(ctx, W.w1, 0)) != FRSG_OK) return st;
  if ((st = timed(ctx, "project_stage2", 3 * sb,
                  [&] { return launch_project_stage(K, W.Un, u, W.w1, W.w2, 0.75, 0.25, 0, s); })))
    return st;
  if ((st = fr_sg_limit(ctx, W.w2, f1)) != FRSG_OK) return st;
  // stage 3: v = 1/3 u + 2/3 (w2 + dt R(w2)), written over u
  if ((st = rhs_passes(ctx, W.w2, 0)) != FRSG_OK) return st;
  if ((st = timed(ctx, "project_stage3", 3 * sb,
                  [&] { return launch_project_stage(K, W.Un, u, W.w2, u, 1.0 / 3.0, 2.0 / 3.0, 0, s); })))
    return st;
  // end of step: sensor-gated filter, then limiter
  if (ctx->prob.filter != FRSG_FILTER_NONE) {
    if ((st = timed(ctx, "sensor_filter", 2 * sb, [&] { return launch_sensor_filter(K, u, f2, s); }))) return st;
  } else if (f2)
    FRSG_TRY_HIP(launch_fill_flags(f2, E, s), ctx);
  if ((st = fr_sg_limit(ctx, u, f3)) != FRSG_OK) return st;
  if (dt_used) FRSG_TRY_HIP(launch_copy_dt(K, dt_used, s), ctx);
  return FRSG_OK;
}

// The three stage states of the fused 1D path: w1 = u + dt R(u), w2 = 3/4 u + 1/4 (w1
// + dt R(w1)), out = 1/3 u + 2/3 (w2 + dt R(w2)).  With lim set every stage output is
// limited (Euler) or its limiter flags cleared, and the third stage also runs the
// detector-switched filter and the CFL maximum of its output (into lam_next); the
// third stage only runs when out is not null.
static fr_sg_status stages_fused1d(fr_sg_ctx* ctx, const double* u, double* out, uint8_t* f0, uint8_t* f1,
                                   uint8_t* f2, uint8_t* f3, bool lim, unsigned long long* lam_next,
                                   int dt_source = 0, double dt_fixed = 0.0,
                                   const unsigned long long* lam_in = nullptr, double* dt_used = nullptr,
                                   double* w1 = nullptr, double* w2 = nullptr) {
  const KParams& K = ctx->kp;
  Workspace W = ctx->ws;  // the stage states go to the workspace, or to the caller's w1, w2
  if (w1) W.w1 = w1;
  if (w2) W.w2 = w2;
  hipStream_t s = ctx->stream;
  const double sb = state_bytes(ctx);
  const int limiter = (lim && ctx->prob.limiter) ? 1 : 0;
  const bool clear = lim && !limiter;
  fr_sg_status st;
  if ((st = timed(ctx, "stage1", 2 * sb, [&] {
         return launch_stage1d(K, u, u, u, W.w1, 0.0, 1.0, 0, clear ? f0 : nullptr, s, limiter, 0, f0, nullptr,
                               nullptr, dt_source, dt_fixed, lam_in, lam_next, dt_used);
       })))
    return st;
  if ((st = timed(ctx, "stage2", 3 * sb, [&] {
         return launch_stage1d(K, W.w1, u, W.w1, W.w2, 0.75, 0.25, 0, clear ? f1 : nullptr, s, limiter, 0, f1);
       })))
    return st;
  if (!out) return FRSG_OK;
  return timed(ctx, "stage3", 3 * sb, [&] {
    return launch_stage1d(K, W.w2, u, W.w2, out, 1.0 / 3.0, 2.0 / 3.0, 0, clear ? f3 : nullptr, s, limiter,
                          lim ? 1 : 0, f3, f2, lam_next);
  });
}

// fused 1D step: CFL pass (dt <= 0 and no maximum from the previous step), three
// stage kernels with the limiter, filter and next CFL maximum in their epilogues;
// the first stage derives and publishes dt
static fr_sg_status step_fused1d(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags,
                                 bool reuse_cfl, double* w1 = nullptr, double* w2 = nullptr) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const int E = ctx->E;
  unsigned long long* lam[2] = {(unsigned long long*)(W.scal + 1), (unsigned long long*)(W.scal + 3)};
  const int cur = ctx->lam_cur;
  fr_sg_status st;
  const bool fixed = dt > 0.0;
  if (!fixed && !reuse_cfl)
    if ((st = timed(ctx, "cfl", state_bytes(ctx), [&] { return launch_cfl1d(K, u, lam[cur], s); }))) return st;
  uint8_t* f0 = flags ? flags : nullptr;
  uint8_t* f1 = flags ? flags + E : nullptr;
  uint8_t* f2 = flags ? flags + 2 * E : nullptr;
  uint8_t* f3 = flags ? flags + 3 * E : nullptr;
  if ((st = stages_fused1d(ctx, u, u, f0, f1, f2, f3, true, lam[cur ^ 1], fixed ? 1 : 2, fixed ? dt : 0.0,
                           lam[cur], dt_used, w1, w2)) != FRSG_OK)
    return st;
  ctx->lam_cur = cur ^ 1;
  return FRSG_OK;
}

// the steps of an fr_sg_steps call on a small 1D problem: the CFL pass of u, then
// every step in one launch of one workgroup (the fused 1D stage code, three
// stages per step separated by workgroup barriers); the CFL maximum of the result
// is left where the next call's first step finds it
static fr_sg_status steps_resident1d(fr_sg_ctx* ctx, double* u, int nsteps, double* dt_used, uint8_t* flags) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  unsigned long long* lam[2] = {(unsigned long long*)(W.scal + 1), (unsigned long long*)(W.scal + 3)};
  const int cur = ctx->lam_cur;
  const double sb = state_bytes(ctx);
  fr_sg_status st;
  if ((st = timed(ctx, "cfl", sb, [&] { return launch_cfl1d(K, u, lam[cur], s); }))) return st;
  const char* name = fr1d_resident_lds_state(K) ? "steps_resident_lds" : "steps_resident";
  // at most kChunk steps per launch (a few tens of milliseconds), the CFL maximum
  // handed from launch to launch through the two accumulators
  constexpr int kChunk = 4096;
  int c = cur;
  for (int done = 0; done < nsteps; done += kChunk) {
    const int n = std::min(kChunk, nsteps - done);
    if ((st = timed(ctx, name, 8 * sb * n, [&] {
           return launch_steps1d_resident(K, u, W.w1, W.w2, n, ctx->prob.limiter ? 1 : 0,
                                          flags ? flags + 4l * ctx->E * done : nullptr,
                                          dt_used ? dt_used + done : nullptr, lam[c], lam[c ^ 1], s);
         })))
      return st;
    c ^= 1;
  }
  ctx->lam_cur = c;
  return FRSG_OK;
}

// fused 2D Euler step: one kernel per stage.  chained: u is the state the
// previous step of the same call produced, so the CFL maximum of u comes from
// the accumulator its end-of-step pass filled and the face traces of u from the
// buffer its last launch wrote.
static fr_sg_status step_fused(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags,
                               bool chained) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const int E = ctx->E;
  const double sb = state_bytes(ctx);
  unsigned long long* lam[2] = {(unsigned long long*)(W.scal + 1), (unsigned long long*)(W.scal + 3)};
  const int cur = ctx->lam_cur;
  fr_sg_status st;
  if (dt > 0.0) {
    FRSG_TRY_HIP(launch_set_dt(K, dt, nullptr, lam[cur ^ 1], s), ctx);
  } else {
    if (!chained)
      if ((st = timed(ctx, "cfl", sb, [&] { return launch_fused_cfl(K, u, lam[cur], s); }))) return st;
    FRSG_TRY_HIP(launch_dt_from(K, lam[cur], lam[cur ^ 1], nullptr, s), ctx);
  }
  uint8_t* f0 = flags ? flags : nullptr;
  uint8_t* f1 = flags ? flags + E : nullptr;
  uint8_t* f2 = flags ? flags + 2 * E : nullptr;
  uint8_t* f3 = flags ? flags + 3 * E : nullptr;
  const int f32 = fp32(ctx);
  // each launch writes the face traces of its output into the buffer the
  // previous launch did not write; stage 1 reads those of u only when the
  // previous step of this call wrote them
  const int tc = ctx->tr_cur;
  FusedStage s1{u, u, W.w1, 0.0, 1.0, 1, f0, nullptr, nullptr, ctx->dDt, ctx->dcmax, ctx->dPhiT, ctx->dPWT,
                f32, ctx->dPhiT32, ctx->dPWT32, chained ? W.tr[tc] : nullptr, W.tr[tc ^ 1]};
  if ((st = timed(ctx, "stage1", 2 * sb, [&] { return launch_fused_stage(K, s1, s); }))) return st;
  FusedStage s2{W.w1, u, W.w2, 0.75, 0.25, 2, f1, nullptr, nullptr, ctx->dDt, ctx->dcmax, ctx->dPhiT, ctx->dPWT,
                f32, ctx->dPhiT32, ctx->dPWT32, W.tr[tc ^ 1], W.tr[tc]};
  if ((st = timed(ctx, "stage2", 3 * sb, [&] { return launch_fused_stage(K, s2, s); }))) return st;
  FusedStage s3{W.w2, u, u, 1.0 / 3.0, 2.0 / 3.0, 3, f3, f2, lam[cur ^ 1], ctx->dDt, ctx->dcmax, ctx->dPhiT,
                ctx->dPWT, f32, ctx->dPhiT32, ctx->dPWT32, W.tr[tc], W.tr[tc ^ 1]};
  if ((st = timed(ctx, "stage3", 3 * sb, [&] { return launch_fused_stage(K, s3, s); }))) return st;
  ctx->tr_cur = tc ^ 1;
  ctx->lam_cur = cur ^ 1;
  ctx->lam_for = u;
  if (dt_used) FRSG_TRY_HIP(launch_copy_dt(K, dt_used, s), ctx);
  return FRSG_OK;
}

// matrix-core 2D Euler step (FP64 or BF16-split): one kernel per stage.  Every
// stage reads the modal face traces of its input from the trace buffer the
// previous launch wrote; the first stage of a call gets them from a trace pass
// over u unless the previous step of the same call wrote them (chained).
static fr_sg_status step_quad(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags, bool chained) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const int E = ctx->E;
  const double sb = state_bytes(ctx);
  unsigned long long* lam[2] = {(unsigned long long*)(W.scal + 1), (unsigned long long*)(W.scal + 3)};
  const int cur = ctx->lam_cur;
  fr_sg_status st;
  if (dt > 0.0) {
    FRSG_TRY_HIP(launch_set_dt(K, dt, nullptr, lam[cur ^ 1], s), ctx);
  } else {
    if (!chained)
      if ((st = timed(ctx, "cfl", sb, [&] { return launch_fused_cfl(K, u, lam[cur], s); }))) return st;
    FRSG_TRY_HIP(launch_dt_from(K, lam[cur], lam[cur ^ 1], nullptr, s), ctx);
  }
  const int tc = ctx->tr_cur;
  if (!chained)
    if ((st = timed(ctx, "traces", 0.0, [&] { return launch_quad_traces(K, u, W.tr[tc], s); }))) return st;
  uint8_t* f0 = flags ? flags : nullptr;
  uint8_t* f1 = flags ? flags + E : nullptr;
  uint8_t* f2 = flags ? flags + 2 * E : nullptr;
  uint8_t* f3 = flags ? flags + 3 * E : nullptr;
  const int bf = ctx->prob.precision == FRSG_BF16_SPLIT ? 1 : 0;
  QuadStage s1{u, u, W.w1, 0.0, 1.0, 1, f0, nullptr, nullptr, ctx->dDt, ctx->dcmax, ctx->dfrag, bf, W.tr[tc],
               W.tr[tc ^ 1]};
  if ((st = timed(ctx, "stage1", 2 * sb, [&] { return launch_quad_stage(K, s1, s); }))) return st;
  QuadStage s2{W.w1, u, W.w2, 0.75, 0.25, 2, f1, nullptr, nullptr, ctx->dDt, ctx->dcmax, ctx->dfrag, bf,
               W.tr[tc ^ 1], W.tr[tc]};
  if ((st = timed(ctx, "stage2", 3 * sb, [&] { return launch_quad_stage(K, s2, s); }))) return st;
  QuadStage s3{W.w2, u, u, 1.0 / 3.0, 2.0 / 3.0, 3, f3, f2, lam[cur ^ 1], ctx->dDt, ctx->dcmax, ctx->dfrag, bf,
               W.tr[tc], W.tr[tc ^ 1]};
  if ((st = timed(ctx, "stage3", 3 * sb, [&] { return launch_quad_stage(K, s3, s); }))) return st;
  ctx->tr_cur = tc ^ 1;
  ctx->lam_cur = cur ^ 1;
  ctx->lam_for = u;
  if (dt_used) FRSG_TRY_HIP(launch_copy_dt(K, dt_used, s), ctx);
  return FRSG_OK;
}

// One step of a tableau integrator (RK4, Bogacki-Shampine 3(2), Tsitouras 5(4)):
//   K_1 = R(u), Y_i = Lim(u + dt sum_{j<i} a_ij K_j), K_i = R(Y_i),
//   u <- Lim(Filter(u + dt sum_i b_i K_i)),
// with the path's right-hand-side kernels, the stage combination kernel and the
// element-wise limiter and sensor/filter passes.  Flags: row 0 = limiter acted
// on any stage state, row 1 = 0, rows 2 and 3 as for SSP-RK3.
// Butcher-tableau step on the fused 1D path, one stage kernel per stage: kernel i takes
// the right-hand side of Y_i (Y_0 = u), keeps it as K_i and forms in its epilogue
// Y_{i+1} = u + dt sum_{j <= i} a_{i+1,j} K_j, limited (flags OR-ed into row 0); the
// last kernel forms u + dt sum_j b_j K_j in place and runs the detector-switched filter,
// the limiter and the CFL maximum of the result.  Kernel 0 derives and publishes dt.
// The same operations in the same order as the combination, limiter and filter passes.
static fr_sg_status step_rk_fused1d(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags,
                                    bool reuse_cfl) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const Tableau& tb = *tableau_of(ctx->prob.integrator);
  const int E = ctx->E;
  const double sb = state_bytes(ctx);
  unsigned long long* lam[2] = {(unsigned long long*)(W.scal + 1), (unsigned long long*)(W.scal + 3)};
  const int cur = ctx->lam_cur;
  fr_sg_status st;
  const bool fixed = dt > 0.0;
  if (!fixed && !reuse_cfl)
    if ((st = timed(ctx, "cfl", sb, [&] { return launch_cfl1d(K, u, lam[cur], s); }))) return st;
  if (flags) FRSG_TRY_HIP(launch_fill_flags(flags, 4l * E, s), ctx);
  uint8_t* f0 = flags ? flags : nullptr;
  uint8_t* f2 = flags ? flags + 2 * E : nullptr;
  uint8_t* f3 = flags ? flags + 3 * E : nullptr;
  const int limiter = ctx->prob.limiter ? 1 : 0;
  double* Y[2] = {W.w1, W.w2};
  const double* in = u;
  for (int i = 0; i < tb.s; ++i) {
    const bool last = i == tb.s - 1;
    const double* row = last ? tb.b : tb.A[i + 1];
    RkTerms T;
    T.n = 0;
    for (int j = 0; j < i; ++j)
      if (row[j] != 0.0) {
        T.K[T.n] = W.rk[j];
        T.a[T.n] = row[j];
        ++T.n;
      }
    double* out = last ? u : Y[i & 1];
    if ((st = timed(ctx, last ? "rk_stage_last" : "rk_stage", (T.n + 3) * sb, [&] {
           return launch_stage1d_tab(K, in, u, out, last ? nullptr : W.rk[i], T, row[i], s, limiter, last ? 1 : 0,
                                     last ? f3 : f0, last ? f2 : nullptr, last ? lam[cur ^ 1] : nullptr,
                                     i == 0 ? (fixed ? 1 : 2) : 0, fixed ? dt : 0.0, i == 0 ? lam[cur] : nullptr,
                                     i == 0 ? lam[cur ^ 1] : nullptr, i == 0 ? dt_used : nullptr);
         })))
      return st;
    in = out;
  }
  ctx->lam_cur = cur ^ 1;
  return FRSG_OK;
}

// Butcher-tableau step on the fused 2D path, one stage kernel per stage, as on the 1D
// path: kernel i keeps R(Y_i) as K_i and forms Y_{i+1} = u + dt sum_{j <= i} a_{i+1,j} K_j,
// limited (flags OR-ed into row 0), in its epilogue; the last kernel forms the update in
// place and runs the filter, the limiter and the CFL maximum.  Each launch writes the
// face traces of its output for the next; the first reads those of u when the previous
// step of the same call wrote them (chained).
static fr_sg_status step_rk_fused2d(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags,
                                    bool chained) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const Tableau& tb = *tableau_of(ctx->prob.integrator);
  const int E = ctx->E;
  const double sb = state_bytes(ctx);
  unsigned long long* lam[2] = {(unsigned long long*)(W.scal + 1), (unsigned long long*)(W.scal + 3)};
  const int cur = ctx->lam_cur;
  fr_sg_status st;
  if (dt > 0.0) {
    FRSG_TRY_HIP(launch_set_dt(K, dt, nullptr, lam[cur ^ 1], s), ctx);
  } else {
    if (!chained)
      if ((st = timed(ctx, "cfl", sb, [&] { return launch_fused_cfl(K, u, lam[cur], s); }))) return st;
    FRSG_TRY_HIP(launch_dt_from(K, lam[cur], lam[cur ^ 1], nullptr, s), ctx);
  }
  if (flags) FRSG_TRY_HIP(launch_fill_flags(flags, 4l * E, s), ctx);
  uint8_t* f0 = flags ? flags : nullptr;
  uint8_t* f2 = flags ? flags + 2 * E : nullptr;
  uint8_t* f3 = flags ? flags + 3 * E : nullptr;
  const int f32 = fp32(ctx);
  double* Y[2] = {W.w1, W.w2};
  const double* in = u;
  int tc = ctx->tr_cur;
  const double* tr_in = chained ? W.tr[tc] : nullptr;
  for (int i = 0; i < tb.s; ++i) {
    const bool last = i == tb.s - 1;
    const double* row = last ? tb.b : tb.A[i + 1];
    FusedStage S{in,        u,         last ? u : Y[i & 1], 0.0, 1.0, last ? 3 : 1, last ? f3 : f0, last ? f2 : nullptr,
                 last ? lam[cur ^ 1] : nullptr, ctx->dDt, ctx->dcmax, ctx->dPhiT, ctx->dPWT, f32, ctx->dPhiT32,
                 ctx->dPWT32, tr_in, W.tr[tc ^ 1]};
    S.tab = 1;
    S.terms.n = 0;
    for (int j = 0; j < i; ++j)
      if (row[j] != 0.0) {
        S.terms.K[S.terms.n] = W.rk[j];
        S.terms.a[S.terms.n] = row[j];
        ++S.terms.n;
      }
    S.ka_cur = row[i];
    S.k_out = last ? nullptr : W.rk[i];
    if ((st = timed(ctx, last ? "rk_stage_last" : "rk_stage", (S.terms.n + 3) * sb,
                    [&] { return launch_fused_stage(K, S, s); })))
      return st;
    in = S.out;
    tr_in = W.tr[tc ^ 1];
    tc ^= 1;
  }
  ctx->tr_cur = tc;
  ctx->lam_cur = cur ^ 1;
  ctx->lam_for = u;
  if (dt_used) FRSG_TRY_HIP(launch_copy_dt(K, dt_used, s), ctx);
  return FRSG_OK;
}

static fr_sg_status step_rk(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const Tableau& tb = *tableau_of(ctx->prob.integrator);
  const int E = ctx->E;
  const long n = (long)ctx->S * ctx->kp.M * E * ctx->nsp;
  const double sb = state_bytes(ctx);
  unsigned long long* lam = (unsigned long long*)(W.scal + 1);
  fr_sg_status st;
  // dt on the device: fixed, or from the CFL maximum of u
  if (dt > 0.0) {
    if (ctx->fused || ctx->quad || ctx->fused1d)
      FRSG_TRY_HIP(launch_set_dt(K, dt, nullptr, nullptr, s), ctx);
    else
      FRSG_TRY_HIP(launch_set_scalars(K, dt, s), ctx);
  } else if (ctx->fused || ctx->quad) {
    if ((st = timed(ctx, "cfl", sb, [&] { return launch_fused_cfl(K, u, lam, s); }))) return st;
    FRSG_TRY_HIP(launch_dt_from(K, lam, nullptr, nullptr, s), ctx);
  } else if (ctx->fused1d) {
    if ((st = timed(ctx, "cfl", sb, [&] { return launch_cfl1d(K, u, lam, s); }))) return st;
    FRSG_TRY_HIP(launch_dt_from(K, lam, nullptr, nullptr, s), ctx);
  } else if (ctx->fused_tri) {
    FRSG_TRY_HIP(launch_set_scalars(K, 0.0, s), ctx);
    if ((st = timed(ctx, "cfl", sb, [&] { return launch_cfl_tri_modal(K, u, s); }))) return st;
    FRSG_TRY_HIP(launch_dt(K, ctx->dim, nullptr, s), ctx);
  } else {
    FRSG_TRY_HIP(launch_set_scalars(K, 0.0, s), ctx);
    if ((st = timed(ctx, "nodal", sb, [&] { return launch_nodal(K, u, W.Un, W.Fn, W.Gn, ctx->is_tri ? 0 : 1, s); })))
      return st;
    if (ctx->is_tri && (st = timed(ctx, "cfl", 0.0, [&] { return launch_cfl_tri(K, W.Un, s); }))) return st;
    FRSG_TRY_HIP(launch_dt(K, ctx->dim, nullptr, s), ctx);
  }
  uint8_t* f0 = flags ? flags : nullptr;
  uint8_t* scratch = (uint8_t*)W.w2;  // per-stage limiter flags, OR-ed into row 0
  if (f0) FRSG_TRY_HIP(launch_fill_flags(f0, E, s), ctx);
  if (flags) FRSG_TRY_HIP(launch_fill_flags(flags + E, E, s), ctx);
  double* Y = W.w1;
  for (int i = 0; i < tb.s; ++i) {
    const double* in = u;
    if (i > 0) {
      RkTerms T;
      T.n = 0;
      for (int j = 0; j < i; ++j)
        if (tb.A[i][j] != 0.0) {
          T.K[T.n] = W.rk[j];
          T.a[T.n] = tb.A[i][j];
          ++T.n;
        }
      if ((st = timed(ctx, "rk_stage", (T.n + 2) * sb,
                      [&] { return launch_rk_combine(u, T, K.dt, Y, n, s); })))
        return st;
      if (ctx->prob.limiter) {
        if ((st = fr_sg_limit(ctx, Y, f0 ? scratch : nullptr)) != FRSG_OK) return st;
        if (f0) FRSG_TRY_HIP(launch_or_flags(f0, scratch, E, s), ctx);
      }
      in = Y;
    }
    if ((st = rhs_into(ctx, in, W.rk[i])) != FRSG_OK) return st;
  }
  RkTerms T;
  T.n = 0;
  for (int i = 0; i < tb.s; ++i)
    if (tb.b[i] != 0.0) {
      T.K[T.n] = W.rk[i];
      T.a[T.n] = tb.b[i];
      ++T.n;
    }
  if ((st = timed(ctx, "rk_update", (T.n + 2) * sb, [&] { return launch_rk_combine(u, T, K.dt, u, n, s); })))
    return st;
  uint8_t* f2 = flags ? flags + 2 * E : nullptr;
  uint8_t* f3 = flags ? flags + 3 * E : nullptr;
  const bool filt = ctx->prob.filter != FRSG_FILTER_NONE;
  if (ctx->fused_tri) {
    // filter and limiter in one element-wise pass
    if (!filt && f2) FRSG_TRY_HIP(launch_fill_flags(f2, E, s), ctx);
    if (!ctx->prob.limiter && f3) FRSG_TRY_HIP(launch_fill_flags(f3, E, s), ctx);
    TriPost p;
    p.filter = filt ? 1 : 0;
    p.limit = ctx->prob.limiter ? 1 : 0;
    p.flag_filt = filt ? f2 : nullptr;
    p.flag_lim = ctx->prob.limiter ? f3 : nullptr;
    if (p.filter || p.limit)
      if ((st = timed(ctx, "filter_limiter", 2 * sb, [&] { return launch_post_tri(K, u, p, s); }))) return st;
  } else if (ctx->fused) {
    // filter and limiter in one element-wise pass
    if (!filt && f2) FRSG_TRY_HIP(launch_fill_flags(f2, E, s), ctx);
    if (!ctx->prob.limiter && f3) FRSG_TRY_HIP(launch_fill_flags(f3, E, s), ctx);
    if (filt || ctx->prob.limiter)
      if ((st = timed(ctx, "filter_limiter", 2 * sb, [&] {
             return launch_fused_post(K, ctx->dPhiT, ctx->dcmax, u, filt ? 1 : 0, ctx->prob.limiter ? 1 : 0,
                                      filt ? f2 : nullptr, ctx->prob.limiter ? f3 : nullptr, s);
           })))
        return st;
  } else {
    if (filt) {
      if ((st = timed(ctx, "sensor_filter", 2 * sb, [&] { return launch_sensor_filter(K, u, f2, s); }))) return st;
    } else if (f2) {
      FRSG_TRY_HIP(launch_fill_flags(f2, E, s), ctx);
    }
    if ((st = fr_sg_limit(ctx, u, f3)) != FRSG_OK) return st;
  }
  ctx->lam_for = nullptr;
  if (dt_used) FRSG_TRY_HIP(launch_copy_dt(K, dt_used, s), ctx);
  return FRSG_OK;
}

static fr_sg_status check_step_args(fr_sg_ctx* ctx, double* u, double dt) {
  if (!ctx) return FRSG_EINVAL;
  if (!u) {
    ctx->err = "null state";
    return FRSG_EINVAL;
  }
  if (!std::isfinite(dt)) {
    ctx->err = "dt must be finite";
    return FRSG_EINVAL;
  }
  return FRSG_OK;
}

fr_sg_status fr_sg_step(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags) {
  fr_sg_status st = check_step_args(ctx, u, dt);
  if (st != FRSG_OK) return st;
  if (ctx->prob.integrator != FRSG_SSPRK3)
    return ctx->fused1d ? step_rk_fused1d(ctx, u, dt, dt_used, flags, false)
           : ctx->fused ? step_rk_fused2d(ctx, u, dt, dt_used, flags, false)
                        : step_rk(ctx, u, dt, dt_used, flags);
  if (ctx->quad) return step_quad(ctx, u, dt, dt_used, flags, false);
  if (ctx->fused) return step_fused(ctx, u, dt, dt_used, flags, false);
  if (ctx->fused1d) return step_fused1d(ctx, u, dt, dt_used, flags, false);
  return step_generic(ctx, u, dt, dt_used, flags);
}

fr_sg_status fr_sg_steps(fr_sg_ctx* ctx, double* u, int32_t nsteps, double* dt_used, uint8_t* flags) {
  fr_sg_status st = check_step_args(ctx, u, 0.0);
  if (st != FRSG_OK) return st;
  if (nsteps < 0) {
    ctx->err = "nsteps must be >= 0";
    return FRSG_EINVAL;
  }
  if (ctx->resident1d && nsteps > 0) return steps_resident1d(ctx, u, nsteps, dt_used, flags);
  const long fl = 4l * ctx->E;
  for (int i = 0; i < nsteps; ++i) {
    double* dtu = dt_used ? dt_used + i : nullptr;
    uint8_t* f = flags ? flags + i * fl : nullptr;
    if (ctx->prob.integrator != FRSG_SSPRK3)
      st = ctx->fused1d ? step_rk_fused1d(ctx, u, 0.0, dtu, f, i > 0)
           : ctx->fused ? step_rk_fused2d(ctx, u, 0.0, dtu, f, i > 0)
                        : step_rk(ctx, u, 0.0, dtu, f);
    else if (ctx->quad)
      st = step_quad(ctx, u, 0.0, dtu, f, i > 0);
    else if (ctx->fused)
      st = step_fused(ctx, u, 0.0, dtu, f, i > 0);
    else if (ctx->fused1d)
      st = step_fused1d(ctx, u, 0.0, dtu, f, i > 0);
    else
      st = step_generic(ctx, u, 0.0, dtu, f, i > 0);
    if (st != FRSG_OK) return st;
  }
  return FRSG_OK;
}

// the conditions both adjoint entry points share
static fr_sg_status check_adjoint_args(fr_sg_ctx* ctx, const double* u_n, const uint8_t* flags_n, double dt,
                                       double* lam) {
  if (!ctx->ws.avb) {
    ctx->err = "the adjoint covers the scalar 1D equations (advection, Burgers) only";
    return FRSG_EUNSUPPORTED;
  }
  if (!u_n || !lam || u_n == lam) {
    ctx->err = "u_n and lam must be distinct device pointers";
    return FRSG_EINVAL;
  }
  if (!(dt > 0.0) || !std::isfinite(dt)) {
    ctx->err = "dt must be positive and finite";
    return FRSG_EINVAL;
  }
  if (ctx->prob.integrator != FRSG_SSPRK3) {
    ctx->err = "the adjoint covers the SSP-RK3 step";
    return FRSG_EUNSUPPORTED;
  }
  if (ctx->prob.filter == FRSG_FILTER_LASSO) {
    ctx->err = "the adjoint covers the linear filters (exponential, L2), not the Lasso filter";
    return FRSG_EUNSUPPORTED;
  }
  if (ctx->prob.filter != FRSG_FILTER_NONE && !flags_n) {
    ctx->err = "flags_n is needed: the filter decisions of the forward step";
    return FRSG_EINVAL;
  }
  if (ctx->prob.precision == FRSG_BF16_SPLIT) {
    ctx->err = "the adjoint runs in FP64 and FP32-mixed precision";
    return FRSG_EUNSUPPORTED;
  }
  if (ctx->kp.fp32 && !adj1d_fused_supported(ctx->kp)) {
    ctx->err = "the FP32-mixed adjoint runs on the fused adjoint kernel (FR degree <= 7, Nq <= 85, one block's "
               "LDS within 48 KiB)";
    return FRSG_EUNSUPPORTED;
  }
  return FRSG_OK;
}

static fr_sg_status adjoint_from_stages(fr_sg_ctx* ctx, const double* u_n, const double* w1, const double* w2,
                                        const uint8_t* flags_n, double dt, double* lam, double* dparams);

fr_sg_status fr_sg_adjoint_step(fr_sg_ctx* ctx, const double* u_n, const uint8_t* flags_n, double dt, double* lam,
                                double* dparams) {
  if (!ctx) return FRSG_EINVAL;
  fr_sg_status st = check_adjoint_args(ctx, u_n, flags_n, dt, lam);
  if (st != FRSG_OK) return st;
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const double sb = state_bytes(ctx);
  // stage states of the forward step, recomputed with the same kernels as the
  // forward step (no limiter: the scalar equations do not use it); the first
  // stage kernel publishes dt for the passes after it
  if (ctx->fused1d) {
    if ((st = stages_fused1d(ctx, u_n, nullptr, nullptr, nullptr, nullptr, nullptr, false, nullptr, 1, dt)) !=
        FRSG_OK)
      return st;
  } else {
    FRSG_TRY_HIP(launch_set_scalars(K, dt, s), ctx);
    if ((st = rhs_passes(ctx, u_n, 0)) != FRSG_OK) return st;
    if ((st = timed(ctx, "adj_fwd_stage1", 2 * sb,
                    [&] { return launch_project_stage(K, W.Un, u_n, u_n, W.w1, 0.0, 1.0, 0, s); })))
      return st;
    if ((st = rhs_passes(ctx, W.w1, 0)) != FRSG_OK) return st;
    if ((st = timed(ctx, "adj_fwd_stage2", 3 * sb,
                    [&] { return launch_project_stage(K, W.Un, u_n, W.w1, W.w2, 0.75, 0.25, 0, s); })))
      return st;
  }
  return adjoint_from_stages(ctx, u_n, W.w1, W.w2, flags_n, dt, lam, dparams);
}

// the transposed step given the forward step's stage states w1, w2 (dt on the device)
static fr_sg_status adjoint_from_stages(fr_sg_ctx* ctx, const double* u_n, const double* w1, const double* w2,
                                        const uint8_t* flags_n, double dt, double* lam, double* dparams) {
  const KParams& K = ctx->kp;
  Workspace& W = ctx->ws;
  hipStream_t s = ctx->stream;
  const double sb = state_bytes(ctx);
  fr_sg_status st;
  // u+ = Filter(v): vb = Filter^T lam
  if (ctx->prob.filter != FRSG_FILTER_NONE) {
    if ((st = timed(ctx, "adj_filter", 2 * sb,
                    [&] { return launch_filter_adjoint(K, lam, flags_n + 2 * (long)ctx->E, W.avb, s); })))
      return st;
  } else {
    FRSG_TRY_HIP(hipMemcpyAsync(W.avb, lam, (size_t)sb, hipMemcpyDeviceToDevice, s), ctx);
  }
  // one transposed right-hand side: nodal values of the state, then the adjoint passes
  const bool fused_adj = adj1d_fused_supported(K);
  auto vjp = [&](const char* name, const double* w, const double* g, const double* x0, const double* x1,
                 const double* x2, double* out, double c0, double c1, double c2, double cg, double pscale) {
    if (fused_adj)
      return timed(ctx, name, 3 * sb, [&] {
        return launch_adj_stage1d(K, w, g, x0, x1, x2, out, c0, c1, c2, cg, W.apart, pscale, dparams, s);
      });
    fr_sg_status r = timed(ctx, "adj_nodal", sb, [&] { return launch_nodal(K, w, W.Un, W.Fn, W.Gn, 0, s); });
    if (r != FRSG_OK) return r;
    return timed(ctx, name, 3 * sb, [&] {
      return launch_rhs_adjoint(K, W.Un, g, W.Fn, W.Corr, W.agT, x0, x1, x2, out, c0, c1, c2, cg, W.apart, pscale,
                                dparams, s);
    });
  };
  // v = u/3 + 2/3 (w2 + dt R(w2)):   b2 = 2/3 vb + 2/3 dt R'(w2)^T vb
  if ((st = vjp("adj_stage3", w2, W.avb, W.avb, nullptr, nullptr, W.ab2, 2.0 / 3.0, 0.0, 0.0, 2.0 / 3.0 * dt,
                2.0 / 3.0 * dt)))
    return st;
  // w2 = 3/4 u + 1/4 (w1 + dt R(w1)):  b1 = 1/4 b2 + 1/4 dt R'(w1)^T b2
  if ((st = vjp("adj_stage2", w1, W.ab2, W.ab2, nullptr, nullptr, W.ab1, 0.25, 0.0, 0.0, 0.25 * dt, 0.25 * dt)))
    return st;
  // w1 = u + dt R(u):  lam_n = vb/3 + 3/4 b2 + b1 + dt R'(u)^T b1
  return vjp("adj_stage1", u_n, W.ab1, W.avb, W.ab2, W.ab1, lam, 1.0 / 3.0, 0.75, 1.0, dt, dt);
}

fr_sg_status fr_sg_step_stages(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags, double* w1,
                               double* w2) {
  fr_sg_status st = check_step_args(ctx, u, dt);
  if (st != FRSG_OK) return st;
  if (!ctx->fused1d || !ctx->ws.avb || ctx->prob.integrator != FRSG_SSPRK3) {
    ctx->err = "stage states are handed out by the fused 1D SSP-RK3 step of the scalar equations";
    return FRSG_EUNSUPPORTED;
  }
  if (!w1 || !w2 || w1 == w2 || w1 == u || w2 == u) {
    ctx->err = "w1 and w2 must be distinct device state buffers, distinct from u";
    return FRSG_EINVAL;
  }
  return step_fused1d(ctx, u, dt, dt_used, flags, false, w1, w2);
}

fr_sg_status fr_sg_adjoint_step_stages(fr_sg_ctx* ctx, const double* u_n, const double* w1, const double* w2,
                                       const uint8_t* flags_n, double dt, double* lam, double* dparams) {
  if (!ctx) return FRSG_EINVAL;
  fr_sg_status st = check_adjoint_args(ctx, u_n, flags_n, dt, lam);
  if (st != FRSG_OK) return st;
  if (!w1 || !w2 || w1 == w2 || w1 == lam || w2 == lam) {
    ctx->err = "w1 and w2 must be distinct device state buffers, distinct from lam";
    return FRSG_EINVAL;
  }
  // the transposed passes read dt from the device, as after a recomputation
  FRSG_TRY_HIP(launch_set_dt(ctx->kp, dt, nullptr, nullptr, ctx->stream), ctx);
  return adjoint_from_stages(ctx, u_n, w1, w2, flags_n, dt, lam, dparams);
}

fr_sg_status fr_sg_sync(fr_sg_ctx* ctx) {
  if (!ctx) return FRSG_EINVAL;
  FRSG_TRY_HIP(hipStreamSynchronize(ctx->stream), ctx);
  unsigned status = 0;
  FRSG_TRY_HIP(hipMemcpy(&status, ctx->kp.status, sizeof(unsigned), hipMemcpyDeviceToHost), ctx);
  if (status) {
    unsigned zero = 0;
    FRSG_TRY_HIP(hipMemcpy(ctx->kp.status, &zero, sizeof(unsigned), hipMemcpyHostToDevice), ctx);
  }
  if (status & kStatusNotRealizable) {
    ctx->err = "element mean density or pressure not positive";
    return FRSG_ENOTREALIZABLE;
  }
  if (status & kStatusNonFinite) {
    ctx->err = "non-finite value (time step or wave speed)";
    return FRSG_ENONFINITE;
  }
  return FRSG_OK;
}

fr_sg_status fr_sg_timing_enable(fr_sg_ctx* ctx, int enable) {
  if (!ctx) return FRSG_EINVAL;
  ctx->timing = enable != 0;
  ctx->pending.clear();
  ctx->events_used = 0;
  return FRSG_OK;
}

fr_sg_status fr_sg_timing_read(fr_sg_ctx* ctx, fr_sg_pass_time* out, int32_t capacity, int32_t* count) {
  if (!ctx || !count || (capacity > 0 && !out)) return FRSG_EINVAL;
  FRSG_TRY_HIP(hipStreamSynchronize(ctx->stream), ctx);
  std::vector<PassTotal> tot;
  for (const PassRecord& r : ctx->pending) {
    float ms = 0.0f;
    FRSG_TRY_HIP(hipEventElapsedTime(&ms, ctx->events[r.ev0], ctx->events[r.ev1]), ctx);
    PassTotal* t = nullptr;
    for (auto& x : tot)
      if (x.name == r.name) t = &x;
    if (!t) {
      tot.push_back(PassTotal());
      t = &tot.back();
      t->name = r.name;
      t->alg_bytes = r.alg_bytes;
    }
    t->launches += 1;
    t->ms += ms;
  }
  ctx->pending.clear();
  ctx->events_used = 0;
  int n = 0;
  for (const auto& t : tot) {
    if (n >= capacity) break;
    std::memset(&out[n], 0, sizeof(fr_sg_pass_time));
    std::strncpy(out[n].name, t.name.c_str(), sizeof(out[n].name) - 1);
    out[n].launches = t.launches;
    out[n].total_ms = t.ms;
    out[n].alg_bytes = t.alg_bytes;
    ++n;
  }
  *count = n;
  return FRSG_OK;
}

fr_sg_status fr_sg_destroy(fr_sg_ctx* ctx) {
  if (!ctx) return FRSG_OK;
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t ev : ctx->events) (void)hipEventDestroy(ev);
  delete ctx;
  return FRSG_OK;
}

const char* fr_sg_last_error(const fr_sg_ctx* ctx) {
  if (!ctx) return g_init_error.c_str();
  return ctx->err.c_str();
}

}  // extern "C"
