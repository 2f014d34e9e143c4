// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <functional>
#include <string>
#include <vector>

#include "fr_sg.h"

namespace frsg {

constexpr int kMaxNp1 = 8;      // p <= 7
constexpr int kMaxModes = 128;  // gPC modes
constexpr int kMaxNodes = 256;  // random quadrature nodes

// device status bits (latched, cleared by fr_sg_sync)
constexpr unsigned kStatusNonFinite = 1u;
constexpr unsigned kStatusNotRealizable = 2u;

// ---------------------------------------------------------------------------
// host tables (FP64), built once per context
// ---------------------------------------------------------------------------
struct HostTables {
  int np1 = 0;                     // p + 1 solution points per direction
  std::vector<double> r, w;        // Legendre-Gauss points / weights (sum 2)
  std::vector<double> D;           // D[i*np1 + j] = l_j'(r_i)
  std::vector<double> lL, lR;      // l_j(-1), l_j(+1)
  std::vector<double> dhL, dhR;    // Radau correction derivatives at r_j
  std::vector<double> V, Vinv;     // V[j*np1 + k] = sqrt(2k+1) P_k(r_j)
  int M = 0, Nq = 0, rdim = 1;
  std::vector<std::array<int, 2>> kidx;  // gPC multi-indices
  std::vector<int> kdeg;                 // |k|
  std::vector<double> z;                 // [Nq * rdim]
  std::vector<double> wq;                // [Nq], sum 1
  std::vector<double> Phi, PW;           // [M * Nq]
  std::vector<double> filt;              // [M * nsp]: exp filter exponent sum or L2 factor
  std::vector<double> shell;             // [M * nsp]: 1 on the outer modal shell
  std::vector<double> swts;              // [nsp]: element-mean weights
  std::vector<double> Dt;                // D - h_L' l(-1)^T - h_R' l(+1)^T (np1 x np1)
  std::vector<double> cmax;              // [M]: max_q |Phi_k(z_q)|
  std::vector<double> PhiT, PWT;         // [Nq * M] node-major copies of Phi, PW
  std::vector<double> qfrag;             // matrix-core operand tables (quadrilateral 2D path)
};

// offsets (in doubles) of the matrix-core operand tables of the quadrilateral
// 2D stage kernel (tables_quad.cpp), for nb = ceil(N_q / 16) node blocks:
//   aexp_f [nb][4][64]  chaos basis, FP64 instruction, mode 4 t + lane/16
//   aexp_b [nb][4][64]  chaos basis, FP64 instruction, mode 4 lane/16 + t
//   aprj   [nb][4][64]  weighted basis for the FP64 projection
//   bexp   [nb][2][64]  chaos basis as bfloat16 high / low parts (4 per lane)
//   bprj   [nb][2][64]  weighted basis as bfloat16 high / low parts
//   wslot  [nb][16]     quadrature weight of the node in register r, lane group g
struct QuadFragLayout {
  int nb = 0;
  int aexp_f = 0, aexp_b = 0, aprj = 0, bexp = 0, bprj = 0, wslot = 0, total = 0;
};
__host__ __device__ inline QuadFragLayout quad_frag_layout(int Nq) {
  QuadFragLayout L;
  L.nb = (Nq + 15) / 16;
  L.aexp_f = 0;
  L.aexp_b = L.aexp_f + L.nb * 4 * 64;
  L.aprj = L.aexp_b + L.nb * 4 * 64;
  L.bexp = L.aprj + L.nb * 4 * 64;
  L.bprj = L.bexp + L.nb * 2 * 64;
  L.wslot = L.bprj + L.nb * 2 * 64;
  L.total = L.wslot + L.nb * 16;
  return L;
}
void build_quad_fragments(HostTables& T);

bool build_host_tables(const fr_sg_problem& P, HostTables& T, std::string& err);
// exponent of the exponential filter along one dimension (Sec. 4.1.1): 0 below the
// cutoff eta* (modes untouched), ((eta - eta*) / (1 - eta*))^s from it on
double exp_filter_term(double eta, double eta_star, double s);
// n-point Gauss-Legendre rule (weights sum 2); Gauss-Jordan inverse of an n x n matrix
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);
bool invert_matrix(int n, const std::vector<double>& A, std::vector<double>& Ainv);

// ---------------------------------------------------------------------------
// triangles (element = FRSG_ELEM_TRI): reference operators and per-element geometry
// ---------------------------------------------------------------------------
constexpr int kTriMaxDeg = 4;                                   // p <= 4
constexpr int kTriMaxNp = (kTriMaxDeg + 1) * (kTriMaxDeg + 2) / 2;  // 15 solution points
constexpr int kTriGeo = 16;                                     // doubles of geometry per triangle
// geometry record of a triangle: dr/dx, dr/dy, ds/dx, ds/dy, det (= area / 2),
// unit outward normals (nx, ny) of faces 0..2, the factors (face length /
// reference face length / det) of faces 0..2, inscribed-circle diameter
enum : int { kGeoRx = 0, kGeoRy, kGeoSx, kGeoSy, kGeoDet, kGeoN0 = 5, kGeoSc0 = 11, kGeoDin = 14 };
struct TriTables {
  int p = 0, np = 0, nfp = 0;
  std::vector<double> r, s;        // solution points on the reference triangle
  std::vector<double> Dr, Ds;      // [np][np]: d l_i/dr, d l_i/ds at point j (row j)
  std::vector<double> Lf;          // [3 nfp][np]: l_i at the flux points, face-major
  std::vector<double> lift;        // [np][3 nfp]: divergence of the correction fields
  std::vector<double> mean_w;      // [np]: element mean = sum_j mean_w[j] u_j
  std::vector<double> geo;         // [E][kTriGeo]
  std::vector<int> nbr;            // [E][6]: neighbour element (or -1 - side), then neighbour face
  std::vector<double> xy_pts;      // [E][np][2]: physical solution-point coordinates
  std::vector<double> V, Vinv;     // [np][np]: V[j][m] = psi_m(r_j) and its inverse
};
// reference tables for degree p, mesh checks and geometry from the problem's arrays
bool build_tri_tables(const fr_sg_problem& P, TriTables& T, std::string& err);
// sensor shell, filter factors and element-mean weights of the host tables, by total degree
void tri_filter_tables(const fr_sg_problem& P, const TriTables& R, HostTables& T);

// ---------------------------------------------------------------------------
// device-side view of the tables (one allocation, sub-arrays by offset)
// ---------------------------------------------------------------------------
struct DevTab {
  const double* r;
  const double* w;
  const double* D;
  const double* lL;
  const double* lR;
  const double* dhL;
  const double* dhR;
  const double* V;
  const double* Vinv;
  const double* Phi;
  const double* PW;
  const double* filt;
  const double* shell;
  const double* swts;
  const double* cmax;  // [M] max over the random nodes of |Phi_k|
  const double* PhiT;  // [Nq][M] node-major copies of Phi and PW (one node's modes contiguous)
  const double* PWT;
};

// Everything a kernel needs about the problem, passed by value.
struct KParams {
  int eq, dim;
  int E, nx, ny, nsp, M, Nq, S, np1;
  double dx, dy, Jx, Jy;
  double adv, gamma;
  int bc[4];
  double bc_state[4][4];
  double cfl;
  int filter, sensor, limiter;
  int flux;  // FRSG_FLUX_*
  double alpha, sensor_thr;
  int fp32;  // 1: FP32-mixed node loops (1D stage and adjoint kernels)
  int bf16;  // 1: BF16-split matrix-core transforms (1D stage kernel)
  DevTab tab;
  // triangles (element = FRSG_ELEM_TRI; tri = 0 on quadrilateral meshes)
  int tri, nfp;
  const double* tri_Dr;    // [N_p][N_p]
  const double* tri_Ds;
  const double* tri_Lf;    // [3 nfp][N_p]
  const double* tri_lift;  // [N_p][3 nfp]
  const double* tri_geo;   // [E][kTriGeo]
  const double* tri_V;     // [N_p][N_p] orthonormal modes at the solution points, and inverse
  const double* tri_Vinv;
  const int* tri_nbr;      // [E][6]
  unsigned* status;
  unsigned long long* lam_bits;  // CFL accumulator (bit pattern of a positive double)
  double* dt;                    // device time step of the current step
};

constexpr int kRkMaxTerms = 8;  // stages of the largest tableau integrator, and more

struct Workspace {
  double* w1 = nullptr;
  double* w2 = nullptr;
  double* Un = nullptr;    // [S][Nq][E][nsp] nodal solution, then nodal residual
  double* Fn = nullptr;    // [S][Nq][E][nsp] nodal x-flux
  double* Gn = nullptr;    // [S][Nq][E][nsp] nodal y-flux (2D)
  double* Corr = nullptr;  // [S][Nq][E][nface] interface-flux minus interpolated flux
  // fused triangles: modal traces [S][M][E][3 nfp] of a stage input, two buffers used in turn
  double* Tm[2] = {nullptr, nullptr};
  double* scal = nullptr;  // scalars: dt, lam bits, status
  // adjoint (scalar 1D problems): stage adjoints, trace adjoints, partial sums
  double* avb = nullptr;   // adjoint of the unfiltered end-of-step state
  double* ab2 = nullptr;   // adjoint of w2
  double* ab1 = nullptr;   // adjoint of w1
  double* agT = nullptr;   // [Nq][E][2] adjoints of the traces at r = -1, +1
  double* apart = nullptr; // per-block partial sums of the parameter derivative
  // fused 2D: modal face traces on tile boundaries, written by one stage launch
  // for the next (two buffers, used in turn)
  double* tr[2] = {nullptr, nullptr};
  // tableau integrators: one right-hand-side buffer per stage
  double* rk[kRkMaxTerms] = {nullptr};
  size_t bytes = 0;
};

// byte offsets of the workspace sub-arrays (each 256-byte aligned) and its size
struct Layout {
  size_t sc = 0, tab = 0, f32 = 0, tri = 0, nbr = 0;
  size_t w1 = 0, w2 = 0, un = 0, fn = 0, gn = 0, co = 0;
  size_t avb = 0, ab2 = 0, ab1 = 0, agt = 0, apt = 0;
  size_t tr0 = 0, tr1 = 0, tm0 = 0, tm1 = 0;
  size_t rk[kRkMaxTerms] = {0};
  int nrk = 0;
  bool adj = false, has_tr = false, has_tm = false;
  size_t total = 0;
};

}  // namespace frsg

struct PassRecord {
  std::string name;
  double alg_bytes;
  int ev0, ev1;  // indices into the event pool
};

struct PassTotal {
  std::string name;
  long launches = 0;
  double ms = 0.0;
  double alg_bytes = 0.0;
};

struct fr_sg_ctx {
  fr_sg_problem prob;
  bool timing = false;
  std::vector<hipEvent_t> events;
  int events_used = 0;
  std::vector<PassRecord> pending;
  frsg::HostTables T;
  frsg::TriTables tri;           // triangle operators and geometry (element = FRSG_ELEM_TRI)
  bool is_tri = false;
  bool fused_tri = false;        // fused triangle stage kernel
  hipStream_t stream = nullptr;
  int dim = 1;
  int S = 1;
  int E = 0;
  int nsp = 0;
  const double* dDt = nullptr;
  const double* dcmax = nullptr;
  const double* dPhiT = nullptr;
  const double* dPWT = nullptr;
  const float* dPhiT32 = nullptr;  // FP32 copies of the node-major tables
  const float* dPWT32 = nullptr;
  bool fused = false;            // fused 2D Euler stage kernel (FP32-mixed, and the element-wise passes)
  bool quad = false;             // matrix-core 2D Euler stage kernel (FP64, BF16-split)
  const double* dfrag = nullptr; // its operand tables
  bool fused1d = false;          // fused 1D stage kernel
  bool resident1d = false;       // SSP-RK3 steps of a small 1D problem in one one-workgroup launch
  int lam_cur = 0;              // which CFL accumulator holds the maximum of the current state
  const double* lam_for = nullptr;  // state whose maximum the previous step recorded (fr_sg_steps)
  int tr_cur = 0;               // fused 2D: which face-trace buffer holds the traces of the current state
  int tm_cur = 0;               // fused triangles: which trace buffer holds the traces of the current state
  frsg::KParams kp;
  frsg::Workspace ws;
  frsg::Layout lay;                  // sub-arrays of the caller's workspace
  std::vector<double> host_tab;      // tables waiting for the upload in fr_sg_init
  std::vector<size_t> tab_off;       // offsets of the tables in host_tab (and on the device)
  std::vector<double> host_tri;      // triangle operators and geometry
  std::vector<float> host_f32;       // FP32 chaos tables of the fused 2D path
  std::string err;
};

namespace frsg {
// fr_sg_init's work on a given device workspace (frsg_api.cpp), and the text that
// fr_sg_last_error(NULL) reports after a failed init
// (check_device: confirm that the caller's pointer is device memory)
fr_sg_status init_with_workspace(const fr_sg_problem* problem, void* hip_stream, void* workspace,
                                 int64_t workspace_bytes, fr_sg_ctx** out, bool check_device);
void set_init_error(const std::string& msg);

// one fused stage of the 2D Euler path (kernels_euler2d.hip)
struct RkTerms {
  const double* K[kRkMaxTerms];
  double a[kRkMaxTerms];
  int n;
};
struct FusedStage {
  const double* in;
  const double* u;
  double* out;
  double cu, cw;
  int stage;  // 0: rhs; 1, 2: limited stage output; 3: end of step
  unsigned char* flag_lim;
  unsigned char* flag_filt;
  unsigned long long* lam_next;
  const double* Dt;
  const double* cmax;
  const double* PhiT;  // [Nq][M] chaos basis at the nodes, node-major
  const double* PWT;   // [Nq][M] quadrature-weighted basis, node-major
  int fp32;            // 1: node loop in FP32 (FP32-mixed precision)
  const float* PhiT32;
  const float* PWT32;
  const double* tr_in = nullptr;  // modal face traces of `in` on tile boundaries (null: from the state)
  double* tr_out = nullptr;       // where to write those of `out` (may be null)
  // tab: out = u + dt (sum_j terms.a[j] terms.K[j] + ka_cur R(in)) instead of cu u + cw (in + dt R),
  // R(in) stored in k_out (may be null), limiter flags OR-ed into flag_lim
  int tab = 0;
  RkTerms terms{};
  double ka_cur = 0.0;
  double* k_out = nullptr;
};
bool fused2d_supported(const KParams& P);

// one stage of the matrix-core 2D Euler path on quadrilaterals (kernels_quad_mfma.hip)
struct QuadStage {
  const double* in;
  const double* u;
  double* out;
  double cu, cw;
  int stage;  // 0: rhs; 1, 2: limited stage output; 3: end of step
  unsigned char* flag_lim;
  unsigned char* flag_filt;
  unsigned long long* lam_next;
  const double* Dt;
  const double* cmax;
  const double* frag;   // operand tables (QuadFragLayout)
  int bf16;             // 1: bfloat16-split transforms (FRSG_BF16_SPLIT)
  const double* tr_in;  // modal face traces of `in` on tile boundaries (required)
  double* tr_out;       // where to write those of `out` (may be null)
};
bool quad_mfma_supported(const KParams& P);
// doubles of one modal face-trace buffer of the matrix-core path
size_t quad_trace_count(int nx, int ny, int M);
hipError_t launch_quad_stage(const KParams& P, const QuadStage& S, hipStream_t s);
// modal face traces of a state on every tile boundary face
hipError_t launch_quad_traces(const KParams& P, const double* u, double* tr, hipStream_t s);
// doubles of one modal face-trace buffer of the fused 2D kernel
size_t fused2d_trace_count(int nx, int ny, int M);
hipError_t launch_fused_stage(const KParams& P, const FusedStage& S, hipStream_t s);
hipError_t launch_fused_cfl(const KParams& P, const double* u, unsigned long long* lam, hipStream_t s);
// sensor-gated filter and/or limiter in place, with the fused kernel's tile layout
hipError_t launch_fused_post(const KParams& P, const double* PhiTd, const double* cmax, double* u, int do_filter,
                             int do_limit, unsigned char* flag_filt, unsigned char* flag_lim, hipStream_t s);
hipError_t launch_dt_from(const KParams& P, const unsigned long long* lam, unsigned long long* lam_reset,
                          double* dt_used, hipStream_t s);
hipError_t launch_set_dt(const KParams& P, double dt, double* dt_used, unsigned long long* lam_reset, hipStream_t s);

// launchers (kernels_generic.hip)
hipError_t launch_set_scalars(const KParams& P, double dt_fixed, hipStream_t s);
hipError_t launch_nodal(const KParams& P, const double* u, double* Un, double* Fn, double* Gn, int do_cfl,
                        hipStream_t s);
hipError_t launch_dt(const KParams& P, int dim, double* dt_used, hipStream_t s);
hipError_t launch_faces(const KParams& P, const double* Un, const double* Fn, const double* Gn, double* Corr,
                        hipStream_t s);
hipError_t launch_resid(const KParams& P, const double* Fn, const double* Gn, const double* Corr, double* Rn,
                        hipStream_t s);
hipError_t launch_project_stage(const KParams& P, const double* Rn, const double* u, const double* w,
                                double* out, double cu, double cw, int rhs_only, hipStream_t s);
hipError_t launch_project_ic(const KParams& P, const double* U0, double* u, hipStream_t s);
hipError_t launch_limiter(const KParams& P, double* u, unsigned char* flags, hipStream_t s);
hipError_t launch_sensor_filter(const KParams& P, double* u, unsigned char* flags, hipStream_t s);
hipError_t launch_fill_flags(unsigned char* flags, long n, hipStream_t s);
// triangle passes (kernels_tri.hip): interactive-flux jumps [S][Nq][E][3 nfp],
// nodal residual into Rn, CFL maximum of the nodal values into P.lam_bits
hipError_t launch_faces_tri(const KParams& P, const double* Un, const double* Fn, const double* Gn, double* Jump,
                            hipStream_t s);
hipError_t launch_resid_tri(const KParams& P, const double* Fn, const double* Gn, const double* Jump, double* Rn,
                            hipStream_t s);
hipError_t launch_cfl_tri(const KParams& P, const double* Un, hipStream_t s);
// end-of-stage work of the fused triangle kernels: the sensor-gated filter (flags of the
// filtered elements into flag_filt) and/or the limiter (flags of the limited ones into
// flag_lim); the flag pointers may be null
struct TriPost {
  int filter = 0, limit = 0;
  unsigned char *flag_filt = nullptr, *flag_lim = nullptr;
};
// fused triangle stage (p = 1..4 and the (M, Nq) pairs of the fused 2D kernel): a trace pass
// over `in` into Tm ([S][M][E][3 nfp]) unless traces_ready, then out = cu u + cw (w + dt R(in)),
// or R(in) with rhs_only; `post` on the output (not with rhs_only); with Tm_out the traces
// of the final `out` go there
bool tri_fused_supported(const KParams& P);
hipError_t launch_stage_tri(const KParams& P, const double* in, const double* u, const double* w, double* out,
                            double cu, double cw, int rhs_only, double* Tm, int traces_ready, double* Tm_out,
                            hipStream_t s, const TriPost& post = TriPost());
// positivity limiter on triangles with the fused lane layout (fused (p, M, N_q) set)
hipError_t launch_limit_tri(const KParams& P, double* u, unsigned char* flags, hipStream_t s);
// the sensor-gated filter and/or the limiter of `post` as a pass of its own (same set)
hipError_t launch_post_tri(const KParams& P, double* u, const TriPost& post, hipStream_t s);
// CFL maximum of a modal state on triangles into P.lam_bits
hipError_t launch_cfl_tri_modal(const KParams& P, const double* u, hipStream_t s);
// explicit Runge-Kutta stage combination: out = u + dt sum_j a[j] K[j] (flat state of n doubles)
hipError_t launch_rk_combine(const double* u, const RkTerms& T, const double* dt, double* out, long n,
                             hipStream_t s);
hipError_t launch_or_flags(unsigned char* dst, const unsigned char* src, long n, hipStream_t s);
hipError_t launch_copy_dt(const KParams& P, double* dt_used, hipStream_t s);

// fused 1D stage kernel (kernels_fr1d.hip)
bool fr1d_supported(const KParams& P);
// limit: positivity limiter on the output (flag_lim); end_of_step: detector-
// switched filter before the limiter (flag_filt) and the CFL maximum of the
// output into lam_next (may be null).  dt_source: 0 reads the device dt; 1 uses
// dt_fixed; 2 derives it from lam_in; with 1 or 2 the kernel also publishes dt
// (device dt, dt_used) and zeroes lam_reset.
hipError_t launch_stage1d(const KParams& P, const double* in, const double* u, const double* w, double* out, double cu,
                          double cw, int rhs_only, unsigned char* clear_flags, hipStream_t s, int limit = 0,
                          int end_of_step = 0, unsigned char* flag_lim = nullptr, unsigned char* flag_filt = nullptr,
                          unsigned long long* lam_next = nullptr, int dt_source = 0, double dt_fixed = 0.0,
                          const unsigned long long* lam_in = nullptr, unsigned long long* lam_reset = nullptr,
                          double* dt_used = nullptr);
// one stage of a Butcher-tableau step: out = u + dt (sum_j T.a[j] T.K[j] + ka_cur R(in)),
// R(in) also stored in k_out (may be null); the limiter acts on out (flags OR-ed into
// flag_lim), and with end_of_step the detector-switched filter, the limiter and the CFL
// maximum follow as in the SSP-RK3 stage; dt as in launch_stage1d
hipError_t launch_stage1d_tab(const KParams& P, const double* in, const double* u, double* out, double* k_out,
                              const RkTerms& T, double ka_cur, hipStream_t s, int limit, int end_of_step,
                              unsigned char* flag_lim, unsigned char* flag_filt, unsigned long long* lam_next,
                              int dt_source, double dt_fixed, const unsigned long long* lam_in,
                              unsigned long long* lam_reset, double* dt_used);
hipError_t launch_cfl1d(const KParams& P, const double* u, unsigned long long* lam, hipStream_t s);
// nsteps SSP-RK3 steps (CFL time steps, limiter on every stage output when limit,
// end-of-step filter and CFL maximum) of an FP64 1D problem whose elements fit one
// workgroup, in one launch; lam_in holds the CFL maximum of u, lam_out receives
// that of the result.  flags [nsteps][4][E] and dt_used [nsteps] may be null.
// With u == nullptr: hipSuccess when the problem fits and the instance runs
// without register spills, launching nothing.
bool fr1d_resident_fits(const KParams& P);
bool fr1d_resident_lds_state(const KParams& P);  // the three states stay in LDS for the whole call
hipError_t launch_steps1d_resident(const KParams& P, double* u, double* w1, double* w2, int nsteps, int limit,
                                   unsigned char* flags, double* dt_used, const unsigned long long* lam_in,
                                   unsigned long long* lam_out, hipStream_t s);

// adjoint launchers (kernels_adjoint.hip)
long adjoint_partials(const KParams& P);
hipError_t launch_rhs_adjoint(const KParams& P, const double* Un, const double* g, double* GU, double* Gside,
                              double* gT, const double* x0, const double* x1, const double* x2, double* out,
                              double c0, double c1, double c2, double cg, double* part, double param_scale,
                              double* dparam, hipStream_t s);
bool adj1d_fused_supported(const KParams& P);
long adj1d_partials(const KParams& P);
hipError_t launch_adj_stage1d(const KParams& P, const double* w, const double* g, const double* x0, const double* x1,
                              const double* x2, double* out, double c0, double c1, double c2, double cg, double* part,
                              double param_scale, double* dparam, hipStream_t s);
hipError_t launch_filter_adjoint(const KParams& P, const double* g, const unsigned char* flags, double* out,
                                 hipStream_t s);
}  // namespace frsg
