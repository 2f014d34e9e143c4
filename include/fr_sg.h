/*
 * fr_sg.h -- C ABI of the MI355X flux reconstruction stochastic Galerkin
 * (FR-SG) hot path.
 *
 * Method: Xiao, Kusch, Koellermeier, Frank, "A flux reconstruction stochastic
 * Galerkin scheme for hyperbolic conservation laws" (arXiv 2112.05946).
 *
 * All device pointers are HIP device memory (e.g. torch CUDA tensors on
 * ROCm); host pointers are ordinary memory.  Every call that launches work is
 * asynchronous on the stream given to fr_sg_init (or fr_sg_set_stream); none
 * synchronises except fr_sg_init, fr_sg_query, fr_sg_points and fr_sg_sync.
 * No exception crosses this boundary: every entry point returns a status.
 *
 * State layout (every state-shaped argument): double u[S][M][E][N_sp],
 * C-contiguous, where
 *   S    conserved variables (1 scalar, 3 Euler 1D, 4 Euler 2D),
 *   M    gPC modes (N_c + 1 in 1D random space; (N_c+1)(N_c+2)/2 for the
 *        total-degree set in 2D random space, graded order
 *        (0,0),(1,0),(0,1),(2,0),(1,1),(0,2),...),
 *   E    elements, row-major e = iy * nx + ix (or the triangles in the
 *        caller's order, element = FRSG_ELEM_TRI),
 *   N_sp solution points per element, (p+1)^dim, j = a + (p+1) * b with a
 *        the x index; points are Legendre-Gauss in each direction.  On
 *        triangles N_sp = (p+1)(p+2)/2 warp-and-blend points (see
 *        FRSG_ELEM_TRI).
 * i.e. the gPC coefficients (Sec. 2.1, Eq. polynomial chaos) held at the FR
 * solution points (Sec. 3.2) of each element.
 *
 * Ownership: the caller owns every device buffer: states, right-hand sides,
 * adjoints, flags, time steps, and the workspace handed to fr_sg_init (size
 * from fr_sg_workspace_size).  The workspace holds the operator tables (read
 * by the kernels through the scalar cache, as constant data), the device
 * scalars (time step, CFL accumulators, status word), the stage states of a
 * step, and whatever the problem's path keeps between launches (face traces,
 * nodal scratch, tableau stage buffers, adjoint vectors, triangle geometry).
 * The library owns only the host-side context.  No entry point allocates or
 * frees device memory.
 *
 * Errors: invalid or unsupported problems are rejected by fr_sg_init before
 * any launch.  Non-finite or non-realizable states met on the device are
 * latched in a device status word and returned by the next fr_sg_sync.
 */
#ifndef FR_SG_H
#define FR_SG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FRSG_ABI_VERSION 5

typedef int32_t fr_sg_status;
#define FRSG_OK 0
#define FRSG_EINVAL (-1)          /* bad argument or inconsistent problem            */
#define FRSG_EUNSUPPORTED (-2)    /* valid but not implemented combination           */
#define FRSG_EDEVICE (-3)         /* HIP runtime error (allocation, launch, copy)    */
#define FRSG_ENONFINITE (-4)      /* a non-finite value met on the device            */
#define FRSG_ENOTREALIZABLE (-5)  /* element mean density or pressure not positive   */
#define FRSG_EABI (-6)            /* problem.abi_version != FRSG_ABI_VERSION        */

/* conservation law (Sec. 5: advection, Burgers, Euler 1D, Euler 2D) */
#define FRSG_ADVECTION 0
#define FRSG_BURGERS 1
#define FRSG_EULER1D 2
#define FRSG_EULER2D 3

/* boundary kinds, per side [x-lo, x-hi, y-lo, y-hi] (Sec. 2.1 boundary operator) */
#define FRSG_BC_PERIODIC 0
#define FRSG_BC_DIRICHLET 1   /* ghost = bc_state[side] (conservative variables) */
#define FRSG_BC_OUTFLOW 2     /* ghost = interior trace                           */
#define FRSG_BC_REFLECT 3     /* ghost = interior trace, normal momentum negated  */

/* interactive flux at the element faces (Sec. 3.3), per random node.
 * FRSG_FLUX_HLL: the two-wave HLL solver with Davis's wave speeds
 * S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R), which the
 * paper names for its Euler runs (Tables 5, 6); Euler equations only
 * (fr_sg_init returns FRSG_EUNSUPPORTED for the scalar equations). */
#define FRSG_FLUX_RUSANOV 0
#define FRSG_FLUX_HLL 1

/* time integrator.  FRSG_SSPRK3: three-stage SSP Runge-Kutta (Shu-Osher form),
 * the limiter after each stage, the sensor-gated filter and the limiter at the
 * end (the fused kernels run it with the stage work in one launch per stage).
 * The others are the explicit integrators the paper's tables name, at the same
 * CFL step (no error control): FRSG_RK4 (classical, Table 1),
 * FRSG_RK_BS3 (Bogacki-Shampine 3(2), Tables 5, 6), FRSG_RK_TSIT5 (Tsitouras
 * 5(4), Table 4); stage states Y_i = Lim(u + dt sum_j a_ij K_j), then
 * u <- Lim(Filter(u + dt sum_i b_i K_i)).  They keep one right-hand-side buffer
 * per stage in the workspace and run the right-hand side, the stage
 * combination and the limiter as separate passes; no adjoint. */
#define FRSG_SSPRK3 0
#define FRSG_RK4 1
#define FRSG_RK_BS3 2
#define FRSG_RK_TSIT5 3

/* modal filter (Sec. 4.1.1 exponential, Sec. 4.1.2 L2, Sec. 4.1.3 Lasso).
 * FRSG_FILTER_LASSO: the soft threshold of Eq. LassoFilterFunction with the
 * strengths of Eq. fStrength taken per element and conserved variable from the
 * highest pure spatial and pure chaos coefficients (which it sets to zero);
 * one physical and one random dimension only (dim 1, rdim 1), no adjoint
 * (fr_sg_init returns FRSG_EUNSUPPORTED otherwise, fr_sg_adjoint_step too). */
#define FRSG_FILTER_NONE 0
#define FRSG_FILTER_EXP 1
#define FRSG_FILTER_L2 2
#define FRSG_FILTER_LASSO 3

/* filter switch: every element, or the modal-decay detector of Sec. 4.2 */
#define FRSG_SENSOR_ALWAYS 0
#define FRSG_SENSOR_DETECTOR 1

/* arithmetic of the right-hand side.  FRSG_FP64: everything in FP64.
 * FRSG_FP32_MIXED: the per-node work of the right-hand side (chaos expansion at
 * the node, fluxes, traces, interface fluxes, nodal residual and the Galerkin
 * projection of the modes k >= 1) in FP32 on the FP64 coefficients and tables
 * rounded to FP32; the projection of the mean mode k = 0, state storage, the
 * Runge-Kutta combination, detector, filter, limiter and CFL reduction stay
 * FP64.  Available on the fused 1D path (FR degree <= 7, Nq <= 85), the fused
 * 2D Euler path (FR degree 3, nx divisible by 4, ny by 2, a compiled (M, Nq)
 * pair) and for fr_sg_adjoint_step on the fused adjoint kernel.
 * FRSG_BF16_SPLIT: the chaos expansion and the Galerkin projection on the
 * bfloat16 matrix cores, each operand split into a high and a low bfloat16 part
 * (x = hi + lo to 2^-16 relative) and the products hi*hi + hi*lo + lo*hi
 * accumulated in FP32; fluxes and residual in FP32; the mean-mode projection
 * and everything after the right-hand side as in FRSG_FP32_MIXED.  Available on
 * the 1D stage kernel (at most 16 gPC modes) and the matrix-core 2D Euler
 * kernel (FR degree 3, nx and ny even, a compiled (M, Nq) pair); not for
 * fr_sg_adjoint_step.
 * Elsewhere fr_sg_init returns FRSG_EUNSUPPORTED for the reduced precisions. */
#define FRSG_FP64 0
#define FRSG_FP32_MIXED 1
#define FRSG_BF16_SPLIT 2

/* element shape (Sec. 3.1).  FRSG_ELEM_QUAD: the nx x ny Cartesian mesh of
 * [xlo, xhi] x [ylo, yhi] (or nx line elements in 1D).  FRSG_ELEM_TRI: an
 * unstructured mesh of n_tri straight-sided triangles, each the image of the
 * isosceles right reference triangle (-1,-1), (1,-1), (-1,1) under
 * x = lam1 x1 + lam2 x2 + lam3 x3 (Sec. 3.1), 2D Euler only.  Its FR form is
 * that of Sec. 3.5: solution points are the warp-and-blend nodes (equispaced
 * lattice warped so that the edge nodes are Legendre-Gauss-Lobatto points;
 * rows of constant s bottom to top, r increasing in a row), p+1
 * Legendre-Gauss flux points per face, and the vector correction fields are
 * the ones that make FR equal to nodal DG (normal component 1 at their own
 * flux point and 0 at the others, zero moments against vector polynomials of
 * degree p-1), whose divergence is the DG lifting.  FR degree 1..4.  Mesh
 * arrays (host memory, read during fr_sg_init only, copied):
 *   tri_xy[n_tri][3][2]   vertex coordinates, counter-clockwise;
 *   tri_nbr[n_tri][3]     across face f (vertex f to vertex f+1 mod 3): the
 *                         neighbouring triangle, or -1 - side for a boundary
 *                         face whose ghost state follows bc[side] (side 0..3;
 *                         that bc must not be FRSG_BC_PERIODIC: periodicity is
 *                         expressed by the neighbour links themselves);
 *   tri_nbr_face[n_tri][3] the neighbour's face index (ignored on boundary
 *                         faces); links must be mutual.
 * Reflection mirrors the velocity about the face.  CFL step:
 * dt = cfl / ((p+1) max(lambda / d_e)) with lambda = |v| + c over the nodes
 * and points of element e and d_e its inscribed-circle diameter.  Shock
 * capturing (Sec. 4) on triangles: a mode of the orthonormal triangle basis
 * carries its total degree d; the detector's outer shell is d = p or
 * |k| = N_c, the exponential filter exponent (d/p)^s + (|k|/N_c)^s, the L2
 * penalty d^2 (d+1)^2 / (eps1 p^2 (p+1)^2) plus the chaos term; the limiter
 * tests the solution and flux points at every node.  Not available on
 * triangles: the Lasso filter, FP32-mixed, the adjoint (fr_sg_init returns
 * FRSG_EUNSUPPORTED; fr_sg_adjoint_step too). */
#define FRSG_ELEM_QUAD 0
#define FRSG_ELEM_TRI 1

typedef struct fr_sg_problem {
  int32_t abi_version;     /* FRSG_ABI_VERSION                                        */
  int32_t equation;        /* FRSG_ADVECTION .. FRSG_EULER2D                          */
  int32_t nx, ny;          /* elements per direction (ny ignored in 1D)               */
  double xlo, xhi, ylo, yhi;
  int32_t bc[4];           /* FRSG_BC_* for x-lo, x-hi, y-lo, y-hi                    */
  double bc_state[4][4];   /* Dirichlet ghost states, conservative                    */
  int32_t fr_degree;       /* p, 1..7; p+1 Legendre-Gauss points, Radau correction    */
  int32_t rdim;            /* random dimensions, 1 or 2, i.i.d. U(-1, 1)              */
  int32_t gpc_order;       /* N_c, total degree of the Legendre chaos                 */
  int32_t nq1d;            /* Gauss-Legendre nodes per random dimension, >= N_c + 1   */
  double adv_speed;        /* a in u_t + a u_x = 0                                    */
  double gamma;            /* ratio of specific heats                                 */
  int32_t filter;          /* FRSG_FILTER_*                                           */
  double alpha, s;         /* exponential filter strength and order                   */
  double nstar;            /* exponential filter cutoff N* (>= 0) of Sec. 4.1.1: per dimension,
                              modes with eta below eta_c are untouched and above it eta is
                              replaced by (eta - eta_c) / (1 - eta_c), with eta_c = nstar / p
                              in physical space (degree j / p per direction, total degree on
                              triangles) and nstar / N_c in random space (|k| / N_c).  Needs
                              nstar < p and nstar < N_c (N_c > 0); 0 filters every mode
                              above the mean                                            */
  double eps1, eps2;       /* L2 filter damping of the last spatial / chaos mode      */
  int32_t sensor;          /* FRSG_SENSOR_*                                           */
  double s0, kappa;        /* detector parameters, Eq. (detector), s_e = log10(S_e)   */
  int32_t limiter;         /* 1: positivity-preserving limiter (Euler only)           */
  double cfl;              /* dt = cfl dx / ((p+1) lambda_max) (1D); 2D analogue      */
  int32_t precision;       /* FRSG_FP64, FRSG_FP32_MIXED or FRSG_BF16_SPLIT           */
  int32_t flux;            /* FRSG_FLUX_RUSANOV (Lax-Friedrichs) or FRSG_FLUX_HLL     */
  int32_t integrator;      /* FRSG_SSPRK3, FRSG_RK4, FRSG_RK_BS3, FRSG_RK_TSIT5       */
  int32_t element;         /* FRSG_ELEM_QUAD or FRSG_ELEM_TRI                         */
  int32_t n_tri;           /* triangles (FRSG_ELEM_TRI; nx, ny, domain ignored)       */
  const double* tri_xy;    /* host, [n_tri][3][2]                                     */
  const int32_t* tri_nbr;  /* host, [n_tri][3]                                        */
  const int32_t* tri_nbr_face; /* host, [n_tri][3]                                    */
} fr_sg_problem;

typedef struct fr_sg_info {
  int64_t n_elem;          /* E                                                       */
  int32_t nsp;             /* N_sp                                                    */
  int32_t n_modes;         /* M                                                       */
  int32_t n_nodes;         /* N_q (nq1d^rdim)                                         */
  int32_t n_states;        /* S                                                       */
  int64_t n_dof;           /* S * M * E * N_sp                                        */
  int64_t state_bytes;     /* 8 * n_dof                                               */
  int64_t flags_len;       /* 4 * E: see fr_sg_step                                   */
  int64_t workspace_bytes; /* bytes of the caller's workspace the context uses           */
} fr_sg_info;

typedef struct fr_sg_ctx fr_sg_ctx;

/* Bytes of device workspace that fr_sg_init needs for this problem (Sec. 1
 * problem statement, Sec. 2.1 gPC degree and quadrature, Sec. 3.1 mesh,
 * Sec. 3.2 FR degree).  Validates the problem exactly as fr_sg_init does and
 * returns the same status for an invalid or unsupported one.  Host only: no
 * HIP call, usable without a device. */
fr_sg_status fr_sg_workspace_size(const fr_sg_problem* problem, int64_t* bytes);

/* Validate the problem, build the operator tables in FP64 on the host
 * (Legendre-Gauss points, Lagrange derivative matrix, Radau correction
 * derivatives, Vandermonde matrix, chaos basis at the Gauss nodes, filter
 * factors), and copy them into the caller's workspace on hip_stream (a
 * hipStream_t; NULL = default stream), then synchronise that stream.
 * workspace: device memory, 256-byte aligned, of workspace_bytes >=
 * fr_sg_workspace_size(problem) bytes; owned by the caller, who keeps it
 * alive and unused by anything else until fr_sg_destroy.  Allocates no
 * device memory.  Invalid problems are rejected before any HIP call; a
 * missing, short, misaligned or non-device workspace gives FRSG_EINVAL.  On
 * failure *out is NULL and nothing is kept. */
fr_sg_status fr_sg_init(const fr_sg_problem* problem, void* hip_stream, void* workspace, int64_t workspace_bytes,
                        fr_sg_ctx** out);

/* fr_sg_init for callers that cannot allocate device memory (code under HIP
 * graph capture of the later calls, tight serving loops, harnesses that forbid
 * hipMalloc): the workspace is a fixed 64 MiB array inside the library's device
 * image, one per GPU, held from the library's first use on that GPU until the
 * process ends; the caller passes no workspace.  Problems whose
 * fr_sg_workspace_size exceeds 64 MiB are rejected with FRSG_EUNSUPPORTED and a
 * message naming both sizes.  Every context made by this call on one GPU shares
 * that GPU's array: a later fr_sg_init_static on the same GPU overwrites the
 * tables and scalars of the earlier contexts (destroy them first), and calls on
 * such contexts that overlap in time race.  The array keeps the last call's
 * contents; this call clears the device scalars (time step, CFL accumulators,
 * status word) and uploads the tables, and every other part of the workspace is
 * written before it is read.  Otherwise as fr_sg_init (synchronises the
 * stream; allocates and frees no device memory). */
fr_sg_status fr_sg_init_static(const fr_sg_problem* problem, void* hip_stream, fr_sg_ctx** out);

/* Sizes of the problem (host struct out). */
fr_sg_status fr_sg_query(const fr_sg_ctx* ctx, fr_sg_info* out);

/* Replace the stream used by later launches. */
fr_sg_status fr_sg_set_stream(fr_sg_ctx* ctx, void* hip_stream);

/* Coordinates of the library's solution points and random nodes, host arrays:
 * x[E*N_sp], y[E*N_sp] (zeros in 1D) in the state's (e, j) order, and
 * z[N_q*rdim] with node q = a + nq1d * b (first coordinate fastest).  Any
 * pointer may be NULL. */
fr_sg_status fr_sg_points(const fr_sg_ctx* ctx, double* x, double* y, double* z);

/* Galerkin projection of nodal initial data (Sec. 2.1, Eq. sg conservation
 * laws, initial condition u_k = <u0 Phi_k> by the quadrature of Eq. discrete
 * expectation value).  u0_nodal: device, double[S][N_q][E][N_sp], values at
 * the points of fr_sg_points; u: device state, fully overwritten. */
fr_sg_status fr_sg_project(fr_sg_ctx* ctx, const double* u0_nodal, double* u);

/* Positivity-preserving limiter of Sec. 4.3 applied in place to a state
 * (Euler problems with limiter = 1; otherwise a no-op that clears flags).
 * flags: device uint8[E] or NULL; 1 where the limiter acted. */
fr_sg_status fr_sg_limit(fr_sg_ctx* ctx, double* u, uint8_t* flags);

/* Semi-discrete right-hand side du/dt = -div f (Sec. 3.2-3.5, Eq. fr
 * update): gPC expansion at the random nodes, flux, Lax-Friedrichs interface
 * flux per node, Radau correction, Galerkin projection.  u, dudt: device
 * states, distinct; dudt fully overwritten.  No limiter or filter. */
fr_sg_status fr_sg_rhs(fr_sg_ctx* ctx, const double* u, double* dudt);

/* One three-stage SSP Runge-Kutta step in place (limit after each stage,
 * sensor-gated filter then limiter at the end of the step; the paper's
 * limit/update/filter order of Eq. schemefullDiscr applied stage-wise).
 * dt > 0: fixed step.  dt <= 0: dt from the CFL condition on u at the start
 * of the step (maximum over solution points x random nodes).
 * dt_used: device double[1] or NULL, receives the step used.
 * flags: device uint8[4*E] or NULL: [0*E+e] limiter after stage 1,
 * [1*E+e] limiter after stage 2, [2*E+e] sensor/filter at the end of the
 * step, [3*E+e] limiter at the end of the step (1 = acted).  With a tableau
 * integrator (RK4, Bogacki-Shampine, Tsitouras) the step is
 * Y_i = Lim(u + dt sum_{j<i} a_ij K_j), K_i = R(Y_i), u <- Lim(Filter(u + dt
 * sum_i b_i K_i)); row 0 then flags the limiter acting on any stage state and
 * row 1 is 0. */
fr_sg_status fr_sg_step(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags);

/* nsteps CFL steps in a row (dt from the CFL condition at the start of each
 * step), in place.  The wave-speed maximum of the first step is computed from
 * u; that of every later step is taken in the previous step's end-of-step
 * pass, so a time loop makes no extra pass over the state for it.  On the
 * fused 2D path the face traces of the neighbours that a stage needs come
 * from the previous launch in the same way (the first stage of the call
 * interpolates them from u).  The end-of-step pass evaluates the wave speeds
 * in another order than the separate CFL pass of fr_sg_step, so a time step
 * can differ from that of a separate fr_sg_step call in the last bits; given
 * equal time steps the states are equal bit for bit.  A scalar 1D problem in
 * FP64 of FR degree <= 3 whose elements fit one workgroup ((E + 2) N_q <=
 * 1024, its stage data within 64 KB of LDS) runs the SSP-RK3 steps of the
 * call in one launch of one workgroup, with the same per-element arithmetic.
 * dt_used: device double[nsteps] or NULL; flags: device uint8[nsteps * 4 * E]
 * or NULL, laid out per step as in fr_sg_step. */
fr_sg_status fr_sg_steps(fr_sg_ctx* ctx, double* u, int32_t nsteps, double* dt_used, uint8_t* flags);

/* Discrete adjoint of one fr_sg_step (the paper has no adjoint; this is the
 * exact transpose of the step as computed here: Sec. 3.2-3.4 right-hand side,
 * the SSP-RK3 stages, the Sec. 4.1 filter) at frozen switch decisions and
 * frozen dt:
 *   lam <- (d u_{n+1} / d u_n)^T lam,
 * where u_{n+1} = fr_sg_step(u_n, dt) produced the filter flags flags_n.  The
 * stage states are recomputed from u_n with the forward passes.  The
 * Lax-Friedrichs dissipation speed is differentiated through the side that
 * attains the maximum.  Covers the scalar 1D equations (advection, Burgers) in
 * FP64 and FP32-mixed (the transposed right-hand side's node and face work in
 * FP32, its mean mode and the stage chain in FP64, the stage states recomputed
 * by the FP32-mixed forward kernel); other problems and BF16-split return
 * FRSG_EUNSUPPORTED.
 * u_n: device state at the start of the step (not modified).
 * flags_n: device uint8[4*E] of that step as written by fr_sg_step (row 2,
 *   the filter decisions, is used); may be NULL when the problem has no filter.
 * dt: the step's dt (> 0), as returned in dt_used.
 * lam: device state-shaped array; in: adjoint of u_{n+1}, out: adjoint of u_n.
 *   Must not alias u_n.
 * dparams: device double[2] or NULL; [0] += d<lam_{n+1}, u_{n+1}>/d adv_speed
 *   at fixed u_n and dt (zero for Burgers), [1] (gamma) is left unchanged.
 * Asynchronous on the context's stream; uses the context's workspace, so calls
 * on one context must not overlap. */
fr_sg_status fr_sg_adjoint_step(fr_sg_ctx* ctx, const double* u_n, const uint8_t* flags_n, double dt, double* lam,
                                double* dparams);

/* fr_sg_step that also leaves its first and second SSP-RK3 stage states
 * (w1 = u + dt R(u), w2 = 3/4 u + 1/4 (w1 + dt R(w1))) in the caller's w1 and
 * w2, for fr_sg_adjoint_step_stages (a checkpointed gradient's recomputation
 * keeps them instead of having every adjoint step recompute them).  Same
 * arguments and results as fr_sg_step otherwise.  Covered where the adjoint
 * runs on the fused 1D stage kernel (scalar 1D equations, SSP-RK3; else
 * FRSG_EUNSUPPORTED).  w1, w2: device state-shaped arrays, distinct from each
 * other and from u (else FRSG_EINVAL), written in full. */
fr_sg_status fr_sg_step_stages(fr_sg_ctx* ctx, double* u, double dt, double* dt_used, uint8_t* flags, double* w1,
                               double* w2);

/* fr_sg_adjoint_step given the step's stage states from fr_sg_step_stages
 * instead of recomputing them: the same transposed passes in the same order, so
 * the same result bit for bit, two launches fewer.  w1, w2: device state-shaped
 * arrays (read only), distinct from each other and from lam (else FRSG_EINVAL);
 * the other arguments, conditions and errors as for fr_sg_adjoint_step. */
fr_sg_status fr_sg_adjoint_step_stages(fr_sg_ctx* ctx, const double* u_n, const double* w1, const double* w2,
                                       const uint8_t* flags_n, double dt, double* lam, double* dparams);

/* Synchronise the stream and return (then clear) the latched device status:
 * FRSG_OK, FRSG_ENONFINITE or FRSG_ENOTREALIZABLE. */
fr_sg_status fr_sg_sync(fr_sg_ctx* ctx);

/* Per-pass device timing.  While enabled, every pass launched by fr_sg_rhs,
 * fr_sg_step and fr_sg_limit is bracketed by a pair of HIP events recorded on
 * the context's stream; fr_sg_timing_read synchronises the stream, sums the
 * elapsed times per pass name and clears the record.  Enabling (or disabling)
 * clears the record too.  Each entry also states the algorithmic HBM bytes of
 * one launch of that pass (the state-sized arrays the method has to read and
 * write in it, 8 bytes per coefficient; 0 for passes that only move
 * intermediate data). */
typedef struct fr_sg_pass_time {
  char name[32];           /* pass name, NUL-terminated                              */
  int64_t launches;        /* launches recorded                                      */
  double total_ms;         /* summed event-to-event device time                      */
  double alg_bytes;        /* algorithmic HBM bytes of one launch                    */
} fr_sg_pass_time;

fr_sg_status fr_sg_timing_enable(fr_sg_ctx* ctx, int enable);

/* out: host array of `capacity` entries; *count receives the number written. */
fr_sg_status fr_sg_timing_read(fr_sg_ctx* ctx, fr_sg_pass_time* out, int32_t capacity, int32_t* count);

/* Free the host-side context (the caller then frees the workspace).  NULL is
 * accepted. */
fr_sg_status fr_sg_destroy(fr_sg_ctx* ctx);

/* Text of the last error on this context (or of the last failed fr_sg_init,
 * fr_sg_workspace_size or fr_sg_copy when ctx is NULL).  Valid until the next
 * call on the same context. */
const char* fr_sg_last_error(const fr_sg_ctx* ctx);

/* Measurement utility, not part of the method: dst[i] = src[i] for i < n with
 * the library's streaming copy kernel (16-byte vector loads and stores, one
 * workgroup per contiguous 32 KiB block), enqueued on
 * hip_stream (NULL: the default stream).  It is the bandwidth reference beside
 * the HBM peak and the kernel of known traffic (8 n bytes read, 8 n bytes
 * written) that calibrates the HBM byte counters of the stage kernels.
 * src, dst: device arrays of n doubles, 16-byte aligned, not overlapping.
 * Returns FRSG_EINVAL for a bad argument (before any device call) and
 * FRSG_EDEVICE for a launch error; asynchronous otherwise. */
fr_sg_status fr_sg_copy(const double* src, double* dst, int64_t n, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FR_SG_H */
