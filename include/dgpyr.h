/*
 * dgpyr -- time-explicit DG for first-order linear acoustics on meshes of
 * vertex-mapped pyramids, with the semi-nodal orthogonal basis of
 * Chan & Warburton, "Orthogonal bases for vertex-mapped pyramids" (Lemma 3).
 *
 * C ABI.  Every call returns a dgpyr_status (0 = success, < 0 = error) and never
 * aborts or throws; on failure a thread-local message is available from
 * dgpyr_last_error().  Device pointers are HIP device addresses; streams are
 * hipStream_t handles passed as void* (NULL = the null stream).
 *
 * Method (Section 4.3): for piecewise-constant density rho and bulk modulus
 * kappa the semi-discrete system is
 *   dp/dt   = -kappa M^-1 ( sum_k S^k u_k + L^f P_p )
 *   du_k/dt = -(1/rho) M^-1 ( S^k p + L^{f,k} P_u ),
 * with S^k the strong derivative matrices (Algorithm 1), L^f, L^{f,k} the
 * surface lifts of the penalty terms P_p = 1/2 (n.[[u]] - tau_p [[p]]) and
 * P_u = 1/2 ([[p]] - tau_u n.[[u]]) (Algorithm 2), [[q]] = q+ - q-,
 * tau_p = alpha / {rho c}, tau_u = alpha {rho c}, {.} the arithmetic mean, and
 * M the mass matrix, diagonal in the semi-nodal basis (Lemma 3).  Time
 * integration is the low-storage RK(5,4) of Carpenter and Kennedy
 * (Section 4.1, Algorithm 3).
 */
#ifndef DGPYR_H
#define DGPYR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DGPYR_OK = 0,
  DGPYR_E_ARG = -1,            /* null pointer, bad size or bad option            */
  DGPYR_E_ORDER = -2,          /* N outside [0, DGPYR_MAX_ORDER]                   */
  DGPYR_E_MESH = -3,           /* degenerate or inverted pyramid (J <= 0)          */
  DGPYR_E_NONCONFORMING = -4,  /* a face is shared by more than two elements, or
                                  the two sides' face points do not coincide       */
  DGPYR_E_HIP = -5,            /* a HIP runtime call failed                        */
  DGPYR_E_OOM = -6,            /* device allocation failed                         */
  DGPYR_E_STATE = -7,          /* context not usable for this call                 */
  DGPYR_E_UNSUPPORTED = -8     /* option combination not built                     */
} dgpyr_status;

#define DGPYR_MAX_ORDER 8

typedef enum {
  DGPYR_BC_WALL = 0, /* rigid wall n.u = 0: mirror p+ = p-, u+ = u- - 2 (n.u-) n */
  DGPYR_BC_FREE = 1  /* free surface p = 0: mirror p+ = -p-, u+ = u-            */
} dgpyr_bc;

typedef enum {
  DGPYR_FP64 = 0,      /* every step in FP64                                         */
  DGPYR_FP32_MFMA = 1, /* volume and lift contractions in FP32 on the matrix cores
                          with FP32 accumulation; geometry, traces, flux, inverse
                          mass and RK state in FP64                                  */
  DGPYR_SPLIT_BF16 = 2 /* as FP32_MFMA, operators split into bf16 hi + lo parts      */
} dgpyr_precision;

/* Mesh, read on the host during dgpyr_setup only (the caller keeps ownership).
 * Element e has vertices e2v[5e .. 5e+4] = (v0, v1, v2, v3, v4): v0..v3 is the
 * base, counter-clockwise seen from the apex v4, i.e.
 * ((x1 - x0) x (x3 - x0)) . (x4 - x0) > 0.  In collapsed coordinates
 * (Section 2) v0 sits at (a, b) = (-1, -1), v1 at (1, -1), v2 at (1, 1),
 * v3 at (-1, 1); the vertex map is x = (1-c)/2 B(a, b) + (1+c)/2 x4 with B the
 * bilinear interpolant of the base, which equals the map built from
 * Bedrosian's vertex functions. */
typedef struct {
  int64_t nverts;
  const double* xyz;    /* [nverts][3]                                            */
  int64_t nelems;
  const int64_t* e2v;   /* [nelems][5], entries in [0, nverts)                    */
  const double* rho;    /* [nelems] density, or NULL for 1                         */
  const double* kappa;  /* [nelems] bulk modulus, or NULL for 1                    */
  int32_t bc;           /* dgpyr_bc, applied on every face without a neighbour    */
  int32_t nsources;     /* number of point sources (0 = none)                      */
  const double* sources;/* [nsources][6]: x, y, z, amplitude, f0, delay; source s
                           adds amplitude R(t) delta(x - x_s) to the pressure
                           equation (the right-hand side f of Section 4.3), with
                           the Ricker wavelet R(t) = (1 - 2 a) exp(-a),
                           a = (pi f0 (t - delay))^2 (delay <= 0 means 1/f0).  At
                           most one source per element.                          */
} dgpyr_mesh;

/* dgpyr_opts.flags bits */
#define DGPYR_FLAG_REFERENCE_KERNELS 1u /* plain FP64 vector-ALU kernels instead of the
                                           matrix-core ones (same results to roundoff) */
#define DGPYR_FLAG_UNFUSED 2u           /* matrix-core volume and surface as separate
                                           launches instead of one fused stage kernel */
#define DGPYR_FLAG_SUM_FACTORIZED 4u    /* FP64 sum-factorised evaluation of the same
                                           contractions through the collapsed tensor
                                           structure of the basis (the cheaper volume
                                           integrals of Section 4.4): O(N^4) instead
                                           of O(N^6) flops per element; on meshes of
                                           hexahedra split into 6 pyramids (groups of
                                           6 consecutive elements around one apex)
                                           and N <= 5 the triangle-face traces stay
                                           on chip.
                                           FP64 precision form only (else
                                           E_UNSUPPORTED); E_UNSUPPORTED too if a
                                           kernel's resources exceed the device's */
#define DGPYR_FLAG_ADJOINT 8u           /* reserve at setup every device buffer the
                                           discrete-adjoint calls use (ten state-sized
                                           arrays, one trace-sized array) and receiver
                                           tables for up to DGPYR_MAX_RESERVED_RECEIVERS
                                           points, so that no later call allocates
                                           device memory                          */

#define DGPYR_FLAG_WATCHDOG 16u         /* after every LSRK step of dgpyr_step and
                                           dgpyr_step_timed, check the state for
                                           NaN or infinite entries (one extra read
                                           of U per step, no change to the results);
                                           read the outcome with dgpyr_watchdog  */

#define DGPYR_MAX_RESERVED_RECEIVERS 4096

typedef struct {
  int32_t precision; /* dgpyr_precision                                           */
  double alpha;      /* penalty scale: 0 = central flux, 1 = the flux of 4.3      */
  uint32_t flags;    /* DGPYR_FLAG_* bits; others must be 0                       */
} dgpyr_opts;

typedef struct {
  int32_t N;               /* polynomial degree                                    */
  int32_t Np;              /* basis functions per element (N+1)(N+2)(2N+3)/6       */
  int32_t Nc;              /* volume cubature points (N+1)^3                       */
  int32_t Nfc;             /* surface cubature points 5 (N+1)^2                    */
  int64_t nelems;          /* K                                                    */
  int64_t state_len;       /* doubles in one state array (U, R or dU/dt)           */
  int64_t canon_len;       /* doubles in the canonical array, K * nfields * Np     */
  double inv_length_max;   /* max over elements of c_K |dK| / |K|                  */
  int32_t hex_groups;      /* 1 if elements come in groups of 6 sharing an apex    */
  int32_t precision;       /* precision form built                                 */
  int64_t device_bytes;    /* device memory held by the context                    */
  int32_t groups_per_wave; /* 4-element groups per wave of the fused matrix-core
                              kernels (dgpyr_set_groups)                         */
  int32_t nfields;         /* fields per element: 4 (acoustics: p, u, v, w) or 1
                              (advection)                                         */
} dgpyr_info;

typedef struct dgpyr_ctx dgpyr_ctx;

/* Build reference rules, basis and operators on the host in FP64 (Lemma 3,
 * Section 4.1 minimal rule), per-element geometry and face connectivity, and
 * upload them to the current HIP device.  Synchronous.  On failure *out is
 * set to NULL.  Errors: E_ARG (null pointers, bad bc/precision/flags),
 * E_ORDER, E_MESH (J <= 0 at a base corner or degenerate vertex map),
 * E_NONCONFORMING, E_UNSUPPORTED, E_OOM, E_HIP. */
dgpyr_status dgpyr_setup(const dgpyr_mesh* mesh, int32_t N, const dgpyr_opts* opts,
                         void* stream, dgpyr_ctx** out);

/* Sizes and derived quantities of a context. */
dgpyr_status dgpyr_get_info(const dgpyr_ctx* ctx, dgpyr_info* info);

/* Time step of the CFL rule of Section 4.3: the spectral radius of the
 * semi-discrete operator grows like C_N max_K c_K |dK| / |K| with
 * C_N = 2 (N+1)(N+3)/3, so *dt = cfl / (C_N max_K c_K |dK| / |K|) for the
 * context's current material (advection: |beta| in place of c_K).  E_ARG for
 * cfl <= 0 or a null pointer. */
dgpyr_status dgpyr_stable_dt(const dgpyr_ctx* ctx, double cfl, double* dt);

/* Convert between the canonical layout and the library's state layout.
 * Canonical: [K][4][Np], fields p, u, v, w; basis index
 * n(i, j, k) = k(k+1)(2k+1)/6 + j(k+1) + i for phi_ijk of Lemma 3 with the
 * Jacobi factor in its standard normalisation.  Both pointers are device
 * arrays of canon_len and state_len doubles; asynchronous on the stream. */
dgpyr_status dgpyr_pack(dgpyr_ctx* ctx, const double* canon, double* U, void* stream);
dgpyr_status dgpyr_unpack(dgpyr_ctx* ctx, const double* U, double* canon, void* stream);

/* dUdt = full semi-discrete right-hand side of Section 4.3 at state U
 * (inverse mass and material factors included).  U and dUdt are device state
 * arrays (may not alias).  t is the time at which the point sources of the
 * mesh (dgpyr_mesh.sources) are evaluated; without sources it has no effect.
 * Asynchronous on the stream. */
dgpyr_status dgpyr_rhs(dgpyr_ctx* ctx, const double* U, double* dUdt, double t, void* stream);

/* nsteps LSRK(5,4) steps of size dt (Algorithm 3): per stage
 * R <- A_s R + dt rhs(U), U <- U + B_s R.  U and R are device state arrays,
 * updated in place; R need not be initialised (A_1 = 0).  Asynchronous. */
dgpyr_status dgpyr_step(dgpyr_ctx* ctx, double* U, double* R, double t0, double dt,
                        int32_t nsteps, void* stream);

/* As dgpyr_step, and also times every kernel launch with HIP events recorded
 * on the stream around it.  kernel_ms[k] receives the summed milliseconds and
 * launches[k] the launch count of kernel kind k, for k < nk (kinds are named by
 * dgpyr_kernel_names).  Returns after the work has completed (synchronises
 * the stream).  For measurement; the numerical result equals dgpyr_step's. */
dgpyr_status dgpyr_step_timed(dgpyr_ctx* ctx, double* U, double* R, double t0, double dt,
                              int32_t nsteps, void* stream, int32_t nk, double* kernel_ms,
                              int64_t* launches);

/* Outcome of the NaN/Inf watchdog (contexts set up with DGPYR_FLAG_WATCHDOG):
 * synchronises the stream, then sets *first_bad_step to -1 if every state
 * checked since setup or the previous dgpyr_watchdog call was finite, else to
 * the 0-based index, counted over the steps of those calls, of the first step
 * after which the state held a NaN or an infinite entry; then starts a new
 * count.  No physics of the method is involved: the paper's scheme is stable
 * under the CFL rule of Section 4.3, and the check catches steps taken beyond
 * it or corrupted input.  Errors: E_ARG (null pointer), E_STATE (context set up
 * without the flag), E_HIP. */
dgpyr_status dgpyr_watchdog(dgpyr_ctx* ctx, int64_t* first_bad_step, void* stream);

/* Semicolon-separated names of the kernel kinds dgpyr_step launches, in the
 * order used by dgpyr_step_timed; the string lives as long as the context. */
const char* dgpyr_kernel_names(const dgpyr_ctx* ctx);

/* Transposed operator for the discrete adjoint (Sections 4.1-4.3 read as
 * dU/dt = A U + b, A = -Kmat M^-1 (volume + surface), Kmat = kappa on
 * pressure rows and 1/rho on velocity rows): out = A^T lam, exactly the
 * transpose of what dgpyr_rhs applies (without sources), for any flux alpha
 * and boundary condition.  lam, out: device state arrays (may not alias).
 * FP64 matrix-core kernels in every precision form.  Uses one state-sized
 * scratch array held by the context: reserved at setup with
 * DGPYR_FLAG_ADJOINT, otherwise allocated by the first call.
 * Asynchronous. */
dgpyr_status dgpyr_adjoint_rhs(dgpyr_ctx* ctx, const double* lam, double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result
 * as dgpyr_adjoint_rhs, with its state-sized scratch (M^-1 Kmat lam) in a
 * static device array of DGPYR_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends (its address is looked up once
 * per device by dgpyr_setup).  The call allocates nothing and calls no
 * allocating routine; the traces go to the context's trace buffer, as in
 * dgpyr_adjoint_rhs.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (every entry the call reads it writes
 * first): calls that overlap in time on one GPU race, so serialise them (one
 * stream, or events).  Errors: E_ARG when 4 K Np doubles exceed the array
 * (then nothing is launched), null or aliasing arrays; E_UNSUPPORTED on an
 * advection context.  Asynchronous. */
#define DGPYR_NOALLOC_SCRATCH_BYTES (64u << 20)
dgpyr_status dgpyr_adjoint_rhs_noalloc(dgpyr_ctx* ctx, const double* lam, double* out,
                                       void* stream);

/* ---- Discrete adjoint: gradient of a receiver misfit w.r.t. kappa --------
 * New per-element bulk modulus kappa = rho c^2 (host array [nelems], rho
 * unchanged): impedances rho c, the per-element CFL length scales
 * c_K |dK| / |K| and their maximum (dgpyr_info.inv_length_max,
 * dgpyr_stable_dt) follow the new sound speeds.  Synchronous. */
dgpyr_status dgpyr_set_kappa(dgpyr_ctx* ctx, const double* kappa);

/* Receiver points (host xyz [nrec][3]), located on the host in the element
 * (lowest index) containing each; several may share an element.  With
 * DGPYR_FLAG_ADJOINT the tables go into the space reserved at setup (E_ARG
 * for more than DGPYR_MAX_RESERVED_RECEIVERS points); otherwise a call with
 * more points than any earlier one allocates device memory held by the
 * context.  E_ARG for a point in no element. */
dgpyr_status dgpyr_set_receivers(dgpyr_ctx* ctx, int32_t nrec, const double* xyz);

/* Pressure at the receivers: out[r] = sum_i phi_i(xi_r) U[e_r][p][i]
 * (device out [nrec]).  Asynchronous. */
dgpyr_status dgpyr_receivers_sample(dgpyr_ctx* ctx, const double* U, double* out, void* stream);

/* Adjoint of the sampling: Ubar[e_r][p][i] += coef[r] phi_i(xi_r) (device coef
 * [nrec]).  Asynchronous. */
dgpyr_status dgpyr_receivers_inject(dgpyr_ctx* ctx, double* Ubar, const double* coef,
                                    void* stream);

/* Reverse of one LSRK(5,4) step (Algorithm 3) of size dt from time t0 whose
 * initial state is U0: on entry Ubar is the adjoint of the step's final
 * state, on exit that of U0; grad [nelems] accumulates the step's part of
 * dJ/dkappa.  The five stage inputs are recomputed from U0 (sources
 * included).  kappa enters through the pressure rows' factor and, for
 * alpha > 0, through the penalty coefficients tau_p = alpha/{rho c},
 * tau_u = alpha {rho c} of every face (Section 4.3).  Uses ten state-sized
 * scratch arrays and one trace-sized array held by the context: reserved at
 * setup with DGPYR_FLAG_ADJOINT, otherwise allocated by the first call.
 * Device arrays; asynchronous. */
dgpyr_status dgpyr_adjoint_step(dgpyr_ctx* ctx, const double* U0, double* Ubar, double* grad,
                                double t0, double dt, void* stream);

/* Work shape of the fused matrix-core stage kernel (FP64 and FP32 forms):
 * groups_per_wave = number of 4-element groups one wave owns, so that each
 * operator fragment loaded feeds that many matrix-core products (the trace
 * kernel's shape is chosen by the library).  1 or 2; 0 restores the
 * library's choice for the context's N.
 * Results are identical up to the same rounding for every choice.  Takes
 * effect at the next launch; not synchronised with work already queued.
 * Errors: E_ARG for other values. */
dgpyr_status dgpyr_set_groups(dgpyr_ctx* ctx, int32_t groups_per_wave);

/* ---- Batches of independent problems (uneven sizes and orders) ----------
 * Problems are grouped by (N, bc); a group's meshes are concatenated into one
 * context whose elements carry their problem's time step.  The state of the
 * batch is one device array: problem i occupies [offset, offset + len) in the
 * canonical layout [nelems][4][Np] of its order.  Every call returns a status
 * and never aborts. */
typedef struct dgpyr_batch dgpyr_batch;

typedef struct {
  int32_t group;          /* group index (problems sharing N and bc)             */
  int32_t N;              /* order                                               */
  int32_t Np;             /* basis functions per element                         */
  int32_t reserved;       /* 0                                                   */
  int64_t nelems;         /* elements of the problem                             */
  int64_t elem_offset;    /* first element inside its group                      */
  int64_t offset;         /* first double of the problem in the batch state      */
  int64_t len;            /* doubles of the problem (nelems * 4 * Np)            */
  double dt;              /* the problem's time step                             */
  double inv_length_max;  /* max over its elements of c_K |dK| / |K|             */
} dgpyr_batch_slot;

/* nproblems meshes (host arrays, each with its own bc, materials and point
 * sources), orders[i] in [0, DGPYR_MAX_ORDER], one dgpyr_opts for all.  Time
 * step of problem i: dts[i] if dts is non-NULL, else the CFL rule of Section
 * 4.3, cfl / (2(N+1)(N+3)/3 * max_K c_K |dK|/|K|) over its own elements.
 * Synchronous.  Errors as dgpyr_setup, for the first failing group. */
dgpyr_status dgpyr_batch_setup(const dgpyr_mesh* meshes, const int32_t* orders,
                               const double* dts, double cfl, int32_t nproblems,
                               const dgpyr_opts* opts, dgpyr_batch** out);

/* Total doubles of the batch state and the number of groups. */
dgpyr_status dgpyr_batch_info(const dgpyr_batch* b, int64_t* state_len, int32_t* ngroups);

/* Layout and time step of problem i. */
dgpyr_status dgpyr_batch_problem(const dgpyr_batch* b, int32_t i, dgpyr_batch_slot* slot);

/* The context of group g (for dgpyr_volume_points / project / eval on that
 * group's part of the state, which starts at *state_offset).  Owned by the
 * batch; do not destroy. */
dgpyr_status dgpyr_batch_group(dgpyr_batch* b, int32_t g, dgpyr_ctx** ctx, int64_t* state_offset);

/* nsteps LSRK(5,4) steps of every problem, each with its own time step;
 * step0 is the number of steps already taken (source times are
 * (step0 + n + c_s) dt_i).  One step of all groups is captured once into a
 * HIP graph, the groups on streams of their own between a fork and a join so
 * that independent groups run concurrently (re-captured when U or R change),
 * and replayed nsteps times on the stream.  U, R: device arrays of the batch
 * state length.  Asynchronous. */
dgpyr_status dgpyr_batch_step(dgpyr_batch* b, double* U, double* R, int64_t step0, int32_t nsteps,
                              void* stream);

/* Autotuner: for every group on an FP64 or FP32 matrix-core path, times
 * nsteps steps of each candidate and keeps the fastest: the fused stage with
 * 1 or 2 element groups per wave times the trace kernel with 1, 2 or 4
 * (chosen[g] = 10 trace_groups + groups_per_wave), and for FP64 the
 * sum-factorised kernels (chosen[g] = 100) when their resources fit the
 * device; chosen[g] = 0 for groups with nothing to tune (chosen may be NULL).
 * The timing runs on the caller's scratch arrays U and R (device, batch state
 * length each; their contents are overwritten), so the call allocates no
 * device memory.  Synchronises the stream. */
dgpyr_status dgpyr_batch_tune(dgpyr_batch* b, double* U, double* R, int32_t nsteps, void* stream,
                              int32_t* chosen);

/* Releases the batch, its contexts and graph. */
void dgpyr_batch_destroy(dgpyr_batch* b);

/* Host-only inspection of the reference data the library builds for degree N
 * (no device needed).  which: 0 volume weights [Nc]; 1 V [Nc][Np];
 * 2 d/dr [Nc][Np]; 3 d/ds; 4 d/dt; 5 face basis values [Nfc][Np]; 6 face
 * parameter weights [Nfc]; 7 reference mass diagonal [Np]; 8 volume points
 * (a, b, c) [Nc][3]; 9 face points (a, b, c) [Nfc][3]; the one-dimensional
 * factors of phi_ijk = l^k_i(a) l^k_j(b) g_k(c), n1 = N+1, h = (1-c)/2:
 * 10 l^k_i(a_p) [k][p][i]; 11 d/da l^k_i(a_p); 12 l^k_i(-1), l^k_i(+1)
 * [k][2][i]; 13 g_k(c_r) [r][k]; 14 h^(k-1) P_{N-k}(c_r) [r][k];
 * 15 g_k'(c_r) [r][k]; 16 g_k(-1) [k]; 17 g_k at the Gauss-Jacobi(1,0) face
 * nodes [m][k].  Writes min(len,
 * needed) doubles to out (out may be NULL to query) and the full size to
 * *needed.  Errors: E_ORDER, E_ARG. */
dgpyr_status dgpyr_host_reference(int32_t N, int32_t which, double* out, int64_t len,
                                  int64_t* needed);

/* Work shape of the matrix-core trace kernel: 4-element groups per wave
 * (1, 2 or 4; 0 = the library's choice for N).  Same results for every
 * choice.  Takes effect at the next launch. */
dgpyr_status dgpyr_set_trace_groups(dgpyr_ctx* ctx, int32_t groups);

/* Operator staging of the fused matrix-core stage kernel: with enable != 0
 * each workgroup copies the derivative, projection and lift fragments of a
 * tile into LDS once and its four waves share them (one 4-element group per
 * wave); used where the tile fits in 64 KiB of LDS (FP64 N <= 5, FP32
 * N <= 6), elsewhere the default kernel runs.  Same results to rounding.
 * Default: on for the FP32 form, off for FP64 (measured).  Takes effect at
 * the next launch. */
dgpyr_status dgpyr_set_operator_staging(dgpyr_ctx* ctx, int32_t enable);

/* Host-only location of the mesh's point sources (what dgpyr_setup does
 * before touching the device): elem[s] (optional, [nsources]) receives the
 * containing element and abc (optional, [nsources][3]) the collapsed
 * coordinates (a, b, c) of the point there.  Errors as dgpyr_setup's host
 * part; E_ARG without sources or when a point lies in no element. */
dgpyr_status dgpyr_host_sources(const dgpyr_mesh* mesh, int32_t N, int64_t* elem, double* abc);

/* Host-only run of the mesh builders (geometry checks and face matching) that
 * dgpyr_setup performs before touching the device.  nbr (optional, [nelems][5])
 * receives the neighbour element of each face or -1; inv_length_max and
 * hex_groups (optional) as in dgpyr_info.  Same errors as dgpyr_setup's host
 * part. */
dgpyr_status dgpyr_host_mesh(const dgpyr_mesh* mesh, int32_t N, int32_t* nbr,
                             double* inv_length_max, int32_t* hex_groups);

/* Physical coordinates of the (N+1)^3 volume cubature points of every element
 * (device [K][Nc][3], point order q = p + (N+1)(m + (N+1) r) for Gauss-Legendre
 * a_p, b_m and Gauss-Jacobi(2,0) c_r, Section 4.1) and, if wJ is not NULL,
 * the quadrature weights w_q J(a_q, b_q) (device [K][Nc]).  Asynchronous. */
dgpyr_status dgpyr_volume_points(dgpyr_ctx* ctx, double* xyz, double* wJ, void* stream);

/* L2 projection onto the semi-nodal basis by the minimal volume rule:
 * U_i = sum_q w_q J_q phi_i(q) f_q / M_ii for each field, with M diagonal
 * (Lemma 3).  f: device [K][4][Nc] values at the points of
 * dgpyr_volume_points; U: device state array.  Asynchronous. */
dgpyr_status dgpyr_project(dgpyr_ctx* ctx, const double* f, double* U, void* stream);

/* Values of state U at the volume cubature points: f (device [K][4][Nc]).
 * With the weights of dgpyr_volume_points this gives L2 norms and errors.
 * Asynchronous. */
dgpyr_status dgpyr_eval(dgpyr_ctx* ctx, const double* U, double* f, void* stream);

/* Release every device buffer of the context (synchronises the device first).
 * NULL is accepted. */
void dgpyr_destroy(dgpyr_ctx* ctx);

const char* dgpyr_status_string(dgpyr_status s);
const char* dgpyr_last_error(void);

/* ------------------------------------------------------------------------
 * Linear advection u_t + div(beta u) = 0 with a constant vector beta
 * (Section 4.1): one field per element, the same basis, cubatures, operators
 * and matrix-core work shapes as the acoustic path (Algorithms 1-3 are stated
 * for this equation).  With outward normal n, beta_n = beta . n and the jump
 * [[u]] = u+ - u- (the sign for which the scheme is energy stable),
 *   du/dt = -M^-1 (S u + L^f F),  S_ij = int_K phi_i beta . grad phi_j,
 *   F = (beta_n - alpha |beta_n|) / 2 [[u]]  (times the face weight and sJ),
 * alpha = 1 the upwind flux, alpha = 0 the central flux.  A face without a
 * partner sees u+ = 0.
 * ------------------------------------------------------------------------ */

/* Mesh, read on the host during dgpyr_advection_setup only.  xyz and e2v as in
 * dgpyr_mesh.  pair_ids (optional, [nverts]) are the vertex identities used to
 * pair faces: two faces are neighbours when their vertex sets have equal ids,
 * so a periodic mesh gives the vertices of opposite boundary faces equal ids
 * (the face-point correspondence follows the ids); NULL pairs faces by the
 * vertex indices of e2v alone. */
typedef struct {
  int64_t nverts;
  const double* xyz;        /* [nverts][3]                                        */
  int64_t nelems;
  const int64_t* e2v;       /* [nelems][5]                                        */
  const int64_t* pair_ids;  /* [nverts] or NULL                                   */
} dgpyr_advection_mesh;

typedef struct {
  double beta[3];    /* advection velocity                                       */
  double alpha;      /* 1 = upwind, 0 = central, values in [0, 1] blend          */
  int32_t precision; /* DGPYR_FP64 (the only form built for advection)           */
  uint32_t flags;    /* 0                                                        */
} dgpyr_advection_opts;

/* Builds an advection context: host reference data and geometry as
 * dgpyr_setup, faces paired through pair_ids.  The state is [K][1][Np]
 * (dgpyr_info.nfields = 1, state_len = K Np); inv_length_max is
 * |beta| max_K |dK| / |K|.  The context then serves dgpyr_get_info, rhs, step,
 * step_timed, pack/unpack, volume_points, project, eval, kernel_names and
 * destroy; the acoustic-only calls (adjoint, receivers, kappa, work shapes)
 * return E_UNSUPPORTED on it.  Synchronous.  Errors: E_ARG (null pointers,
 * bad pair_ids, alpha outside [0, 1], flags), E_UNSUPPORTED (precision other
 * than FP64), E_ORDER, E_MESH, E_NONCONFORMING, E_OOM, E_HIP. */
dgpyr_status dgpyr_advection_setup(const dgpyr_advection_mesh* mesh, int32_t N,
                                   const dgpyr_advection_opts* opts, void* stream,
                                   dgpyr_ctx** out);

/* Host-only run of what dgpyr_advection_setup does before touching the device
 * (geometry checks and face pairing through pair_ids): nbr (optional,
 * [nelems][5]) receives the neighbour element of each face or -1 and nface
 * (optional, [nelems][5]) the neighbour's face (faces ordered c = -1, a = -1,
 * a = +1, b = -1, b = +1) or -1.  Errors as the setup's host part; a periodic
 * direction with fewer than three element layers gives faces with equal
 * vertex-identity sets and E_NONCONFORMING. */
dgpyr_status dgpyr_host_advection_mesh(const dgpyr_advection_mesh* mesh, int32_t N, int32_t* nbr,
                                       int32_t* nface);

#ifdef __cplusplus
}
#endif

#endif /* DGPYR_H */
