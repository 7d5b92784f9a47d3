/* mss.h -- C ABI of the MI355X (gfx950) spin-1/2 / spin-1 Schroedinger solver.
 *
 * Method: arXiv:2204.05586 ("Spinsim").  The library integrates
 *   i d psi / dt = H(t) psi,   H(t) = 2 pi (f_x J_x + f_y J_y + f_z J_z [+ f_q Q])
 * (Sec. "Quantum mechanics background"; hbar = 1, fields f_j in Hz,
 * J = sigma/2 for spin-1/2, the spin-1 matrices and Q = diag(1,-2,1)/3 for
 * spin-1, basis ordered m = +s ... -s).  For every output interval
 * [t_k, t_k + Dt] it builds the time-evolution operator U_k from L fine
 * commutator-free fourth-order Magnus (CF4) steps (Sec. "Unitary time
 * evolution and the Magnus expansion", eqs. cf4_sample_1/2 and
 * cf4_implementation) inside a per-interval rotating frame (Sec.
 * "Dynamically rotating frame", eq. exit_rotating_frame), with an analytic
 * SU(2) exponential for spin-1/2 and the Lie-Trotter exponentiator with
 * 2^tau residual squarings for spin-1 (Sec. "Lie-Trotter based
 * exponentiator", eq. lie_trotter_4).  The state series is the ordered
 * product psi_0 = psi_init, psi_{k+1} = U_k psi_k (Sec. "Discretization and
 * parallelization", eq. integration_compilation), computed on the GPU as
 * an associative prefix product.
 *
 * Conventions
 *   complex   interleaved double (re, im); matrices row-major; N = 2 or 3
 *   U         [K][N][N] complex  (K*N*N*2 doubles)
 *   psi       [K][N] complex     psi[k] = psi(t_k), psi[0] = psi_init
 *   psi_final [N] complex        psi(t_start + K Dt)
 *   time      [K] double         t_k = t_start + k * Dt
 *   units     seconds and Hz
 *
 * Ownership: the caller owns every buffer.  Array arguments of the solve
 * calls are DEVICE pointers (HIP device memory of the current device);
 * mss_problem and its term array are HOST memory and are only read during
 * the call.  `stream` is a hipStream_t (NULL: the default stream); work is
 * enqueued asynchronously.  The single-simulation calls keep no pointer
 * after return; batch plans, adjoint plans and servers keep the device
 * pointers of their last run or of admitted requests, as documented with
 * each.
 *
 * Errors: every call returns an mss_status.  Arguments are validated on
 * the host before anything is launched; on failure nothing is launched and
 * mss_last_error() (thread-local) describes the problem.  A HIP runtime
 * failure returns MSS_E_DEVICE with the HIP error string.
 */
#ifndef MSS_H
#define MSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSS_MAX_TERMS 32
#define MSS_MAX_SQUARES 60

typedef enum mss_status {
  MSS_OK = 0,
  MSS_E_INVALID = 1,     /* bad argument (see mss_last_error) */
  MSS_E_NOMEM = 2,       /* workspace too small or device memory exhausted */
  MSS_E_DEVICE = 3,      /* HIP runtime failure / no usable device */
  MSS_E_UNSUPPORTED = 4, /* valid request this build cannot run */
  MSS_E_BUSY = 5,
  MSS_E_NOTREADY = 6
} mss_status;

/* Field-program term kinds.  A term adds to component `comp` at time t,
 * only while t_on < t < t_off (use -inf / +inf for "always"):
 *   MSS_TERM_CONST    a
 *   MSS_TERM_COS      a * cos(2 pi f t + phi)
 *   MSS_TERM_SIN      a * sin(2 pi f t + phi)
 *   MSS_TERM_PWC      a_s
 *   MSS_TERM_PWC_COS  a_s * cos(2 pi f t + phi_s)
 *   MSS_TERM_PWC_SIN  a_s * sin(2 pi f t + phi_s)
 * with s = clamp(floor((t - seg_t0) / seg_len), 0, n_seg - 1),
 * a_s = params[seg_a_slot + s] (literal a if seg_a_slot < 0) and
 * phi_s = params[seg_phi_slot + s] (literal phi if seg_phi_slot < 0).
 * a, f, phi are replaced by params[a_slot], params[f_slot], params[phi_slot]
 * when the slot is >= 0 -- the per-simulation parameter vector plays the
 * role of the paper's sweep_parameters (Sec. "Compilation of integrator").
 * The phase is evaluated as 2 pi * (f * t) + phi; terms of one component
 * are summed in list order. */
typedef enum mss_term_kind {
  MSS_TERM_CONST = 0,
  MSS_TERM_COS = 1,
  MSS_TERM_SIN = 2,
  MSS_TERM_PWC = 3,
  MSS_TERM_PWC_COS = 4,
  MSS_TERM_PWC_SIN = 5
} mss_term_kind;

/* Field components: the spin operators J_x, J_y, J_z and the quadrupole Q
 * (spin-1), and for spin-1 in the full su(3) basis (Sec. "Spin-one": the
 * paper adds w_u1 U_1 + w_u2 U_2 + w_v1 V_1 + w_v2 V_2 with operators from
 * a reference it does not print) the Cartesian quadrupoles
 * U_1 = J_x^2 - J_y^2, U_2 = J_x J_y + J_y J_x (Delta m = 2) and
 * V_1 = J_z J_x + J_x J_z, V_2 = J_y J_z + J_z J_y (Delta m = 1).  A spin-1
 * problem with a term on U_1, U_2, V_1 or V_2 runs the full-basis
 * exponentiator: exp(-i G) by scaling and squaring, the residual of
 * exp(-i G / 2^tau) from its degree-4 Taylor polynomial, then the tau
 * residual squarings (n_squares); in the rotating frame (u1 + i u2) turns
 * with e^{-2i w_r t} and (v1 + i v2) with e^{-i w_r t}.  Such problems
 * have no adjoint and no specialised sampler (MSS_E_UNSUPPORTED). */
typedef enum mss_component {
  MSS_X = 0, MSS_Y = 1, MSS_Z = 2, MSS_Q = 3,
  MSS_U1 = 4, MSS_U2 = 5, MSS_V1 = 6, MSS_V2 = 7
} mss_component;

typedef struct mss_term {
  int32_t kind;          /* mss_term_kind */
  int32_t comp;          /* mss_component; MSS_Q only for spin-1 */
  int32_t a_slot, f_slot, phi_slot;     /* -1: literal */
  int32_t n_seg;         /* PWC kinds: number of segments (>= 1) */
  int32_t seg_a_slot, seg_phi_slot;     /* first slot of the per-segment arrays, -1: literal */
  double a, f, phi;      /* Hz, Hz, rad */
  double t_on, t_off;    /* s */
  double seg_t0, seg_len;/* s; seg_len > 0 for PWC kinds */
} mss_term;

typedef struct mss_problem {
  int32_t spin_twice;     /* 1: spin-1/2 (N = 2), 2: spin-1 (N = 3) */
  int32_t n_terms;        /* 0 .. MSS_MAX_TERMS */
  const mss_term* terms;  /* host array of n_terms terms */
  int32_t n_params;       /* length of the parameter vector (>= every slot used + 1) */
  int32_t n_fine;         /* L >= 1 fine CF4 steps per interval, dt = Dt / L */
  int64_t n_samples;      /* K >= 1 output intervals */
  double t_start;         /* s, finite */
  double dt_out;          /* Dt > 0, s */
  int32_t n_squares;      /* tau in [0, MSS_MAX_SQUARES], spin-1 only (paper default 24) */
  int32_t rotating_frame; /* 0/1: per-interval frame at omega_r = 2 pi f_z(t_k + Dt/2) */
  int32_t method;         /* mss_method (0: CF4) */
} mss_problem;

/* Integration method per fine step (Sec. "Evaluation of accuracy" compares
 * the first with the other two):
 *   MSS_CF4       exp(-i Hbar_2 dt) exp(-i Hbar_1 dt), Gauss nodes (default)
 *   MSS_MIDPOINT  exp(-i H(t + dt/2) dt)                ("modified Euler")
 *   MSS_HEUN      exp(-i (H(t) + H(t + dt))/2 dt)        ("improved Euler")
 * The adjoint supports MSS_CF4 only. */
typedef enum mss_method { MSS_CF4 = 0, MSS_MIDPOINT = 1, MSS_HEUN = 2 } mss_method;

/* Launch shape of the integrator.  slices: lanes cooperating on one
 * interval (power of two, 1..64, <= n_fine); each lane takes a contiguous
 * run of fine steps and the partial products are combined in order.
 * block: threads per workgroup (64, 128 or 256).
 * Zero fields mean "choose" (mss_plan_launch). */
typedef struct mss_launch {
  int32_t slices;
  int32_t block;
} mss_launch;

/* Human-readable name of a status code (static string). */
const char* mss_status_str(mss_status s);

/* Last error message of the calling thread ("" if none). */
const char* mss_last_error(void);

/* Library version string, e.g. "mss 0.1 gfx950". */
const char* mss_version(void);

/* Host-only validation of a problem (Sec. "Discretization and
 * parallelization": K, L, Dt; field program limits).  No device access. */
mss_status mss_validate(const mss_problem* p);

/* Launch shape the library would use for `p` on the current device (or a
 * 256-CU gfx950 when no device is visible).  Host only. */
mss_status mss_plan_launch(const mss_problem* p, mss_launch* out);

/* Bytes of device workspace mss_solve needs for `p`; store_u = 0 means
 * the caller passes U = NULL, so the operators live in the workspace.
 * Host only. */
mss_status mss_workspace_size(const mss_problem* p, int32_t store_u, size_t* bytes);

/* Bytes of device workspace mss_propagate needs for K operators of size N. */
mss_status mss_propagate_workspace_size(int32_t spin_twice, int64_t n_samples, size_t* bytes);

/* Interval operators U_k, k = 0..K-1 (the integrator: CF4 fine steps in the
 * rotating frame, then the frame exit).  params: device array of
 * p->n_params doubles (may be NULL when n_params == 0).  U: device output
 * [K][N][N] complex.  time: optional device output [K] (NULL: skipped).
 * launch: NULL for the planned shape. */
mss_status mss_integrate(const mss_problem* p, const double* params, double* U, double* time,
                         const mss_launch* launch, void* stream);

/* Ordered product of operators (eq. integration_compilation):
 * psi[0] = psi0, psi[k+1] = U[k] psi[k], psi_final = U[K-1] psi[K-1].
 * U: device [K][N][N]; psi0: device [N]; psi: device [K][N] (required);
 * psi_final: device [N] or NULL.  ws: device workspace of at least
 * mss_propagate_workspace_size bytes (may be NULL if that size is 0). */
mss_status mss_propagate(int32_t spin_twice, int64_t n_samples, const double* U,
                         const double* psi0, double* psi, double* psi_final, void* ws,
                         size_t ws_bytes, void* stream);

/* mss_propagate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument and no allocation of any kind.  The
 * scan's workspace is a static device array of 8 MiB that each GPU the
 * library runs on holds until the process ends; its address is looked up
 * on the first call on a device.  Every call on one GPU shares that array,
 * so calls that overlap on one GPU (other streams, other threads) race;
 * calls in order on one stream are fine.  Arguments, outputs and errors as
 * mss_propagate (same kernels, same results bit for bit), plus
 * MSS_E_INVALID, before any launch, when n_samples exceeds what the array
 * holds: MSS_NOALLOC_MAX_SAMPLES_SPIN_ONE spin-1 or
 * MSS_NOALLOC_MAX_SAMPLES_SPIN_HALF spin-1/2 intervals. */
#define MSS_NOALLOC_MAX_SAMPLES_SPIN_ONE 11141120LL
#define MSS_NOALLOC_MAX_SAMPLES_SPIN_HALF 22280192LL
mss_status mss_propagate_noalloc(int32_t spin_twice, int64_t n_samples, const double* U,
                                 const double* psi0, double* psi, double* psi_final,
                                 void* stream);

/* mss_propagate that also writes the expected spin projection of every
 * state as the states are formed (the projection of mss_spin_projection,
 * fused into the last pass of the product, so the states are not read
 * back): spin: device [n_samples][3] doubles, required.  Same errors as
 * mss_propagate, and MSS_E_INVALID for a NULL spin. */
mss_status mss_propagate_spin(int32_t spin_twice, int64_t n_samples, const double* U,
                              const double* psi0, double* psi, double* psi_final, double* spin,
                              void* ws, size_t ws_bytes, void* stream);

/* Expected spin projection <J_x>, <J_y>, <J_z> of each state (Sec.
 * "Quantum mechanics background": the measurable ensemble average of the
 * spin): out[3k + a] = psi_k^H J_a psi_k.  psi: device [n_samples][N]
 * complex; out: device [n_samples][3] doubles. */
mss_status mss_spin_projection(int32_t spin_twice, int64_t n_samples, const double* psi,
                               double* out, void* stream);

/* Whole path: mss_integrate then mss_propagate.  U may be NULL (the
 * operators then live in the workspace, see mss_workspace_size). */
mss_status mss_solve(const mss_problem* p, const double* params, const double* psi0, double* U,
                     double* psi, double* psi_final, double* time, void* ws, size_t ws_bytes,
                     void* stream);

/* ---- user field samplers ------------------------------------------------
 * A field function written by the user in HIP C++, compiled at run time
 * (hiprtc) into its own integrator: the counterpart of the paper's user
 * field function compiled into the integrator (Sec. "Compilation of
 * integrator"), for fields the term kinds cannot express.  The source
 * defines
 *
 *   __device__ void mss_user_field(double t, const double* params, double* field);
 *
 * which receives field[0..3] zeroed and sets f_x, f_y, f_z, f_q in Hz at
 * time t (s); f_q is ignored for spin-1/2.  params is the device parameter
 * vector passed to mss_sampler_integrate (NULL when n_params == 0).  The
 * source is compiled after the library's device header, so namespace mss
 * (e.g. mss::sincos_cw, accurate for phases up to 1.5e6 rad) and the device
 * math library are available; flags: gfx950, -O3, C++17, fused multiply-add
 * contraction as hipcc's default (put `#pragma clang fp contract(off)` in
 * the function to fix its evaluation order).  The code must be safe to run
 * by every lane: it must read params within n_params and write only
 * field[0..3]. */
typedef struct mss_sampler_s* mss_sampler;

/* Compile `source` (NUL-terminated) with n_options extra compiler options
 * (options may be NULL when n_options == 0, e.g. "-DAMP=2.0").  Host only:
 * no GPU is needed.  On success *out owns the compiled code object.  A
 * compile error returns MSS_E_INVALID with the compiler log in
 * mss_last_error() and *out = NULL. */
mss_status mss_sampler_create(const char* source, const char* const* options, int32_t n_options,
                              mss_sampler* out);

/* Specialised field program: a sampler whose mss_user_field is generated
 * from a term list (the format of mss_problem.terms) and compiled as by
 * mss_sampler_create.  The generated function performs the field-program
 * interpreter's operations for these terms in the same order, so the
 * operators it gives are bit for bit those of the interpreter on the same
 * terms; the field is compiled into the integrator instead of interpreted
 * per node (the counterpart of the paper's field function compiled into its
 * integrator, Sec. "Compilation of integrator").  Problems run with it carry
 * no terms (n_terms = 0) and at least mss_sampler_min_params(s) parameters:
 * the terms' slots index that vector.  A term on the quadrupole component
 * makes the sampler spin-1 only.  terms (host, n_terms in [0, MSS_MAX_TERMS])
 * are read during the call only; the checks are those of a problem's terms.
 * Errors as mss_sampler_create, plus MSS_E_INVALID for invalid terms. */
mss_status mss_sampler_create_for_terms(const mss_term* terms, int32_t n_terms,
                                        mss_sampler* out);

/* Parameters a problem run with the sampler must carry: one past the
 * highest slot its terms read (mss_sampler_create_for_terms), 0 for a
 * sampler compiled from source (whose reads the caller keeps within
 * n_params).  Problems with fewer are rejected with MSS_E_INVALID by
 * mss_sampler_integrate, mss_sampler_solve and
 * mss_batch_plan_create_sampled. */
int32_t mss_sampler_min_params(mss_sampler s);

/* Compiler log of a successful compile (warnings; "" if none).  Owned by
 * the sampler, valid until mss_sampler_destroy. */
const char* mss_sampler_log(mss_sampler s);

/* Interval operators U_k of `p` with the field from the sampler, as
 * mss_integrate (same outputs, launch shapes and errors).  p->n_terms must
 * be 0.  The code object is loaded on the current device at its first use
 * there (MSS_E_DEVICE if loading fails).  Thread-safe. */
mss_status mss_sampler_integrate(mss_sampler s, const mss_problem* p, const double* params,
                                 double* U, double* time, const mss_launch* launch, void* stream);

/* Whole path with a sampler: mss_sampler_integrate then mss_propagate, with
 * the workspace of mss_solve (mss_workspace_size). */
mss_status mss_sampler_solve(mss_sampler s, const mss_problem* p, const double* params,
                             const double* psi0, double* U, double* psi, double* psi_final,
                             double* time, void* ws, size_t ws_bytes, void* stream);

/* Synchronise every device the sampler was loaded on, unload it there and
 * free it.  NULL is a no-op. */
void mss_sampler_destroy(mss_sampler s);

/* ---- batches ------------------------------------------------------------
 * Many independent simulations (uneven K, mixed spin allowed) in one
 * persistent integrator launch and one segmented scan.  Sweeps over
 * parameters (the paper's use of one compiled simulator for many
 * evaluate() calls, Sec. "Compilation of integrator") become one batch.
 *
 * Packed layout (complex units), simulation i in order:
 *   psi0 / psi_final  N_i entries at psi0_off[i]
 *   psi               K_i N_i entries at state_off[i]
 *   U                 K_i N_i^2 entries at op_off[i]
 * mss_batch_layout returns these offsets (n + 1 entries, the last = total).
 * params: one device array; simulation i reads its n_params values from
 * index param_off[i].
 *
 * A plan owns device descriptors (uploaded synchronously at creation) and,
 * with use_graph, one instantiated HIP graph of the whole batch; it is not
 * thread-safe.  Work enqueued by mss_batch_run reads the plan's
 * descriptors: destroy the plan only after that work has completed. */
typedef struct mss_batch_plan mss_batch_plan;

typedef struct mss_batch_options {
  int32_t slices_spin_half; /* lanes per spin-1/2 interval, power of two <= 64, 0: choose */
  int32_t slices_spin_one;  /* lanes per spin-1 interval, 0: choose */
  int32_t waves_per_simd;   /* persistent grid: resident waves per SIMD (0: 2; chained
                               plans take at most the two a CU holds) */
  int32_t use_graph;        /* 1: capture the batch as one HIP graph, replayed while the
                               buffer pointers stay the same */
  int32_t scan_per_lane;    /* operators per lane in the scan tiles: 2, 4 or 8 (0: 4) */
  int32_t chained;          /* 1: mss_batch_run forms the states inside the integrator's
                               launch: each unit (3 x 64 / S consecutive intervals, one wave)
                               multiplies its operators together in registers and passes its
                               leaving state to the next unit of its simulation, units being
                               taken round by round across the simulations; no operator
                               buffer and no scan (U, when given, is
                               still written).  The workspace is then a 256-byte head plus 128
                               bytes per simulation, mss_batch_propagate is not available and
                               mss_batch_integrate needs U.  0: separate scan. */
  int32_t chain_wait_us;    /* chained plans: bound of one unit's wait for the state the unit
                               before leaves, in microseconds (0: 10 s, far beyond any real
                               wait).  A wait that runs out marks the run failed: every later
                               wait gives up at once, the launch drains its queue and ends, and
                               mss_batch_check reports MSS_E_DEVICE (the states are then
                               undefined).  Must be >= 0. */
} mss_batch_options;

typedef struct mss_batch_info_t {
  int32_t n_sims;
  int32_t scan_levels;
  int32_t grid_blocks;      /* 256-thread workgroups of the persistent integrator */
  int32_t pad;
  int64_t n_items;          /* work items (one wave's worth of intervals each; in a chained
                               plan the units, 3 x 64 / S intervals each) */
  int64_t total_samples;    /* sum of K_i */
} mss_batch_info_t;

/* Validate every problem (as mss_validate) and build a plan.  problems and
 * param_off are host arrays of n entries; param_off may be NULL when no
 * simulation has parameters.  options may be NULL (all defaults). */
mss_status mss_batch_plan_create(int32_t n, const mss_problem* problems, const int64_t* param_off,
                                 const mss_batch_options* options, mss_batch_plan** out);

/* As mss_batch_plan_create, with every simulation's field from one user
 * sampler (a parameter sweep of one compiled field function in a single
 * persistent launch).  Every problem must have n_terms = 0.  The sampler
 * must outlive the plan; it is loaded on the device current at each run. */
mss_status mss_batch_plan_create_sampled(int32_t n, const mss_problem* problems,
                                         const int64_t* param_off,
                                         const mss_batch_options* options, mss_sampler sampler,
                                         mss_batch_plan** out);

/* Packed offsets (host arrays of n + 1 entries each; any may be NULL). */
mss_status mss_batch_layout(const mss_batch_plan* plan, int64_t* psi0_off, int64_t* state_off,
                            int64_t* op_off);

/* Device workspace bytes for mss_batch_run; store_u = 0 when U is NULL. */
mss_status mss_batch_workspace_size(const mss_batch_plan* plan, int32_t store_u, size_t* bytes);

/* Shape of the planned launch. */
mss_status mss_batch_info(const mss_batch_plan* plan, mss_batch_info_t* info);

/* Run the batch: operators (into U, or the workspace when U is NULL), then
 * states psi and (optional) psi_final, all device arrays in the packed
 * layout.  Asynchronous on `stream`. */
mss_status mss_batch_run(mss_batch_plan* plan, const double* params, const double* psi0,
                         double* psi, double* psi_final, double* U, void* ws, size_t ws_bytes,
                         void* stream);

/* The two halves of mss_batch_run, always launched eagerly (no graph):
 * the persistent integrator (operators into U, or the workspace when U is
 * NULL) and the segmented scan that reads them.  Pass the same U / ws to
 * both. */
mss_status mss_batch_integrate(mss_batch_plan* plan, const double* params, double* U, void* ws,
                               size_t ws_bytes, void* stream);
mss_status mss_batch_propagate(mss_batch_plan* plan, const double* psi0, double* psi,
                               double* psi_final, const double* U, void* ws, size_t ws_bytes,
                               void* stream);

/* Completion check of a chained plan's run: waits for `stream`, then reads
 * the failure word the run keeps in the first bytes of `ws` (the workspace
 * the run was given).  MSS_E_DEVICE when a wait ran out (see
 * chain_wait_us) or a wave found lanes missing at its dequeue: the states
 * of that run are undefined.  MSS_OK otherwise, and always for a
 * separate-scan plan (which keeps no failure word). */
mss_status mss_batch_check(const mss_batch_plan* plan, const void* ws, void* stream);

/* Free the plan (its graph, stream and descriptors). */
void mss_batch_plan_destroy(mss_batch_plan* plan);

/* A whole batch in one call, the paper's evaluate() over many simulations
 * (Sec. "Compilation of integrator"): plans a chained batch with default
 * options, runs it on `stream`, waits for it and frees what it allocated
 * (descriptors and a workspace of 256 + 128 n bytes).  problems / param_off
 * as mss_batch_plan_create; params, psi0, psi, psi_final (optional) and U
 * (optional) are device arrays in the packed layout of mss_batch_layout,
 * which follows from the problems alone: simulation i's psi0 / psi_final at
 * the sum of N_j over j < i, its states at the sum of K_j N_j, its
 * operators at the sum of K_j N_j^2 (complex units).  Synchronous: returns
 * once the outputs are written.  Errors as the plan calls, plus
 * MSS_E_NOMEM when the workspace cannot be allocated and MSS_E_DEVICE when
 * the run failed (mss_batch_check). */
mss_status mss_solve_batch(int32_t n, const mss_problem* problems, const int64_t* param_off,
                           const double* params, const double* psi0, double* psi,
                           double* psi_final, double* U, void* stream);

/* ---- serving ------------------------------------------------------------
 * Continuous batching of simulation requests (mixed spin and length) on the
 * current device.  Requests are admitted in arrival order while their
 * device block (K (N^2 + N) 16 bytes plus a small final-state and scan
 * arrays) fits in the HBM budget and an active slot is free; otherwise they
 * wait (back-pressure).  A scheduler thread runs rounds: every active
 * request gets a share of the round's work, all shares are integrated in
 * one persistent launch, requests whose last share is in the round are
 * scanned in it, and requests arriving meanwhile join the next round.
 * Results stay in device memory until mss_server_release.  All calls are
 * thread-safe. */
typedef struct mss_server mss_server;

typedef struct mss_server_options {
  size_t hbm_budget;      /* bytes of device memory for requests (0: 80 % of free memory) */
  int32_t max_active;     /* requests admitted at once (0: 512) */
  int32_t slices;         /* lanes per interval, power of two <= 64, capped at each request's
                             n_fine; 0: per request, the least 2^s (s <= log2 n_fine) with
                             n_samples 2^s >= the device's resident lanes (CUs x 512) */
  double iteration_steps; /* spin-1 fine steps per round (spin-1/2 steps weigh 1/16; 0: 3e7) */
} mss_server_options;

enum { MSS_REQ_QUEUED = 0, MSS_REQ_RUNNING = 1, MSS_REQ_DONE = 2, MSS_REQ_FAILED = 3 };

typedef struct mss_request_info {
  int32_t state;          /* MSS_REQ_* */
  int32_t spin_twice;
  int64_t n_samples;
  const double* psi;      /* device [K][N] complex, valid when DONE until release */
  const double* psi_final;/* device [N] */
  const double* U;        /* device [K][N][N] */
  double t_submit, t_admit, t_done; /* seconds on the server clock */
} mss_request_info;

typedef struct mss_server_stats {
  int64_t submitted, completed, rounds;
  int32_t queued, active;
  double fine_steps;      /* fine steps integrated so far */
  size_t bytes_in_use, bytes_peak, budget;
} mss_server_stats;

/* Reserve the budget on the current device and start the scheduler. */
mss_status mss_server_create(const mss_server_options* options, mss_server** out);

/* Queue a request.  problem, its terms, params (n_params doubles) and psi0
 * (N complex) are HOST memory, copied before return.  MSS_E_NOMEM if the
 * request can never fit in the budget. */
mss_status mss_server_submit(mss_server* server, const mss_problem* problem, const double* params,
                             const double* psi0, uint64_t* ticket);

/* Current state of a request (never blocks). */
mss_status mss_server_poll(mss_server* server, uint64_t ticket, mss_request_info* out);

/* Block until the request is done (MSS_OK), failed (MSS_E_DEVICE) or the
 * timeout passes (MSS_E_NOTREADY). */
mss_status mss_server_wait(mss_server* server, uint64_t ticket, double timeout_s,
                           mss_request_info* out);

/* Device-to-device copy of a finished request's results into caller
 * buffers (any may be NULL), enqueued on `stream`. */
mss_status mss_server_copy_out(mss_server* server, uint64_t ticket, double* psi, double* psi_final,
                               double* U, void* stream);

/* Forget a request: a queued one is dropped, a finished one returns its
 * device block to the pool; a running one gives MSS_E_BUSY. */
mss_status mss_server_release(mss_server* server, uint64_t ticket);

mss_status mss_server_stats_get(mss_server* server, mss_server_stats* out);

/* Lanes per interval the server gives a problem (options.slices, or its
 * per-request choice): a served request's operators and states are bit for
 * bit those of mss_integrate with launch {slices, block} followed by
 * mss_propagate.  problem: host, validated as by mss_validate. */
mss_status mss_server_request_slices(const mss_server* server, const mss_problem* problem,
                                     int32_t* slices);

/* Seconds since the server was created (the clock of the request times). */
double mss_server_clock(const mss_server* server);

/* Stop the scheduler after in-flight rounds and free everything. */
void mss_server_destroy(mss_server* server);

/* ---- adjoint ------------------------------------------------------------
 * Gradients of final-state populations with respect to field parameters,
 * for a batch of simulations: loss_i = |psi_final_i[m]|^2 and
 * grad[param_off[i] + p] = d loss_i / d params[param_off[i] + p].  A
 * discrete adjoint of the whole path (derivatives of the computed CF4
 * steps, exponentiators included, through the frame and field terms).
 * Interval boundaries are the checkpoints: forward states and costates are
 * kept per interval and each interval's fine steps are replayed backward.
 * Parameters may be used by x and y terms (any kind, at most 4
 * parameterised terms per simulation); a z or q term with a parameter slot
 * gives MSS_E_UNSUPPORTED.  Gradients are summed with FP64 atomics, so
 * their last bits may vary between runs. */
typedef struct mss_adjoint_plan mss_adjoint_plan;

/* Validate and plan (host arrays of n problems / parameter offsets); the
 * packed layout of psi0 / psi_final is that of mss_batch_layout. */
mss_status mss_adjoint_plan_create(int32_t n, const mss_problem* problems, const int64_t* param_off,
                                   int32_t level_m, mss_adjoint_plan** out);
/* The same plan with the forward pass run by `forward`, a sampler that
 * mss_sampler_create_for_terms made from the term list every problem
 * carries (compared byte for byte; otherwise MSS_E_INVALID).  Its operators
 * are bit for bit the interpreter's, so losses and gradients are those of
 * mss_adjoint_plan_create; the backward pass still reads the terms.  The
 * sampler stays owned by the caller and must outlive the plan. */
mss_status mss_adjoint_plan_create_compiled(int32_t n, const mss_problem* problems,
                                            const int64_t* param_off, int32_t level_m,
                                            mss_sampler forward, mss_adjoint_plan** out);
mss_status mss_adjoint_workspace_size(const mss_adjoint_plan* plan, size_t* bytes);
/* Length of the gradient array: max over i of param_off[i] + n_params_i. */
mss_status mss_adjoint_param_count(const mss_adjoint_plan* plan, int64_t* count);
/* loss: device [n]; grad: device [param count] (overwritten); psi_final:
 * optional device copy of the final states.  Asynchronous on `stream`. */
mss_status mss_adjoint_run(mss_adjoint_plan* plan, const double* params, const double* psi0,
                           double* loss, double* grad, double* psi_final, void* ws,
                           size_t ws_bytes, void* stream);
void mss_adjoint_plan_destroy(mss_adjoint_plan* plan);

/* Losses and gradients in one call: plans as mss_adjoint_plan_create, runs
 * mss_adjoint_run on `stream` with a workspace it allocates, waits and
 * frees everything.  Buffers as mss_adjoint_run (grad has
 * mss_adjoint_param_count entries: the largest param_off[i] + n_params_i).
 * Synchronous.  Errors as the plan calls, plus MSS_E_NOMEM when the
 * workspace cannot be allocated. */
mss_status mss_adjoint_population(int32_t n, const mss_problem* problems,
                                  const int64_t* param_off, int32_t level_m,
                                  const double* params, const double* psi0, double* loss,
                                  double* grad, double* psi_final, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSS_H */
