/*
 * grmhd.h -- C-ABI of the MI355X (gfx950) coupled BSSN + Valencia GRMHD
 * spectral RK stage (arXiv 2508.18221).
 *
 * What the library computes (paper citations by section/equation):
 *  - grid: Chebyshev-Gauss-Lobatto nodes x_j = cos(j pi/(N-1)) in r (log map
 *    ln r = Lc + Lh x) and theta (affine map onto [th_min, th_max]), uniform
 *    phi_l = 2 pi l / N_phi (Methods, "Grid Discretization");
 *  - derivatives: derivative of the Chebyshev / trigonometric interpolant at
 *    the nodes, as dense differentiation matrices applied along grid lines
 *    (Methods, "The Spectral Derivative Operators"; Fourier Nyquist mode:
 *    dropped from odd, kept as -(N/2)^2 in even derivatives);
 *  - one RHS evaluation: per-point con2prim (Methods, "The Primitive Variable
 *    Recovery": the unique primitive state reproducing U), densitised fluxes
 *    alpha sqrt(gamma) F^i and 3+1 geometric sources (Results, "GRMHD
 *    Conservative Form"; Methods, "The Conserved Fluxes and Geometric Source
 *    Terms"), BSSN + 1+log + Gamma-driver right-hand side with matter
 *    coupling (Methods, "BSSN Evolution Equations", "Gauge Conditions",
 *    "Stress-Energy Tensor"); RHS frozen (= 0) at r_out and both theta ends;
 *  - one step: classic RK4 (Methods, "Time Integration") followed by the
 *    exponential filter sigma(k) = exp(-alpha (|k|/k_max)^p) along r, theta,
 *    phi (Methods, "Dealiasing and Spectral Filtering").
 *
 * State layout: 32 FP64 fields, field-major, each field laid out
 * [phi][theta][r] with r fastest (P = n_r n_theta n_phi doubles per field):
 *    0 phi (conformal factor, (1/12) ln det gamma)
 *    1-6  gt_rr gt_rth gt_rph gt_thth gt_thph gt_phph   (conformal metric)
 *    7-12 At_rr ... At_phph                             (trace-free curvature)
 *   13 K, 14-16 Gt^r Gt^th Gt^ph, 17 alpha, 18-20 beta^i, 21-23 Bd^i (driver)
 *   24 sqrt(gamma) D, 25-27 sqrt(gamma) S_j (lower), 28 sqrt(gamma) tau,
 *   29-31 sqrt(gamma) B^i (upper).
 * Node order: index 0 of r is r_out, index 0 of theta is th_max.
 *
 * Ownership: the caller owns all device memory.  grmhd_query_bytes() gives
 * the sizes of the two device buffers ("resident": state, static fields,
 * operators; "scratch": stage temporaries) that grmhd_create() borrows for
 * the context's lifetime.  The library never allocates or frees device
 * memory.  Every call that takes a device pointer expects memory on the
 * context's device.  All work is enqueued on the caller's HIP stream; a
 * right-hand side evaluation also forks part of its work (primitive recovery,
 * flux derivatives) to a stream the context owns (default priority) and
 * joins it back into the caller's stream before its last launch, so the
 * caller's stream alone orders every result.  Calls marked "syncs" wait for
 * that stream.
 *
 * Errors: functions return GRMHD_OK (0) or a negative code; the thread-local
 * message of the last failure is grmhd_last_error().  Device-side faults
 * surface at the next syncing call.  Con2prim failures are not errors: they
 * are counted (grmhd_diagnostics) and handled by the atmosphere policy.
 * A context is single-threaded; different contexts are independent.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GRMHD_OK = 0,
  GRMHD_E_ARG = -1,      /* invalid argument (null pointer, bad size, ...) */
  GRMHD_E_SIZE = -2,     /* buffer size does not match the grid            */
  GRMHD_E_DEVICE = -3,   /* HIP runtime error                              */
  GRMHD_E_STATE = -4,    /* call out of order (e.g. step before a state)   */
  GRMHD_E_BUDGET = -5,   /* server: job does not fit the memory budget     */
  GRMHD_E_UNAVAILABLE = -6  /* entry point switched off in this library       */
};

#define GRMHD_NFIELDS 32
#define GRMHD_NFIELDS_GLM 33   /* with GLM constraint damping: psi is field 32 */

/* Precision of the derivative contractions (the only part that changes):
 * FP64; FP32 MFMA with FP32 accumulation; split-BF16 x3 MFMA with FP32
 * accumulation; FP64 MFMA writing FP32 derivative arrays (GRMHD_STORE_FP32:
 * the FP64 arithmetic, rounded once when stored).  In the reduced forms the
 * derivative arrays are FP32 (half the bytes the stage reads and writes for
 * them); the metric reconstruction, con2prim, RHS algebra, constraint damping
 * terms, the RK accumulator and the filter stay FP64. */
typedef enum {
  GRMHD_FP64 = 0,
  GRMHD_MIX_FP32 = 1,
  GRMHD_MIX_BF16X3 = 2,
  GRMHD_STORE_FP32 = 3
} grmhd_prec;

/* Grid (Methods, "Grid Discretization"; readings: log radial map, Chebyshev
 * theta on [th_min, th_max]).  n_r, n_theta >= 4; n_phi even, >= 4;
 * each <= 256. */
typedef struct {
  int32_t nr, nth, nph;
  double r_in, r_out;       /* radial domain, 0 < r_in < r_out               */
  double th_min, th_max;    /* polar domain, 0 < th_min < th_max < pi        */
  double filt_alpha;        /* exponential filter strength (36)              */
  int32_t filt_order;       /* filter order p (16)                           */
  int32_t filter_on;        /* 1: filter after every RK4 step                */
  int32_t dealias;          /* 1: 2/3 truncation after every RK4 step
                               (Methods, "Dealiasing and Spectral Filtering":
                               Chebyshev modes k > 2(N-1)/3 and Fourier modes
                               |k| > N/3 zeroed), before the filter; the two
                               share one operator pass                       */
} grmhd_grid;

/* Initial-data kinds: magnetised Michel accretion (monopole field, density
 * perturbation) or a Fishbone-Moncrief torus (constant u^t u_phi, one
 * poloidal field loop, pressure perturbation). */
enum { GRMHD_ID_MICHEL = 0, GRMHD_ID_TORUS = 1 };

/* Physics and initial-data parameters. */
typedef struct {
  double M, a;              /* black-hole mass and spin (Kerr-Schild)        */
  double gamma_ad;          /* ideal-gas adiabatic index Gamma               */
  double cfl;               /* dt = cfl * min(dr, r dth, r sin th dph)       */
  double eta;               /* Gamma-driver damping                          */
  int32_t cowling;          /* 1: fixed background (the paper's fixed-
                               background version, "Numerical Implementation
                               of Coupled GRMHD-Einstein Evolution"): only
                               fields 24.. evolve and are filtered; the 24
                               spacetime fields keep their values bit for bit */
  int32_t gauge_k0;         /* 1: d_t alpha = ... - 2 alpha (K - K0)         */
  double r_c, rho_c;        /* Michel sonic radius, density there            */
  double beta_min;          /* min over nodes of 2p/b^2 (monopole field)     */
  double pert_amp;          /* rho -> rho (1 + pert_amp (2u - 1))            */
  uint64_t seed;            /* SplitMix64 seed of the perturbation           */
  double rho_floor, p_floor;/* atmosphere: rho_floor r^-1.5, p_floor r^-2.5  */
  int32_t id_kind;          /* GRMHD_ID_MICHEL or GRMHD_ID_TORUS             */
  double tor_r_in, tor_r_max;/* torus inner edge and pressure maximum (M)    */
  double tor_rho_max;       /* torus density at the pressure maximum         */
  double tor_atm;           /* atmosphere rho = tor_atm rho_max (r/r_max)^-1.5,
                               at Eulerian rest on the torus isentrope       */
  double tor_loop_cut;      /* A_phi = max(rho/rho_max - tor_loop_cut, 0)    */
  /* GLM constraint damping (Methods, "GLM Constraint Damping Source"; reading:
   * index raised with the spatial metric, Dedner's sign): a 33rd field psi
   * with d_t psi = -c_h^2 d_i(sqrt(gamma) B^i)/sqrt(gamma) - psi/tau and the
   * induction source -sqrt(gamma) gamma^{ij} d_j psi.  0: off (32 fields). */
  int32_t glm;
  double glm_ch, glm_tau;   /* c_h (<= 1 for the CFL bound) and tau > 0      */
  /* 1: the paper's operator-split coupled step (Methods, "Coupled Main Loop";
   * reading: symmetric form) in place of the unsplit classic RK4: classic RK4
   * over dt/2 of fields 24.. on the frozen spacetime, one forward-Euler step
   * dt of the 24 spacetime fields (BSSN + gauge) with the matter frozen,
   * classic RK4 over dt/2 of fields 24.. on the new spacetime, then the
   * filter.  Requires cowling = 0. */
  int32_t split;
  /* Primitive recovery: 0 the exact inverse (safeguarded Newton), 1 the
   * paper's damped iteration (Methods, "The Primitive Variable Recovery";
   * readings: predicted values from the standard conserved variables, velocity
   * update with the index raised by gamma^{ij}, lambda = 0.5 halved on a
   * residual increase, at most 40 tries, then one Newton step on eps) started
   * from the previous recovery; the recovery right after init_state or
   * set_state is exact. */
  int32_t c2p_damped;
} grmhd_phys;

/* Diagnostics (Results: "Magnetic Constraint", "The Entropy Curve"; the
 * Hamiltonian and momentum constraints the coupled evolution monitors,
 * Results, coupled-evolution passage, and Methods, "Initial Data Solver XCTS
 * Approximation").  The primitives behind rest mass, entropy and max W come
 * from an exact recovery of the current state. */
typedef struct {
  double t;                 /* simulation time                              */
  int64_t step;             /* completed RK4 steps                          */
  int64_t c2p_fail;         /* points that took the atmosphere policy in the
                               evolution's last primitive recovery (the last
                               RHS evaluation, or the recovery that primes the
                               warm start after init_state / set_state)     */
  int64_t nonfinite;        /* NaN/Inf entries in the state                  */
  double rest_mass;         /* sum sqrt(gamma) D w (quadrature weights w)    */
  double entropy;           /* E^n = sum rho s sqrt(gamma) w                 */
  double max_abs_divB;      /* max |d_i (sqrt(gamma) B^i)|                  */
  double min_alpha, max_W;
  double ham_l2;            /* sqrt(sum H^2 w / sum w), Hamiltonian constraint
                               H = R + 2/3 K^2 - A_ij A^ij - 16 pi E          */
  double ham_linf;          /* max |H| over the nodes                        */
  double mom_l2;            /* sqrt(sum |M|^2 w / sum w), momentum constraint
                               M_i = D_j (K^j_i - delta^j_i K) - 8 pi S_i in
                               BSSN form, |M|^2 = gamma^ij M_i M_j           */
  double mom_linf;          /* max |M| over the nodes                        */
} grmhd_diag;

typedef struct grmhd_ctx grmhd_ctx;

/* Bytes of device memory the context borrows (resident, scratch). */
int grmhd_query_bytes(const grmhd_grid* grid, grmhd_prec prec,
                      size_t* resident_bytes, size_t* scratch_bytes);

/* Build operators (host, long double) and upload them into dev_resident.
 * dev_resident / dev_scratch: device buffers of at least the queried sizes,
 * 256-byte aligned; hip_stream: a hipStream_t (0 = null stream).  Syncs.
 * GRMHD_E_ARG for a grid or parameter out of range (Gamma > 1, cfl > 0,
 * 0 <= |a| <= M, finite floors > 0, switches 0 or 1, ...).
 * dev_scratch may be NULL: such a context is stepped by grmhd_step_noalloc
 * only; its state comes from grmhd_set_state with a host K0 (init_state,
 * set_state without K0, rhs, step, step_batch, diagnostics and profile_step
 * return GRMHD_E_STATE), and get_state, state_ptr, con2prim and
 * apply_operator work as usual. */
int grmhd_create(const grmhd_grid* grid, const grmhd_phys* phys, grmhd_prec prec,
                 void* dev_resident, void* dev_scratch, void* hip_stream,
                 grmhd_ctx** out);

/* Waits for the streams, releases the context's own stream and events and
 * the host metadata (never device memory). */
int grmhd_destroy(grmhd_ctx* ctx);

/* Kerr-Schild background in BSSN variables + magnetised Michel flow + seeded
 * density perturbation (or the torus of id_kind), computed on the host (the
 * (theta, r) plane) and expanded on the device; sets K0 and primes the
 * con2prim guesses.  t = 0.  Syncs.  GRMHD_E_ARG, state untouched, when the
 * data do not exist for the parameters: M = 0, pert_amp outside [0, 1),
 * rho_c or beta_min not > 0, r_c inside the Michel bound
 * M (3 Gamma - 2) / (2 (Gamma - 1)), or any non-finite plane value. */
int grmhd_init_state(grmhd_ctx* ctx);

/* Copy a state in (host, n = 32 P doubles, layout above; a GLM context also
 * takes n = 33 P with psi last, and sets psi = 0 for n = 32 P), set the static
 * 1+log source K0 (host, P doubles; NULL: K0 = K - beta^k d_k alpha/(2 alpha)
 * computed on the device from the state) and the time t; primes the
 * con2prim guesses by a cold-start recovery.  Syncs. */
int grmhd_set_state(grmhd_ctx* ctx, const double* host_U, size_t n,
                    const double* host_K0, double t);

/* Copy the state (n = 32 P, or 33 P with psi last in a GLM context; and
 * optionally K0, P doubles) out.  Syncs. */
int grmhd_get_state(grmhd_ctx* ctx, double* host_U, size_t n, double* host_K0);

/* Device pointers of the resident state (32 P doubles, then psi in a GLM
 * context) and K0 (P doubles);
 * valid for the context's lifetime.  No copy, no sync.  With cowling = 1 the
 * background (fields 0..23) is read, and its first derivatives recomputed, at
 * the first step after init_state, set_state or this call: write the
 * background through the pointer before stepping, not between steps. */
int grmhd_state_ptr(grmhd_ctx* ctx, double** dev_U, double** dev_K0);

/* One RHS evaluation dU/dt = L(U) of a device state (32 P doubles, 33 P in
 * a GLM context) into dev_dUdt (as many); uses the context's K0 and con2prim
 * guesses.  With cowling = 1 the background is dev_U's spacetime (its first
 * derivatives are recomputed) and fields 0..23 of dev_dUdt are set to zero.
 * dev_U may be the resident state; dev_dUdt must not overlap dev_U
 * (GRMHD_E_ARG).  Async. */
int grmhd_rhs(grmhd_ctx* ctx, const double* dev_U, double* dev_dUdt);

/* nsteps classic RK4 steps of size grmhd_dt(), each followed by the filter
 * when enabled.  Async. */
int grmhd_step(grmhd_ctx* ctx, int32_t nsteps);

/* nsteps RK4 steps (+ filter) of n contexts of one grid class, each kernel
 * launched once for all of them (continuous batching; up to 32 jobs per
 * launch, larger n is split).  The contexts must share grid sizes, precision,
 * the filter and dealiasing switches, the kernel parameters (Gamma, eta,
 * floors, cowling, gauge_k0, GLM with c_h and tau), the split step and the
 * damped recovery switches, the stream and the offset between their scratch
 * and resident buffers (else GRMHD_E_ARG); r_in, r_out, the theta range, the
 * filter constants, the spin, the initial data and dt may differ.  Each job's arithmetic is the same
 * as when stepped alone (bitwise).  Async. */
int grmhd_step_batch(grmhd_ctx* const* ctxs, int32_t n, int32_t nsteps);

/* Size of the library's own device array behind grmhd_step_noalloc (one per
 * GPU the library runs on, held until the process ends): the largest scratch
 * size (grmhd_query_bytes) of a grid it steps, about 29,000 grid points. */
#define GRMHD_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): nsteps
 * RK4 steps exactly as grmhd_step takes them (the same kernels, bitwise the
 * same result), with the stage temporaries in the library's own device
 * array instead of the context's scratch buffer, so the context may have
 * been created with dev_scratch = NULL.  Allocates nothing.  GRMHD_E_SIZE
 * when the grid's scratch size exceeds GRMHD_NOALLOC_SCRATCH_BYTES;
 * GRMHD_E_ARG unless the context's device is the current one.  The array is
 * shared by every call on a GPU and keeps the last call's contents (nothing
 * in it is assumed to start at zero; a fixed background's derivatives are
 * recomputed at each call): calls that overlap on one GPU -- from other
 * threads, or queued on different streams -- race.  Async. */
int grmhd_step_noalloc(grmhd_ctx* ctx, int32_t nsteps);

/* Override the time step (e.g. dt = T / ceil(T / dt) to land on an end time). */
int grmhd_set_dt(grmhd_ctx* ctx, double dt);

/* Move the context to another stream (waits for the old one). */
int grmhd_set_stream(grmhd_ctx* ctx, void* hip_stream);

/* Host only: the CFL time step of a grid without creating a context. */
int grmhd_time_step(const grmhd_grid* grid, double cfl, double* dt);

/* Reductions over the current state (FP64 derivatives whatever the context's
 * precision; uses the scratch buffer, so call it between steps).  Leaves the
 * evolution's primitive warm start and failure flags untouched.  Syncs. */
int grmhd_diagnostics(grmhd_ctx* ctx, grmhd_diag* out);

double grmhd_dt(const grmhd_ctx* ctx);
double grmhd_time(const grmhd_ctx* ctx);
const char* grmhd_last_error(void);

/* ---- operator access (tests and tools) --------------------------------- */

/* Apply one spectral operator along one axis to nfields device fields
 * (each P doubles, layout above) from dev_in into dev_out.
 * axis: 0 = r, 1 = theta, 2 = phi.  op: 1 = first derivative, 2 = second
 * derivative, 3 = filter.  Uses the same contraction kernels as the RHS.
 * Async. */
int grmhd_apply_operator(grmhd_ctx* ctx, int32_t axis, int32_t op,
                         const double* dev_in, double* dev_out, int32_t nfields);

/* Primitive recovery (Methods, "The Primitive Variable Recovery": the
 * unique primitive state reproducing U) and densitised fluxes of a device
 * state (32 P doubles, layout above; the metric is reconstructed from its
 * fields 0..6): writes dev_prim (5 P doubles: rho, p, v^r, v^theta, v^phi)
 * and, if non-null, dev_flux (24 P doubles, [direction][variable], variables
 * in state order 24..31) and dev_fail (P doubles: 1.0 where the point took
 * the atmosphere policy -- D <= 0, tau + D <= 0, no root with v^2 < 1, no
 * convergence within the iteration budget, or rho, p below the floors --
 * else 0.0).  The iteration starts from the context's last recovery and
 * leaves its result there as the next warm start.  Async. */
int grmhd_con2prim(grmhd_ctx* ctx, const double* dev_U, double* dev_prim,
                   double* dev_flux, double* dev_fail);

/* ---- initial data: conformally flat, time-symmetric (XCTS approximation) -- */

/* The conformal factor psi of the conformally flat, time-symmetric data
 * gamma_ij = psi^4 f_ij (f the flat metric of the grid's spherical
 * coordinates, A_ij = 0, K = 0) of Methods, "Initial Data: Approximate XCTS
 * Solution": the Hamiltonian constraint Lap psi = -2 pi E psi^5 solved by
 * fixed-point relaxation -- each iteration solves the linear problem
 * Lap psi_{k+1} = -2 pi E psi_k^5 (flat Laplacian, the grid's spectral
 * collocation) exactly, by fast diagonalisation: real Fourier transform in
 * phi and, per mode, the eigenvectors of the radial and polar operators
 * (host eigen-decompositions, once per call), applied along grid lines on the
 * device.
 * dev_E: energy density seen by normal observers (P doubles, layout of a
 * field), held fixed.  dev_psi (P doubles): in, the initial guess, whose
 * values on the r-end and theta-end nodes are the Dirichlet data (phi is
 * periodic); out, the solution.  Iterates until the largest change is at most
 * tol times max |psi| or max_iter iterations; iters and change (optional)
 * receive the count and the last relative change (NaN propagates: a
 * non-finite iterate stops the iteration).  Uses the context's grid and
 * scratch buffer (between steps); the state is not touched.  n_r, n_theta
 * >= 3.  GRMHD_E_ARG if an operator has complex eigenvalues.  Syncs.
 * Switched off: after the argument checks it returns GRMHD_E_UNAVAILABLE
 * without touching the device.  Its first run on the hardware ended in a
 * device fault whose cause has not been found (the kernels' indexing checks
 * out on the CPU); the solver stays in the source until one is. */
int grmhd_xcts_solve(grmhd_ctx* ctx, const double* dev_E, double* dev_psi, int32_t max_iter, double tol,
                     int32_t* iters, double* change);

/* ---- served form: continuous-batching job server ------------------------- */

typedef struct grmhd_server grmhd_server;

typedef struct {
  int64_t id;
  int32_t state;            /* 0 queued, 1 running, 2 done, 3 rejected,
                               4 cancelled                                   */
  int32_t nr, nth, nph, prec;
  int64_t steps_done, steps_total;
  double dt;                /* T / steps_total                               */
  double t_arrival, t_admit, t_done;  /* server clock, seconds               */
  double latency;           /* t_done - t_arrival (done jobs), else -1       */
  size_t bytes;             /* device footprint (resident + scratch)         */
} grmhd_job_info;

typedef struct {
  int64_t submitted, completed, rejected, running, queued, cancelled;
  double p50_latency, p99_latency, mean_latency;  /* completed jobs, seconds  */
  double point_stage_updates;  /* completed work: sum over jobs of 4 P steps */
  double wall;              /* first submission to last completion, seconds  */
  double busy;              /* seconds with device work in flight, as seen
                               by the ticks (0 in a dry run)                */
  size_t bytes_in_use, bytes_peak;
} grmhd_server_summary;

/* A server that places jobs in the caller's device arena (dev_arena,
 * arena_bytes = the memory budget; 256-byte aligned) and steps jobs of one
 * grid class together, at most max_batch per launch sequence.  Each grid
 * class runs on a stream of its own (default priority) and advances at its
 * own pace, with up to two RK4 steps in flight; initial data are built on an
 * admission stream of the server's.  hip_stream is the fallback stream.
 * dev_arena NULL: dry run, no device work (each job step completes at once),
 * for exercising the scheduling logic without a GPU. */
int grmhd_server_create(void* dev_arena, size_t arena_bytes, int32_t max_batch, void* hip_stream,
                        grmhd_server** out);
int grmhd_server_destroy(grmhd_server* srv);

/* Queue a job that evolves (grid, phys) from its initial data to t_end; the
 * arrival time is the server clock now.  keep_state: copy the final state to
 * host memory at completion (grmhd_server_result).  A job larger than the
 * whole budget is recorded as rejected (GRMHD_E_BUDGET); a grid, precision
 * or parameter set that grmhd_create would refuse, or for which
 * grmhd_init_state has no data (M = 0, pert_amp outside [0, 1), beta_min or
 * rho_c not > 0, r_c inside the Michel bound, bad torus parameters), is
 * refused with GRMHD_E_ARG and not queued. */
int grmhd_server_submit(grmhd_server* srv, const grmhd_grid* grid, const grmhd_phys* phys,
                        grmhd_prec prec, double t_end, int32_t keep_state, int64_t* job_id);

/* One scheduling round: count the RK4 steps that have completed on the
 * device (event queries per grid class) and retire jobs that reached their
 * end time, freeing their memory; admit queued jobs in arrival order while
 * they fit, at most four per tick (a dry run admits all that fit; a job whose
 * context or initial data cannot be built is marked
 * rejected, its message left in grmhd_server_last_error, and the round goes
 * on); launch the next step of every class with room in its two-step
 * pipeline (one batched launch sequence per class).  Returns without waiting
 * for launched work, except that a round with nothing to complete, admit or
 * launch waits until some class's step completes.  n_pending: queued +
 * running after the tick. */
int grmhd_server_tick(grmhd_server* srv, int32_t* n_pending);

int grmhd_server_poll(grmhd_server* srv, int64_t job_id, grmhd_job_info* out);
/* Cancel a queued or running job.  A queued job leaves the queue at once; a
 * running job takes part in no further step and its context and arena block
 * are released by the first tick at which none of its steps is still in
 * flight on the device (until then it polls as running, with no steps to
 * go).  Either way it ends in state 4 (cancelled), its memory available to
 * the jobs admitted after it.  GRMHD_E_ARG for an unknown job, GRMHD_E_STATE
 * for one already done, rejected or cancelled. */
int grmhd_server_cancel(grmhd_server* srv, int64_t job_id);
/* Final state of a finished job submitted with keep_state (n = 32 P; 33 P,
 * psi last, for a GLM job). */
int grmhd_server_result(grmhd_server* srv, int64_t job_id, double* host_U, size_t n);
int grmhd_server_stats(grmhd_server* srv, grmhd_server_summary* out);
double grmhd_server_clock(const grmhd_server* srv);
const char* grmhd_server_last_error(void);

/* ---- timing ---------------------------------------------------------------- */

/* Launch kinds of one RK4 step (per stage: con2prim, 3 flux-derivative and
 * 3 (folded forms) or 6 state-derivative launches, RHS; then 3 filter
 * launches). */
enum {
  GRMHD_K_C2P_FLUX = 0,   /* con2prim + densitised fluxes                        */
  GRMHD_K_DERIV_R2 = 1,   /* r axis, first + second derivative (11 fields)        */
  GRMHD_K_DERIV_R1 = 2,   /* r axis, first derivative (10 fields)                 */
  GRMHD_K_DERIV_T2 = 3,   /* theta axis, first + second                            */
  GRMHD_K_DERIV_T1 = 4,   /* theta axis, first (10 + 11 mixed)                     */
  GRMHD_K_DERIV_P2 = 5,   /* phi axis, first + second                              */
  GRMHD_K_DERIV_P1 = 6,   /* phi axis, first (10 + 22 mixed)                       */
  GRMHD_K_RHS_RK = 7,     /* BSSN (Ricci tensor included) + Valencia RHS, RK4 stage */
  GRMHD_K_FILTER_R = 8, GRMHD_K_FILTER_T = 9, GRMHD_K_FILTER_P = 10,
  GRMHD_K_DERIV_R = 11,   /* r axis, first + second and first-only tasks in one launch */
  GRMHD_K_DERIV_T = 12,   /* theta axis, likewise                                      */
  GRMHD_K_DERIV_P = 13,   /* phi axis, likewise                                        */
  GRMHD_K_RICCI = 14,     /* a separate Ricci launch: none (count 0; the RHS forms it) */
  GRMHD_K_DFLUX_R = 15,   /* r derivatives of the 8 densitised fluxes                  */
  GRMHD_K_DFLUX_T = 16,   /* theta derivatives of the fluxes                           */
  GRMHD_K_DFLUX_P = 17,   /* phi derivatives of the fluxes                             */
  GRMHD_K_COUNT = 18
};

/* Advance nsteps RK4 steps as grmhd_step does, but with every launch in
 * order on the context stream (no fork to the context's own stream), and
 * record a HIP event after every launch; ms[k] (nkinds >= GRMHD_K_COUNT)
 * receives the average duration in milliseconds of launch kind k (time
 * between the event before and after it) and counts[k] (optional) the
 * number of launches of that kind.  Syncs. */
int grmhd_profile_step(grmhd_ctx* ctx, int32_t nsteps, double* ms, int32_t nkinds, int32_t* counts);

#ifdef __cplusplus
}
#endif

#endif /* GRMHD_H */
