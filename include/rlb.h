/*
 * rlb.h -- C ABI of the MI355X (gfx950) implementation of the per-cell,
 * per-timestep update of the ultra-relativistic lattice Boltzmann model of
 * Mohseni, Mendoza, Succi and Herrmann, "Lattice Boltzmann model for
 * ultra-relativistic flows" (arXiv:1302.1125).
 *
 * One update (rlb_step) performs, for every cell, the steps of the extended
 * model of Sec. II.A:
 *   1. moments T^{00}, T^{0a} of f and N^0 of h (Eq. (36) and the number
 *      current of Sec. II);
 *   2. recovery of eps, u, n with the equation of state eps = 3p (Eq. (38));
 *   3. the discrete Maxwell-Juttner equilibrium on the extended D3Q19 set
 *      (Eqs. (29), (36), (42)-(46), moment-exact reading) and the density
 *      equilibrium (Eq. (58));
 *   4. minmod flux-limited streaming (Eqs. (47)-(53)) and the bulk-viscosity
 *      term (Eqs. (54)-(55));
 *   5. the implicit BGK/Marle update (Eq. (57)), or in Euler mode
 *      f := f^eq of the post-streaming moments (Sec. III, inviscid case).
 *
 * Conventions
 *   - Every call returns an rlb_status; no C++ exception crosses the ABI.
 *   - Host field arrays are FP64, length nx*ny*nz, C order [z][y][x]
 *     (x fastest).  The caller owns them; calls copy synchronously on the
 *     context's stream.
 *   - The context owns all device memory (allocated in rlb_create, released
 *     in rlb_destroy).  Device memory per cell: 2 x 19 populations of f and
 *     (with density) of h in the storage precision (ping-pong), plus 5 FP64
 *     fields of the previous step (and, for the implicit mixed-precision
 *     step of a 2D or 3D grid, 5 FP32 ones: the step keeps its history in
 *     FP32) and, with obstacles, 1 byte.
 *   - Threading: one context per host thread at a time.  Contexts are
 *     independent.  Results are deterministic for a given configuration
 *     and device.
 *   - No CPU fallback exists: without a usable gfx950 device rlb_create
 *     returns RLB_E_DEVICE.
 */
#ifndef RLB_H
#define RLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlb_ctx rlb_ctx; /* opaque */

typedef enum {
  RLB_OK = 0,
  RLB_E_INVALID_ARG = -1,   /* bad pointer, size, enum or parameter      */
  RLB_E_OUT_OF_MEMORY = -2, /* device allocation failed                   */
  RLB_E_DEVICE = -3,        /* HIP runtime error / no usable device       */
  RLB_E_INADMISSIBLE = -4,  /* initial fields or a step left the
                               admissible set (see rlb_step)              */
  RLB_E_STATE = -5          /* call out of order, or context poisoned by a
                               previous inadmissible step                */
} rlb_status;

enum { RLB_FP64 = 0, RLB_MIXED = 1 };              /* storage/arith precision */
enum { RLB_FLUX_MINMOD = 0, RLB_FLUX_RUSANOV = 1 }; /* Eqs. (47)-(53) | Rusanov */
enum { RLB_COLL_IMPLICIT = 0, RLB_COLL_EULER = 1 }; /* Eq. (57) | Sec. III     */
enum { RLB_TAU_UNIFORM = 0, RLB_TAU_ETA_OVER_S = 1 };
enum { RLB_BC_PERIODIC = 0, RLB_BC_FIXED = 1, RLB_BC_OUTFLOW = 2 };
enum { RLB_LATTICE_EXTENDED = 0, RLB_LATTICE_BASIC = 1 };  /* Sec. II.A | Sec. II */
enum { RLB_DENSW_PAPER = 0, RLB_DENSW_ISOTROPIC = 1 };      /* density weights */

/* Run configuration.  Lattice units: delta x = 1. */
typedef struct {
  uint32_t struct_size; /* = sizeof(rlb_config) (ABI check)                 */
  int32_t nx, ny, nz;   /* grid; ny == 1 requires nz == 1; nx >= 2.  Axes
                           of size 1 must be periodic (quasi-1D / 2D).
                           At most 2^28 - 128 cells in all, counted as
                           stored: a 2D/3D grid takes (nx rounded up to a
                           multiple of 64) x (ny rounded up to a multiple
                           of 4) x nz cells on the device.                  */
  int32_t precision;    /* RLB_FP64: populations stored and updated in FP64.
                           RLB_MIXED: populations stored and streamed in
                           FP32; moments accumulated in FP64; recovery and
                           equilibrium coefficients in FP64.                */
  int32_t collision;    /* RLB_COLL_IMPLICIT | RLB_COLL_EULER               */
  int32_t tau_mode;     /* RLB_TAU_UNIFORM: tau given.
                           RLB_TAU_ETA_OVER_S: per cell from Eq. (41),
                           tau = 1/2 + nu^2 (eta/s) s/(eps+p), with
                           s = n (4 - ln(n/T^3)), T = p/n (lattice units,
                           d_G/pi^2 = 1); without density n = T^3.
                           The extended scheme's shear viscosity is
                           (4/sqrt 27) tau (eps+p)/nu^2 (Chapman-Enskog
                           with the moment-exact equilibrium), so this
                           mode realises 4/sqrt(27) = 0.77 of the given
                           eta/s.                                          */
  int32_t with_density; /* 1: carry the density distribution h (Eq. (58)) */
  double nu;            /* nu = c/c_s (Sec. II); > 0                        */
  double dt_over_dx;    /* time step; (0, 0.5]                              */
  double tau;           /* relaxation time (RLB_TAU_UNIFORM); > 0           */
  double eta_over_s;    /* shear viscosity to entropy ratio; >= 0           */
  double alpha;         /* bulk constant alpha of Eq. (55); >= 0; 0 = off   */
  int32_t bc[6];        /* faces -x,+x,-y,+y,-z,+z: RLB_BC_*.  Periodic
                           faces come in pairs.  FIXED ghosts hold the
                           equilibrium of face_states (the paper's inlet,
                           Sec. III); OUTFLOW is a zero-gradient copy.      */
  double face_states[6][5]; /* (eps, ux, uy, uz, n) per FIXED face          */
  double guard_umax;    /* continuous admissibility guard: 0 = off, else a
                           speed in (0,1).  After each update a cell whose
                           new moments leave |T^{0a}| <= m_1 T^{00} is
                           blended towards the equilibrium of its moments
                           projected into T^{00} >= floor,
                           |T^{0a}| <= m_max T^{00} (and n >= floor);
                           m(u) = 4u/(3+u^2), m_max = m(guard_umax),
                           m_1 = m(1 - 2(1 - guard_umax)).  Not in the
                           paper; it is silent on inadmissible states.      */
  double guard_efloor;  /* floor of T^{00} and n used by the guard; > 0     */
  int32_t lattice;      /* RLB_LATTICE_EXTENDED (default): the extended
                           model above.  RLB_LATTICE_BASIC: the basic model
                           of Sec. II -- standard D3Q19 set (diagonal links
                           (+-1,+-1,0), c_a = sqrt(19)/nu), exact streaming
                           with dt = c_t dx/(c_a c_0) = sqrt(27/19) dx (so
                           dt_over_dx is ignored), explicit Marle collision
                           f' = f - omega (f - f^eq), omega = nu^2/(sqrt(19)
                           tau), no limiter, no bulk term.  Requires
                           collision = RLB_COLL_IMPLICIT (the regular
                           collision), with_density = 0 (the paper gives the
                           density distribution for the extended set only),
                           alpha = 0 and guard_umax = 0.  The explicit
                           collision is stable only for omega < 2.          */
  int32_t density_weights; /* weights w'_i of the density equilibrium,
                           Eq. (58), which fixes them only through
                           sum w' = 1 and sum w' c^a c^b = delta^{ab}/3 (one
                           free parameter with one weight per shell).
                           RLB_DENSW_PAPER (default): Eqs. (59)-(60),
                           w'_0 = 1/10; the diagonal weight is negative for
                           c_a^2 = 13/nu^2 > 10/9 (nu < 3.42), where the
                           density part is linearly unstable for uniform
                           flows faster than |u| ~ 0.2.
                           RLB_DENSW_ISOTROPIC (not in the paper): the free
                           parameter fixed by isotropy of the fourth moment,
                           w' = (1 - 17/(24 c_a^2), 1/(9 c_a^2),
                           1/(288 c_a^2)), non-negative; no linear growth of
                           the density part up to |u| = 0.995 at dt 0.25
                           (1D) and 0.15 (3D).  Extended lattice only, and
                           nu <= sqrt(13 * 24/17) = 4.28.                   */
  int32_t flux;         /* streaming flux of the extended lattice.
                           RLB_FLUX_MINMOD (default): the minmod-limited
                           upwind flux of Eqs. (47)-(53).
                           RLB_FLUX_RUSANOV (not in the paper): the
                           first-order Rusanov (local Lax-Friedrichs) flux
                           1/2 p (f_L + f_R) - 1/2 s (f_R - f_L) with the
                           speed of light as the dissipation speed s of every
                           population, moving or not; the moments of the
                           update are then the Rusanov scheme of the fluid
                           equations, and in the Euler mode
                           (RLB_COLL_EULER) an admissible state stays
                           admissible (e.g. the gamma = 10 colliding slabs
                           run without the guard; the convexity holds for
                           dt/dx <= 1/(number of axes)).  With this flux the
                           bulk term of Eq. (54) acts on the rest population
                           too, so that it diffuses every moment alike.  The implicit update
                           is not made admissible by it.  Extended lattice
                           only; not in the server (1D grids run it in the
                           blocked step, 2D and 3D grids in the staged step,
                           not the z-march).                               */
} rlb_config;

typedef struct {
  int64_t steps;          /* steps taken since the last rlb_init_fields     */
  int64_t guard_events;   /* cell-steps in which the guard blended          */
  int64_t first_bad_step; /* index of the first inadmissible step, or -1   */
  double sum_T00;         /* domain sums of T^{00}, T^{0a}, N^0 of the     */
  double sum_T0x;         /* current populations (FP64, fixed reduction    */
  double sum_T0y;         /* order, so deterministic)                       */
  double sum_T0z;
  double sum_N0;
} rlb_stats;

/* Fill *cfg with defaults: 64x1x1, FP64, implicit, uniform tau = 1,
   nu = 27^(1/4), dt = 0.25, alpha = 0, no density, periodic, guard off,
   guard_efloor = 1e-10, extended lattice. */
rlb_status rlb_config_default(rlb_config* cfg);

/* Set up one run of the extended model (Sec. II.A) for the problem
   statement of the paper's Sec. III set-ups: lattice (nu), time step,
   viscosity (tau or eta/s, Eq. (41)), bulk constant alpha (Eq. (55)),
   boundaries (fixed inlet states, open faces).  Validate cfg, allocate
   device memory on the current HIP device and compute the fixed-face
   equilibria (Eq. (36) reading, Eq. (58)).  hip_stream: a hipStream_t to run on
   (e.g. torch's current stream), or NULL for a stream the context creates
   and owns.  On error *out is NULL and nothing is allocated. */
rlb_status rlb_create(const rlb_config* cfg, void* hip_stream, rlb_ctx** out);

/* Set the initial fields (Sec. III initial conditions): f := f^eq(eps,u),
   h := h^eq(n,u) in every cell, and the previous-step fields := these
   fields (so f^eq(t - dt) = f^eq(t) at the first step).  eps, ux, uy, uz:
   required; n: required iff with_density (ignored otherwise; the lattice
   equilibrium density (eps/3)^(3/4) is used); obstacle: NULL or an nx*ny*nz
   byte mask whose non-zero cells are held at the equilibrium of their
   initial fields at every step (Sec. III, shock-cloud setup).
   Returns RLB_E_INADMISSIBLE (state unchanged) if any value is non-finite,
   eps <= 0, |u| >= 1 or (with density) n <= 0.  Resets the step counter,
   the guard counter and a poisoned state. */
rlb_status rlb_init_fields(rlb_ctx* ctx, const double* eps, const double* ux,
                           const double* uy, const double* uz, const double* n,
                           const uint8_t* obstacle);

/* Advance nsteps >= 0 updates of Eq. (57) (moments, recovery with
   eps = 3p, equilibria, minmod-limited streaming of Eqs. (47)-(53), bulk
   term of Eqs. (54)-(55), implicit collision; Euler mode: f := f^eq of the
   post-streaming moments, Sec. III) -- one fused kernel launch per update
   on the context's stream (1D grids: several updates per launch, see
   rlb_steps_per_launch) -- then synchronise once.  If a step's recovery met a
   non-obstacle cell with T^{00} <= 0, |T^{0a}| >= T^{00}, N^0 <= 0 (with
   density) or a non-finite value, returns RLB_E_INADMISSIBLE; rlb_stats
   reports the first such step and later calls return RLB_E_STATE until
   rlb_init_fields. */
rlb_status rlb_step(rlb_ctx* ctx, int64_t nsteps);

/* Enqueue nsteps updates without synchronising or checking (for callers
   that time or overlap work on the stream).  Check the outcome later with
   rlb_sync. */
rlb_status rlb_step_async(rlb_ctx* ctx, int64_t nsteps);

/* Synchronise the context's stream and report inadmissible steps as
   rlb_step does. */
rlb_status rlb_sync(rlb_ctx* ctx);

/* Fields of the current populations: eps, u (and n) recovered in FP64 as
   in step 2, from the moments T^{00}, T^{0a} of f (Eq. (36)) and N^0 of h
   with eps = 3p (Eq. (38)).  Any output pointer may be NULL (skipped).  n without density
   is (eps/3)^(3/4).  Cells whose moments are inadmissible get NaN. */
rlb_status rlb_moments(rlb_ctx* ctx, double* eps, double* ux, double* uy,
                       double* uz, double* n);

/* rlb_moments without any device allocation, for callers that cannot
   allocate (code running between the captures of a HIP graph, tight serving
   loops, harnesses that forbid hipMalloc).  Same fields, same kernel and the
   same results as rlb_moments; the five FP64 fields are staged in a fixed
   device array that the library holds on every GPU it runs on until the
   process ends (40 MiB: 5 x 2^20 doubles) instead of a buffer allocated per
   call.  Grids of more than 2^20 cells (nx*ny*nz) return RLB_E_INVALID_ARG
   (use rlb_moments).  The array is shared by every context on one GPU and
   keeps the last call's contents (every call overwrites the cells it reads
   back); calls that overlap on one GPU, from different host threads or
   streams, race on it and must be serialised by the caller. */
rlb_status rlb_moments_noalloc(rlb_ctx* ctx, double* eps, double* ux, double* uy,
                               double* uz, double* n);

/* Steps one kernel launch advances: 1 for 2D/3D grids and the basic
   lattice; for 1D grids of the extended lattice the temporal-blocking depth
   (default 16 when nx <= 192 x the device's compute-unit count, so that each
   workgroup has a CU of its own, else 8; the RLB_TB_STEPS environment
   variable read at rlb_create overrides it, 1..16, 1 = one step per launch).  A launch then reads and
   writes every cell's state once for that many steps.  0 if ctx is NULL. */
int32_t rlb_steps_per_launch(const rlb_ctx* ctx);

/* Counters and FP64 domain sums (conservation diagnostics). */
rlb_status rlb_stats_get(rlb_ctx* ctx, rlb_stats* out);

/* Release the context and its device memory.  NULL is a no-op. */
void rlb_destroy(rlb_ctx* ctx);

/* Static description of a status code. */
const char* rlb_status_str(rlb_status s);

/* Message of the last error on the calling thread ("" if none). */
const char* rlb_last_error(void);

/* Device bytes a context with this configuration allocates (0 if cfg is
   invalid).  Used for memory-based admission. */
uint64_t rlb_footprint_bytes(const rlb_config* cfg);

/* ------------------------------------------------------------------------
 * Batched serving of many independent 1D solves (segment step).
 *
 * A server owns one device arena and a worker thread that runs a continuous
 * batching loop: requests submitted at any time are admitted as soon as an
 * arena range of their footprint and a slot are free (first fit, FIFO with
 * backfill); every resident request is advanced by the same fused launches
 * (one launch per step covers all of them, each with its own size, steps,
 * eta/s, alpha and end states), chained in hipGraph chunks of chunk_steps
 * steps; a request whose steps are done is read back (fields as in
 * rlb_moments) and its memory is freed for the next one.  The per-cell
 * arithmetic is the update of rlb_step (Sec. II.A, Eq. (57)), so a request's
 * result does not depend on which other requests share the launches.
 * ---------------------------------------------------------------------- */
typedef struct rlb_server rlb_server; /* opaque */

typedef struct {
  uint32_t struct_size;  /* = sizeof(rlb_request)                            */
  int32_t n;             /* cells, >= 4                                      */
  int64_t steps;         /* steps to take, >= 0                              */
  const double* eps;     /* initial fields, length n; copied at submission   */
  const double* ux;
  const double* uy;
  const double* uz;
  const double* dens;    /* required iff the server carries the density      */
  double eta_over_s;     /* used when the server's tau_mode is ETA_OVER_S    */
  double tau;            /* used when tau_mode is UNIFORM; > 0               */
  double alpha;          /* bulk constant, >= 0                              */
  int32_t bc_lo, bc_hi;  /* RLB_BC_* of the two ends (periodic in pairs)      */
  double face_lo[5];     /* (eps, ux, uy, uz, n) of a FIXED end               */
  double face_hi[5];
} rlb_request;

typedef struct {
  uint64_t submitted, admitted, completed, failed, rejected;
  uint64_t capacity_cells;          /* arena size                            */
  uint64_t resident_cells_peak;     /* most arena cells in use at once        */
  uint64_t resident_requests_peak;
  uint64_t chunks;                  /* graph launches                          */
  uint64_t global_steps;            /* steps of the batched loop               */
  double cell_updates;              /* sum of n * steps taken over retired    */
  double busy_seconds;              /* wall time with resident work            */
  double wall_seconds;              /* first submission to last completion    */
  double latency_p50, latency_p99, latency_max; /* s, submission -> result  */
} rlb_server_stats;

/* Create a server.  From *common only precision, collision, tau_mode,
   with_density, nu, dt_over_dx and the guard fields are used (grid, bc, tau,
   eta_over_s and alpha are per request).  budget_bytes: device memory of the
   arena (populations, ping-pong, previous fields; at most 2^28 - 128 cells
   are used); chunk_steps: steps per
   graph launch, even, >= 2.  The server runs on a stream it creates.
   The extended lattice only (RLB_E_INVALID_ARG for RLB_LATTICE_BASIC).
   Each launch of a chunk advances every resident request by up to 8 steps
   with the state held on chip (temporal blocking; the largest depth <= 8,
   or <= RLB_TB_STEPS from the environment, that gives an even number of
   launches per chunk; results equal one step per launch to rounding). */
rlb_status rlb_server_create(const rlb_config* common, uint64_t budget_bytes, int32_t chunk_steps,
                             rlb_server** out);

/* Queue a request (inputs are copied; returns at once).  RLB_E_OUT_OF_MEMORY
   if it can never fit the arena, RLB_E_INADMISSIBLE for inadmissible fields,
   RLB_E_INVALID_ARG for bad sizes or parameters. */
rlb_status rlb_server_submit(rlb_server* srv, const rlb_request* req, uint64_t* id);

/* Non-blocking: *done = 1 when the request's result is ready. */
rlb_status rlb_server_poll(rlb_server* srv, uint64_t id, int32_t* done);

/* Block until the request is done, copy its fields (any pointer may be NULL)
   and release it.  latency_s: submission -> result ready on the host;
   first_bad: first inadmissible local step or -1; guard_events: its count.
   A request that meets an inadmissible state stops at the first chunk
   boundary after that step (a multiple of chunk_steps from its start, so the
   same alone and in a mix); its fields are those at that boundary and the
   call returns RLB_E_INADMISSIBLE. */
rlb_status rlb_server_result(rlb_server* srv, uint64_t id, double* eps, double* ux, double* uy,
                             double* uz, double* n, double* latency_s, int64_t* first_bad,
                             int64_t* guard_events);

/* Block until every submitted request is done. */
rlb_status rlb_server_drain(rlb_server* srv);

rlb_status rlb_server_stats_get(rlb_server* srv, rlb_server_stats* out);

/* Stop the loop (pending requests fail) and free everything.  NULL: no-op. */
void rlb_server_destroy(rlb_server* srv);

/* Arena bytes one request of n cells occupies in a server with *common. */
uint64_t rlb_request_footprint_bytes(const rlb_config* common, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* RLB_H */
