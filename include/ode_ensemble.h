/*
 * ode_ensemble.h -- C ABI of the MI355X (gfx950) ensemble ODE integrator.
 *
 * Integrates very many small, independent ODE systems y' = f(y, t; p), one
 * system per GPU lane, with the adaptive Runge-Kutta-Cash-Karp 4(5) scheme or
 * fixed-step classical RK4 (paper: Hegedus, arXiv:1810.03931, Sec. 3).
 * Trajectories are never stored; per-system "accessories" (running extrema
 * and their times, Sec. 5), event detection with secant location, event
 * actions such as impact laws, and stop conditions (Sec. 4, Sec. 6.6) are
 * evaluated on the fly.
 *
 * Layout (paper Sec. 6.1, problem pool): every per-system array is a
 * structure of arrays with leading dimension `ld`; component i of system s
 * is at index i*ld + s.  All array arguments are DEVICE pointers owned by
 * the caller, who keeps them alive until the stream passed to
 * ode_ensemble_solve has completed.  The library never copies them to the
 * host.
 *
 * Errors: every call returns ODE_OK (0) or a negative ode_error code, and
 * then ode_ensemble_last_error() describes the problem (thread-local string).
 * Numerical outcomes of individual systems (NaN at the minimum step, event
 * stop, equilibrium stop, step budget) are NOT call errors: they are written
 * to the per-system status array.
 */
#ifndef ODE_ENSEMBLE_H
#define ODE_ENSEMBLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ODE_MAX_STATE 8
#define ODE_MAX_EVENTS 4
#define ODE_MAX_ACCESSORIES 4
#define ODE_MAX_STEPS_LIMIT 2000000000LL /* largest accepted max_steps */

/* Call results. */
enum ode_error {
  ODE_OK = 0,
  ODE_EINVAL = -1,  /* an argument is invalid (checked before any GPU work) */
  ODE_ENOMEM = -2,  /* a device or host allocation failed                  */
  ODE_EHIP = -3,    /* a HIP runtime call failed                            */
  ODE_ENOTSUP = -4  /* valid request the library does not implement       */
};

/* Built-in models (paper Sec. 2).  Parameters, in order:
 *   DUFFING        2 states, 5 params (k, B, omega, lin, cub):
 *                  y1' = y2, y2' = -lin*y1 - cub*y1^3 - k*y2 + B*cos(omega*t)
 *                  (Sec. 2.1; the paper's double well is lin = -1, cub = 1).
 *   KELLER_MIKSIS  2 states, 13 params C0..C12 of the dimensionless form of
 *                  Sec. 2.2 (time is tau, one period of the first forcing).
 *   RELIEF_VALVE   3 states, 5 params (kappa, delta, beta, q, r), Sec. 2.3;
 *                  r is available to event actions through action_param.
 *   BALLISTIC      2 states, 1 param (g): y1' = y2, y2' = -g (test model).
 *   DUFFING_LYAPUNOV  4 states (y1, y2, r, phi), the DUFFING params: the
 *                  Duffing system with its linearisation attached in polar
 *                  coordinates (Sec. 2.1 Eqs. (3)-(6)); r and phi are the
 *                  length and angle of a tangent vector, with
 *                  g1 = -lin - 3*cub*y1^2 and g2 = -k.  Combined with
 *                  section_period and an ODE_ACC_LOG_RESET accessory on r it
 *                  gives the largest Lyapunov exponent. */
enum ode_model {
  ODE_MODEL_DUFFING = 1,
  ODE_MODEL_KELLER_MIKSIS = 2,
  ODE_MODEL_RELIEF_VALVE = 3,
  ODE_MODEL_BALLISTIC = 4,
  ODE_MODEL_DUFFING_LYAPUNOV = 5
};

/* Integration schemes (paper Sec. 3 and Sec. 6.4). */
enum ode_method { ODE_RKCK45 = 0, ODE_RK4 = 1 };

/* Arithmetic of the integrator.
 *   ODE_FP64         everything in binary64, the paper's arithmetic (Sec. 6.1).
 *   ODE_FP32_STAGES  the right-hand side and the stage sums in binary32; time,
 *                    step size, error norm, state accumulation, accessories and
 *                    event location in binary64.  The FP32 rounding of the
 *                    stage derivatives (~6e-8 relative) sets a noise floor on
 *                    the error estimate and on the result, so it suits
 *                    tolerances of about 1e-7 and looser. */
enum ode_precision { ODE_FP64 = 0, ODE_FP32_STAGES = 1 };

/* Accessory kinds (paper Sec. 5 and Sec. 6.7).  Accessory a occupies rows 2a
 * and 2a+1 of the accessories array.
 *   ODE_ACC_MAX / ODE_ACC_MIN  running maximum / minimum of one state
 *       component over the recording window (row 2a) and the time at which it
 *       was first reached (row 2a+1).
 *   ODE_ACC_LOG_RESET  the Lyapunov accumulator of Sec. 2.1: at every
 *       Poincare section (see section_period) the component is reset to 1,
 *       after ln of its value has been added to row 2a when the section lies
 *       after t_record; row 2a+1 counts the sections added.  The largest
 *       Lyapunov exponent is row 2a / (row 2a+1 * section_period).  Requires
 *       section_period > 0. */
enum ode_accessory_kind { ODE_ACC_MAX = 1, ODE_ACC_MIN = 2, ODE_ACC_LOG_RESET = 3 };

/* Per-system status (low byte) and flags. */
enum ode_lane_status {
  ODE_LANE_DONE = 0,             /* reached t1                                  */
  ODE_LANE_STOP_EVENT = 1,       /* an event reached its stop count (Sec. 6.6)  */
  ODE_LANE_STOP_EQUILIBRIUM = 2, /* max_equilibrium_steps accepted steps inside
                                    an event zone (Sec. 4, configuration d)    */
  ODE_LANE_FAIL_NAN = 3,         /* NaN with the minimum step (Sec. 6.5)        */
  ODE_LANE_MAX_STEPS = 4,        /* max_steps attempts used                     */
  ODE_LANE_BAD_INPUT = 5         /* non-finite t0 or t1, or invalid per-system
                                    tolerances                                */
};
#define ODE_LANE_FLAG_SECANT_CAP 0x100 /* an event location hit its 50-iteration cap */

/* Event j: F_j = y[component] - level (paper Sec. 4: F_Ej(y, t) = 0 with a
 * zone of half width `tolerance` around it; Sec. 6.6 event properties). */
typedef struct {
  int32_t component;        /* state component the event watches            */
  int32_t direction;        /* -1: F decreasing, +1: F increasing, 0: both   */
  int32_t stop_after;       /* stop the system at this detection; 0: never   */
  int32_t action_component; /* -1: no action; else y[c] <- coef * y[c]       */
  int32_t action_param;     /* -1: coef = action_coef; else action_coef*p[i] */
  int32_t record_component; /* -1: none; else store (t, y[c]) of every event
                               inside the window (at most one event records) */
  double level;
  double tolerance;         /* >= 0                                          */
  double action_coef;
} ode_event_spec;

typedef struct {
  int32_t kind;      /* ode_accessory_kind */
  int32_t component;
} ode_accessory_spec;

/* What a handle integrates: the kernel is chosen here (paper Sec. 6.2,
 * solver object; Sec. 6.4, solver choice). */
typedef struct {
  int32_t model;      /* ode_model                                          */
  int32_t method;     /* ode_method                                         */
  int32_t precision;  /* ode_precision                                      */
  int32_t block_size; /* threads per workgroup, multiple of 64 in [64, 256];
                         0 selects the library default                      */
  int32_t blocks_per_cu; /* >= 0: at most this many resident workgroups per
                         compute unit (fewer resident lanes, each taking more
                         systems from the work queue); 0: as many as fit    */
} ode_ensemble_desc;

/* One integration call (paper Sec. 6.4 Solve; Sec. 6.5 ODE properties;
 * Sec. 6.6 event properties; Sec. 6.7 accessories; Sec. 6.8 finalization).
 * All pointers are device pointers; rows are indexed by r*ld + s. */
typedef struct {
  int64_t n_systems;          /* systems to integrate; with system_index this
                                 is its length                              */
  int64_t ld;                 /* leading dimension: ld >= n_systems without
                                 system_index, ld >= 1 with it              */
  double *time_domain;        /* [2][ld] in: (t0, t1); out: row 0 <- final t */
  double *state;              /* [n_state][ld] in: y0; out: final y          */
  const double *params;       /* [n_param][ld], never written                */
  double *accessories;        /* [2*n_accessories][ld] out; NULL iff none    */
  double *next_h;             /* [ld] in: step to start with if > 0 (RKCK45);
                                 out: step to continue with; may be NULL     */
  int32_t *status;            /* [ld] out: ode_lane_status | flags           */
  int64_t *counts;            /* [3][ld] out: accepted, rejected and event-
                                 location attempts; may be NULL             */
  int32_t *event_counts;      /* [n_events][ld] out: detections inside the
                                 recording window; may be NULL              */
  double *event_records;      /* [event_record_capacity][2][ld] out: (t, y[c])
                                 of recorded events in order; detections past
                                 the capacity are counted, not stored; NULL
                                 iff capacity is 0                           */
  const int64_t *system_index;/* [n_systems] systems to integrate (paper
                                 Sec. 6.3 RandomSet); NULL: 0..n_systems-1.
                                 Entries outside [0, ld) are skipped        */
  const double *record_start; /* [ld] per-system start of the recording
                                 window, replacing t_record (so requests with
                                 different windows can share one launch);
                                 NaN: the window never opens; NULL: t_record
                                 for every system                          */
  const double *tolerances;   /* [2*n_state][ld] per-system tolerances
                                 (RKCK45), replacing rtol and atol: rows
                                 0..n_state-1 relative, n_state..2*n_state-1
                                 absolute, per component (so requests with
                                 different tolerances can share one launch).
                                 A system whose entries are not finite and
                                 >= 0 with a positive rtol+atol sum per
                                 component gets ODE_LANE_BAD_INPUT.  NULL:
                                 rtol and atol for every system.  Not part
                                 of the paper, whose tolerances are shared by
                                 all systems of a solver object (Sec. 6.5)  */
  double rtol[ODE_MAX_STATE]; /* per component, >= 0, rtol+atol > 0 (RKCK45) */
  double atol[ODE_MAX_STATE];
  double h0;                  /* initial step (RKCK45) or fixed step (RK4), > 0 */
  double h_min;               /* RKCK45: > 0; at h_min steps are accepted
                                 whatever the error (Sec. 6.5)               */
  double h_max;               /* RKCK45: >= h_min                            */
  double grow;                /* RKCK45: largest step growth, >= 1           */
  double shrink;              /* RKCK45: smallest step factor, in (0, 1]     */
  double t_record;            /* start of the recording window (absolute
                                 time); accessories are initialised from the
                                 state there (Sec. 6.8) and event counts and
                                 records only cover t >= t_record            */
  double section_period;      /* T >= 0, finite.  T > 0: the Poincare sections
                                 t_n = n*T (n integer, counted from time 0)
                                 are forced step boundaries, where
                                 ODE_ACC_LOG_RESET accessories act (Sec. 2.1).
                                 0: no sections                              */
  int64_t max_steps;          /* attempt budget per system, 1..ODE_MAX_STEPS_LIMIT */
  int32_t max_equilibrium_steps; /* >= 0; 0 disables the equilibrium stop   */
  int32_t n_events;           /* 0..ODE_MAX_EVENTS                           */
  int32_t n_accessories;      /* 0..ODE_MAX_ACCESSORIES                      */
  int32_t event_record_capacity; /* >= 0                                     */
  ode_event_spec events[ODE_MAX_EVENTS];
  ode_accessory_spec accessory_specs[ODE_MAX_ACCESSORIES];
} ode_solve_args;

/* Opaque handle: one solver object per (model, method, precision) and device
 * (paper Sec. 6.2).  It owns only its small device work-queue counters. */
typedef struct ode_ensemble ode_ensemble;

/* Launch facts of a handle (for measurement and tuning). */
typedef struct {
  int32_t block_size;         /* threads per workgroup                      */
  int32_t blocks_per_cu;      /* resident workgroups per compute unit       */
  int32_t compute_units;      /* of the handle's device                     */
  int32_t max_grid;           /* workgroups of a full persistent launch     */
  int64_t resident_systems;   /* systems integrated concurrently at most    */
} ode_ensemble_info;

/* Number of states and parameters of a built-in model.  Host only, needs no
 * GPU.  Returns ODE_OK or ODE_EINVAL for an unknown model. */
int ode_ensemble_model_dims(int32_t model, int32_t *n_state, int32_t *n_param);

/* Create a handle for one (model, method, precision) on the current HIP
 * device (paper Sec. 6.2: a solver object per device, created after the
 * device is selected).  Allocates the handle's small device work-queue
 * counters.  *out is set to NULL on failure.  Errors: ODE_EINVAL (NULL
 * arguments, unknown model/method/precision, bad block size), ODE_ENOMEM,
 * ODE_EHIP. */
int ode_ensemble_create(const ode_ensemble_desc *desc, ode_ensemble **out);

/* Enqueue one integration of args->n_systems systems on `hip_stream` (a
 * hipStream_t; NULL is the default stream) and return without waiting.
 * Every system is integrated from its own t0 to t1 (paper Sec. 6.1, each
 * system has its own time domain) and its results are written in place:
 * final state, final time into t0 (so a second call continues, Sec. 6.8),
 * next step, status, counts, accessories, event counts and records.
 * Arguments are validated before anything is enqueued (ODE_EINVAL); a HIP
 * launch failure returns ODE_EHIP.  With n_systems == 0 nothing is read,
 * written or launched, and the array pointers may be NULL.  One handle must not run two solves at
 * the same time; separate handles may run concurrently. */
int ode_ensemble_solve(ode_ensemble *e, const ode_solve_args *args, void *hip_stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * integration as ode_ensemble_create(desc) + ode_ensemble_solve(args) +
 * ode_ensemble_destroy, with the same kernels, arguments, results and errors,
 * but without a handle: the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  The caller passes the inputs and outputs as
 * for ode_ensemble_solve.
 * The work-queue counters live in a static device array of the library (two
 * 64-bit counters, 16 bytes, whatever the problem size; each GPU the library
 * runs on holds its own copy until the process ends).  Its device address is
 * looked up on the first call on each device, with that device current.  Each
 * call clears the counters with a small kernel on hip_stream before the
 * integrator launch (no memset node, so the call can be captured into a graph
 * and replayed).  Every call on one GPU shares that array: calls whose work
 * overlaps on one GPU (e.g. on two streams) race on it and must not be made;
 * calls on one stream are ordered and safe.  Problem sizes are limited as for
 * ode_ensemble_solve (ld <= 2^40).
 * Errors: ODE_EINVAL (as create + solve), ODE_ENOTSUP (device index >= 64),
 * ODE_EHIP. */
int ode_ensemble_solve_noalloc(const ode_ensemble_desc *desc, const ode_solve_args *args,
                               void *hip_stream);

/* Repeated horizons, captured once as a HIP graph.  This is the paper's
 * Sec. 7 workflow: a sweep advanced one excitation period per solve call,
 * each end point starting the next call, with the points of the last calls
 * kept.  The call is equivalent to the host loop
 *     for k = 0 .. n_segments-1:
 *       time_domain[1][s] = time_domain[0][s] + segment    (every system s)
 *       ode_ensemble_solve(e, args, hip_stream)
 *       if k >= first_snapshot: copy rows of system s into snapshot
 *                               k - first_snapshot
 * and its results are bit-identical to it.
 * A snapshot is [n_state + 2*n_accessories][ld]: the state after that
 * segment, then the accessories of that segment.  `snapshots` (device) holds
 * (n_segments - first_snapshot) of them, back to back, and is NULL iff
 * first_snapshot == n_segments.
 * The n_segments x 3 kernel launches are recorded once into a HIP graph on a
 * stream private to the handle.  The graph is kept on the handle and
 * relaunched while the arguments (pointers and values) stay the same.  It
 * contains kernel nodes only.  Each call enqueues one graph launch on
 * hip_stream and returns without waiting.
 * Requires n_segments >= 1, 0 <= first_snapshot <= n_segments and a finite
 * segment > 0; args as for ode_ensemble_solve (its t1 row is overwritten).
 * Errors: ODE_EINVAL, ODE_EHIP, ODE_ENOMEM. */
int ode_ensemble_solve_segments(ode_ensemble *e, const ode_solve_args *args,
                                int32_t n_segments, double segment, int32_t first_snapshot,
                                double *snapshots, void *hip_stream);

/* Result of ode_ensemble_tune. */
typedef struct {
  int32_t block_size;    /* chosen threads per workgroup                    */
  int32_t blocks_per_cu; /* chosen cap on resident workgroups per CU (0: none) */
  int32_t candidates;    /* launch configurations timed                     */
  int32_t reserved;
  double best_ms;        /* probe time of the chosen configuration          */
  double default_ms;     /* probe time of the handle's configuration before */
} ode_tune_result;

/* Autotune the handle's launch configuration for problems like `args` (the
 * paper tunes threads per block by hand, Sec. 7.1 tables; here the library
 * measures).  Every candidate (block sizes 64, 128, 256; all resident
 * workgroups that fit, or half of them) integrates the problem of `args`
 * over the first probe_fraction of each system's time domain, on private
 * copies of every array the solve writes, and is timed with HIP events on
 * hip_stream; the fastest becomes the handle's configuration.  The caller's
 * arrays are only read.  Synchronous: returns after the probes finished.
 * Allocates and frees device memory for the copies (about the size of the
 * caller's arrays).  0 < probe_fraction <= 1.  Errors: ODE_EINVAL,
 * ODE_ENOMEM, ODE_EHIP. */
int ode_ensemble_tune(ode_ensemble *e, const ode_solve_args *args, double probe_fraction,
                      void *hip_stream, ode_tune_result *result);

/* Queue order for a solve, from per-system cost estimates.  The paper's
 * warps run as long as their slowest thread (Sec. 7.1.1, 7.2-7.3); here a
 * SIMD runs as long as the chains of the waves resident on it together, and
 * with every system resident from the start the queue order decides which
 * systems share a SIMD.
 *
 * Host only, no GPU: cost[q] (q < n) estimates the work of queue position q
 * (e.g. its attempted steps over part of the horizon) and queue[q] is the
 * system at position q (NULL: q itself).  The positions are taken in chunks
 * of 64 (one wave), a chunk costing its largest entry, and sorted by cost,
 * most expensive first (ties keep their order).
 *  - If waves * 64 >= n (every position has a lane from the start: wave w of
 *    the launch takes positions 64w .. 64w+63), the sorted chunks are dealt
 *    to the waves in rounds of round_waves (one wave per SIMD across the
 *    chip; a wave's SIMD partners are the waves at the same place in the
 *    other rounds), in alternating direction, so that a SIMD's waves get one
 *    long and one short chunk.  *n_out = waves * 64; positions no chunk
 *    reaches hold -1 (the solve skips negative entries).
 *  - Otherwise the lanes take positions as they free up: the chunks follow
 *    each other in sorted order (longest processing time first), *n_out = n.
 * n == 0 gives *n_out = 0.  out (capacity entries, host) receives the
 * system per position; out NULL only sets *n_out.  Errors: ODE_EINVAL (n < 0, waves or round_waves < 1,
 * cost NULL with n > 0, n_out NULL, capacity < *n_out). */
int ode_plan_order(const int64_t *cost, const int64_t *queue, int64_t n, int64_t waves,
                   int64_t round_waves, int64_t *out, int64_t capacity, int64_t *n_out);

/* Plan the queue order of a solve on this handle (ode_plan_order on measured
 * costs).  A probe integrates the problem of `args` over the first
 * probe_fraction of each system's time domain, with rtol and atol multiplied
 * by probe_tolerance_scale (RKCK45 step counts scale alike across systems, so
 * a looser probe covers more of the horizon for the same work), on private
 * copies of every array the solve writes (the caller's arrays are only read),
 * with the handle's launch configuration; a position's cost is its system's
 * attempted steps in the probe.  waves is the solve's launch size and round_waves is
 * 4 x the device's compute units.  The order is written to index_out (device,
 * capacity int64 entries) and its length to *n_positions; pass index_out as
 * args->system_index and *n_positions as args->n_systems of the solve (same
 * handle, same other arguments).  Each system's results are bit-identical to
 * those of the unplanned solve; only its lane changes.  index_out NULL only
 * sets *n_positions (no probe).  Synchronous.  Allocates and frees device
 * memory for the copies.  0 < probe_fraction <= 1, probe_tolerance_scale >= 1
 * and finite.  Errors: ODE_EINVAL, ODE_ENOMEM, ODE_EHIP. */
int ode_ensemble_plan(ode_ensemble *e, const ode_solve_args *args, double probe_fraction,
                      double probe_tolerance_scale, int64_t *index_out, int64_t capacity,
                      int64_t *n_positions, void *hip_stream);

/* ---- Served queues: continuous admission into a running launch ----
 *
 * Not part of the paper, whose Solve integrates one fixed chunk of systems per
 * launch (Sec. 6.3-6.4).  A served launch is a persistent integrator launch
 * that keeps taking systems while the host appends them, so requests that
 * arrive while others are integrating start on the lanes that free up,
 * without waiting for a launch to end.
 *
 * The caller owns a pool of `ld` slots: the arrays of an ode_solve_args with
 * leading dimension ld (inputs, outputs, and the per-system record_start and
 * tolerances, which let requests with different windows and tolerances share
 * the launch), a position ring (args->system_index, [ld] int64: queue
 * position q holds the system in slot system_index[q % ld]) and
 * request_of_slot ([ld] int32: the request each slot's system belongs to, in
 * [0, max_requests)).  To admit a request of m systems into free slots:
 *   1. copy its inputs into the slots, its request id into request_of_slot
 *      and its slots into the next m ring entries, all on one stream
 *      (`copy_stream`);
 *   2. ode_serve_begin_request(request, m);
 *   3. ode_serve_publish(published + m).
 * A slot, its ring entry and its request id must stay unchanged from step 1
 * until the request's done flag is set.  The flag (ode_serve_done_flags,
 * host memory) turns 1 once every system of the request has been integrated
 * and its results written back to the pool; the caller then copies the
 * results out and may reuse the slots.  Positions are published in order and
 * each is taken once.
 *
 * Every wait of the launch is bounded: a wave with no work polls the
 * published count, sleeping between polls.  It leaves at once when the queue
 * is closed and every published position is taken; otherwise it keeps
 * polling while some taken position is still being integrated (each within
 * its step budget), and leaves after idle_polls empty polls in a row with
 * every published position finished.  So a launch keeps all its waves while
 * any of its work is in flight, and requests published meanwhile start on
 * every idle lane, not only on those of the waves still integrating.  A launch that has left while positions are
 * still unpublished-or-untaken is simply launched again (ode_serve_launch
 * continues from the queue's position).  Results are bit-identical to an
 * ode_ensemble_solve of the same systems: no system's arithmetic depends on
 * its lane, its neighbours or the time it was admitted.
 *
 * Streams: the queue owns a launch stream and a copy stream
 * (ode_serve_stream), each created over every compute unit with a CU mask so
 * that it has a hardware queue of its own.  Streams without one share the
 * device's few hardware queues round-robin, and work on a stream that shares
 * a hardware queue with a running persistent launch waits for that launch
 * to end: an admission copy, a result copy or a relaunch of one served
 * class would then wait for another class's launch.
 *
 * Memory: the queue owns 32 bytes of device counters, max_requests int32
 * device counts, max_requests int32 flags in coherent host memory and its
 * two streams.  One served launch per queue may run at a time. */
typedef struct ode_serve ode_serve;

/* Create a served queue on the current device for up to max_requests
 * request ids (1 .. 2^24).  Errors: ODE_EINVAL, ODE_ENOMEM. */
int ode_serve_create(int32_t max_requests, ode_serve **out);

/* Host pointer to the max_requests done flags (coherent host memory, written
 * by the GPU); NULL for a NULL queue. */
volatile int32_t *ode_serve_done_flags(ode_serve *s);

/* The queue's launch stream (which = 0) or copy stream (which = 1), as a
 * hipStream_t owned by the queue; NULL for a NULL queue or another `which`.
 * Any stream may be passed where the calls below take one; these two have
 * hardware queues of their own (see above). */
void *ode_serve_stream(ode_serve *s, int32_t which);

/* Start a new session: published count, closed flag and queue position to
 * zero, every done flag to 0.  No launch may be running.  Synchronous on
 * copy_stream.  Errors: ODE_EINVAL, ODE_EHIP. */
int ode_serve_reset(ode_serve *s, void *copy_stream);

/* Arm request `request` (in [0, max_requests)) for n_systems >= 1 systems:
 * its done flag to 0 and its device count to n_systems.  Synchronous on
 * copy_stream (so the copies enqueued there before have completed).
 * Errors: ODE_EINVAL, ODE_EHIP. */
int ode_serve_begin_request(ode_serve *s, int32_t request, int32_t n_systems, void *copy_stream);

/* Set the published count to `published` (positions [0, published) may be
 * taken).  Synchronous on copy_stream: everything enqueued there before has
 * completed when the count changes.  Errors: ODE_EINVAL, ODE_EHIP. */
int ode_serve_publish(ode_serve *s, int64_t published, void *copy_stream);

/* Close the queue: running waves leave once every published position is
 * taken.  Synchronous on copy_stream.  Errors: ODE_EINVAL, ODE_EHIP. */
int ode_serve_close(ode_serve *s, void *copy_stream);

/* Enqueue a served launch of handle e on hip_stream over the pool described
 * by args (system_index is the position ring; n_systems is ignored; the other
 * fields as for ode_ensemble_solve, with ld the pool size).  At most
 * max_workgroups workgroups (0: as many as are resident), so several served
 * launches of different models can share the device.  idle_polls >= 1 bounds
 * the idle wait (see above).  Errors: ODE_EINVAL, ODE_EHIP. */
int ode_serve_launch(ode_serve *s, ode_ensemble *e, const ode_solve_args *args,
                     const int32_t *request_of_slot, int32_t max_workgroups, int32_t idle_polls,
                     void *hip_stream);

/* Release the queue's memory and streams (no launch may be running).  NULL
 * is ignored. */
void ode_serve_destroy(ode_serve *s);

/* Launch facts for the handle.  Errors: ODE_EINVAL for NULL arguments. */
int ode_ensemble_query(const ode_ensemble *e, ode_ensemble_info *info);

/* Release the handle, its device memory, its private stream and any cached
 * graph.  NULL is ignored.  The caller must have synchronised every stream
 * the handle was used on. */
void ode_ensemble_destroy(ode_ensemble *e);

/* Description of the last error on the calling thread ("" if none). */
const char *ode_ensemble_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ODE_ENSEMBLE_H */
