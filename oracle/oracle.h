/*
 * oracle.h -- plain, slow CPU reference for ensemble ODE integration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call anything under oracle/.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg use it.  It shares no code, header, table
 * or constant with the HIP library: every coefficient and every rule below is
 * typed here a second time, from the paper (Hegedus, "Modular, general purpose
 * ODE integration package to solve large number of independent ODE systems on
 * GPUs", arXiv:1810.03931).
 *
 * Arithmetic: IEEE binary64, round to nearest, no contraction (compiled with
 * -ffp-contract=off), glibc libm for cos/sin/pow/sqrt.
 *
 * Layout (paper Sec. 6.1, problem pool): every per-system array is
 * structure-of-arrays with leading dimension ld; component i of system s sits
 * at [i*ld + s].
 */
#ifndef ODE_ORACLE_H
#define ODE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_STATE 8
#define OR_MAX_PARAM 16
#define OR_MAX_EVENTS 4
#define OR_MAX_ACC 4

/* Models (paper Sec. 2; ballistic flight is a test-only model). */
enum {
  OR_MODEL_DUFFING = 1,          /* 2 states, params (k, B, omega, lin, cub)   */
  OR_MODEL_KELLER_MIKSIS = 2,    /* 2 states, params C0..C12                   */
  OR_MODEL_RELIEF_VALVE = 3,     /* 3 states, params (kappa, delta, beta, q, r) */
  OR_MODEL_BALLISTIC = 4,        /* 2 states, params (g)                        */
  OR_MODEL_DUFFING_LYAPUNOV = 5  /* 4 states (y1, y2, r, phi), Duffing's params */
};

/* Integration schemes (paper Sec. 3). */
enum { OR_RKCK45 = 0, OR_RK4 = 1 };

/* Accessory kinds (paper Sec. 5): running extreme of a component + its time;
 * OR_ACC_LOG_RESET is the Lyapunov-exponent accumulator of paper Sec. 2.1:
 * at every Poincare section t_n the component is reset to 1 after its
 * logarithm has been added to the first slot; the second slot counts the
 * sections added.  Both start at 0 when the recording window opens, and only
 * sections after the window start are added (the reset happens at all). */
enum { OR_ACC_MAX = 1, OR_ACC_MIN = 2, OR_ACC_LOG_RESET = 3 };

/* Per-system outcome. */
enum {
  OR_DONE = 0,             /* reached t1                                   */
  OR_STOP_EVENT = 1,       /* an event reached its stop count              */
  OR_STOP_EQUILIBRIUM = 2, /* too many accepted steps inside an event zone */
  OR_FAIL_NAN = 3,         /* NaN with the minimum step                    */
  OR_MAX_STEPS = 4,        /* attempt budget exhausted                     */
  OR_BAD_INPUT = 5         /* non-finite time domain                       */
};
#define OR_FLAG_SECANT_CAP 0x100 /* a secant location hit its iteration cap */

typedef struct {
  int component;        /* F = y[component] - level                         */
  double level;
  int direction;        /* -1: F decreasing, +1: F increasing, 0: both      */
  double tolerance;     /* half width of the event zone, in units of F      */
  int stop_after;       /* stop when this event's count reaches it; 0 never */
  int action_component; /* -1 none; else y[c] <- coef * y[c] at the event   */
  double action_coef;
  int action_param;     /* -1: coef = action_coef; else action_coef*p[idx]  */
  int record_component; /* -1 none; else store (t, y[c]) per in-window event */
} or_event;

typedef struct {
  int kind;      /* OR_ACC_MAX or OR_ACC_MIN */
  int component;
} or_accessory;

typedef struct {
  int model;
  int method;
  double rtol[OR_MAX_STATE];
  double atol[OR_MAX_STATE];
  double h0;        /* initial step (RKCK45) or the fixed step (RK4)        */
  double h_min;
  double h_max;
  double grow;      /* largest step growth factor after an accepted step   */
  double shrink;    /* smallest step factor after a rejected step          */
  double t_record;  /* start of the recording window (absolute time)       */
  double section_period; /* > 0: Poincare sections at t_n = n*T (absolute,
                          * n integer) are forced step boundaries; 0: none */
  const double *record_start; /* [ld] per-system window start replacing
                               * t_record; NULL: t_record for every system */
  const double *tolerances;   /* [2*n_state][ld] per-system relative (rows
                               * 0..n_state-1) and absolute tolerances
                               * replacing rtol/atol; NULL: rtol/atol      */
  int max_equilibrium_steps; /* 0 disables the equilibrium stop            */
  long long max_steps;       /* attempt budget per system                  */
  int n_events;
  int n_acc;
  int record_cap;
  or_event ev[OR_MAX_EVENTS];
  or_accessory acc[OR_MAX_ACC];
} or_options;

/* Number of states / parameters of a model, or -1 if unknown. */
int oracle_model_dims(int model, int *n_state, int *n_param);

/* Right-hand side f(t, y; p) of one system (paper Eq. (38) general form). */
int oracle_rhs(int model, double t, const double *y, const double *p, double *dydt);

/* One step of length h from (t, y): Cash-Karp gives the propagated 5th-order
 * solution in y_new and the embedded error estimate in err; RK4 leaves err
 * untouched. */
int oracle_step(int model, int method, double t, const double *y,
                const double *p, double h, double *y_new, double *err);

/* Butcher tableau exactly as the oracle uses it (for the order-condition
 * pins).  c[6], a[6][6] (row-major, lower triangle), b[6], bstar[6] and the
 * error weights e[6] = b - bstar. */
void oracle_cash_karp_tableau(double *c, double *a, double *b, double *bstar, double *e);

/*
 * Integrate n systems.  Arrays (row*ld + s):
 *   time_domain [2][ld]   in: t0, t1       out: row 0 <- final t
 *   state       [n_state][ld]  in: y0      out: final y
 *   params      [n_param][ld]
 *   acc         [2*n_acc][ld]  out: (value, time) per accessory; may be NULL if n_acc == 0
 *   next_h      [ld]  in: initial step if > 0 (RKCK45), out: next step; may be NULL
 *   status      [ld]  out
 *   counts      [3][ld] out: accepted, rejected, location attempts; may be NULL
 *   event_counts[n_events][ld] out: in-window detections; may be NULL
 *   event_records [record_cap][2][ld] out: (t, y[c]) per recorded event; may be NULL
 *   index       [n] optional list of systems to integrate (NULL: 0..n-1)
 * threads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad options.
 */
int oracle_solve_batch(const or_options *opt, long long n, long long ld,
                       double *time_domain, double *state, const double *params,
                       double *acc, double *next_h, int *status, long long *counts,
                       int *event_counts, double *event_records,
                       const long long *index, int threads);

#ifdef __cplusplus
}
#endif
#endif
