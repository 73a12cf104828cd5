/*
 * ode_oracle.c -- plain CPU reference integrator ("the oracle").
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
 * CPU-baseline leg; never by the product path.  It shares no code with the HIP
 * library.
 *
 * It follows the paper (Hegedus, arXiv:1810.03931) step by step for a single
 * system at a time:
 *   - Sec. 3: adaptive Runge-Kutta-Cash-Karp 4(5) and fixed-step RK4;
 *   - Sec. 6.5 (ODE properties): per-component tolerances, step limits,
 *     growth/shrink limits, the minimum-step and NaN rules;
 *   - Sec. 4 (event handling): event zones of half width "tolerance", the
 *     normal / detected / leaving states, secant location when a step jumps
 *     over the zone, largest-index precedence, the equilibrium stop;
 *   - Sec. 6.6: event direction, stop count and the event action (impact law);
 *   - Sec. 5 / 6.7 / 6.8: ordinary accessories (running max / min and time),
 *     initialised from the state, and the final time written back to t0.
 * Readings of points the paper leaves open are marked READING below; every one
 * is listed in the design notes.
 *
 * Arithmetic: binary64, no contraction, glibc libm.
 *
 * Parity unpinned: the step-size controller's decision sequence (READINGS
 * R3/R4/R11: error norm, step factor, the step after a clipped or located
 * step).  The paper prints no formula, so these are readings; the
 * matrix-polynomial replica in the tests restates the same reading (it pins
 * the stage arithmetic and the step counts that reading gives, not the
 * reading).  Only invariants pin the controller from outside: the
 * accepted-step count scales as tol^(-1/5) and the global error with tol.
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Models (paper Sec. 2)                                                     */
/* ------------------------------------------------------------------------ */

int oracle_model_dims(int model, int *n_state, int *n_param) {
  int ns = -1, np = -1;
  switch (model) {
  case OR_MODEL_DUFFING: ns = 2; np = 5; break;
  case OR_MODEL_KELLER_MIKSIS: ns = 2; np = 13; break;
  case OR_MODEL_RELIEF_VALVE: ns = 3; np = 5; break;
  case OR_MODEL_BALLISTIC: ns = 2; np = 1; break;
  case OR_MODEL_DUFFING_LYAPUNOV: ns = 4; np = 5; break;
  default: return -1;
  }
  if (n_state) *n_state = ns;
  if (n_param) *n_param = np;
  return 0;
}

/* Duffing oscillator, paper Sec. 2.1 Eqs. (1)-(2), with the linear and cubic
 * stiffness as parameters (READING R17): the paper's double well has
 * lin = -1 (the +delta*y1 term with delta = 1) and cub = 1; a hardening single
 * well has lin = cub = 1; cub = 0 is the linear driven damped oscillator.
 *   p = (k, B, omega, lin, cub)
 *   y1' = y2
 *   y2' = -lin*y1 - cub*y1^3 - k*y2 + B*cos(omega*t)                        */
static void rhs_duffing(double t, const double *y, const double *p, double *f) {
  double k = p[0], B = p[1], w = p[2], lin = p[3], cub = p[4];
  double y1 = y[0], y2 = y[1];
  f[0] = y2;
  f[1] = -lin * y1 - cub * y1 * y1 * y1 - k * y2 + B * cos(w * t);
}

/* Duffing oscillator with its linearisation attached in polar coordinates
 * (paper Sec. 2.1 Eqs. (3)-(6)): the tangent vector (u, v) = r (cos phi,
 * sin phi) obeys u' = v, v' = g1 u + g2 v with g1 = dF2/dy1 and
 * g2 = dF2/dy2 at the current point, so that
 *   r'   = r ((1 + g1) sin(phi) cos(phi) + g2 sin(phi)^2)
 *   phi' = -sin(phi)^2 + (g1 cos(phi) + g2 sin(phi)) cos(phi).
 * For y2' = -lin*y1 - cub*y1^3 - k*y2 + B*cos(omega*t):
 *   g1 = -lin - 3*cub*y1^2,  g2 = -k.
 * y = (y1, y2, r, phi), p = (k, B, omega, lin, cub).                        */
static void rhs_duffing_lyapunov(double t, const double *y, const double *p, double *f) {
  double k = p[0], lin = p[3], cub = p[4];
  double y1 = y[0], r = y[2], phi = y[3];
  rhs_duffing(t, y, p, f);
  double g1 = -lin - 3.0 * cub * y1 * y1;
  double g2 = -k;
  double s = sin(phi), c = cos(phi);
  f[2] = r * ((1.0 + g1) * s * c + g2 * s * s);
  f[3] = -s * s + (g1 * c + g2 * s) * c;
}

/* Keller-Miksis equation in the paper's dimensionless form, Sec. 2.2
 * (numerator N_KM, denominator D_KM, coefficients C0..C12).  Time is the
 * dimensionless tau (one period of the first forcing component = 1),
 * y1 = R/R_E, y2 = dy1/dtau.                                                */
static void rhs_keller_miksis(double tau, const double *y, const double *C, double *f) {
  const double two_pi = 6.283185307179586476925286766559;
  double y1 = y[0], y2 = y[1];
  double rx = 1.0 / y1;
  double arg1 = two_pi * tau;
  double arg2 = two_pi * C[11] * tau + C[12];
  double N = (C[0] + C[1] * y2) * pow(rx, C[10])
           - C[2] * (1.0 + C[9] * y2)
           - C[3] * rx
           - C[4] * y2 * rx
           - (1.0 - C[9] * y2 / 3.0) * 1.5 * y2 * y2
           - (C[5] * sin(arg1) + C[6] * sin(arg2)) * (1.0 + C[9] * y2)
           - y1 * (C[7] * cos(arg1) + C[8] * cos(arg2));
  double D = y1 - C[9] * y1 * y2 + C[4] * C[9];
  f[0] = y2;
  f[1] = N / D;
}

/* Pressure relief valve, paper Sec. 2.3 Eqs. (29)-(31).
 *   p = (kappa, delta, beta, q, r); r is only used by the impact action.    */
static void rhs_relief_valve(double t, const double *y, const double *p, double *f) {
  (void)t;
  double kappa = p[0], delta = p[1], beta = p[2], q = p[3];
  f[0] = y[1];
  f[1] = -kappa * y[1] - (y[0] + delta) + y[2];
  f[2] = beta * (q - y[0] * sqrt(y[2]));
}

/* Free flight under constant gravity (test model): y1' = y2, y2' = -g.      */
static void rhs_ballistic(double t, const double *y, const double *p, double *f) {
  (void)t;
  f[0] = y[1];
  f[1] = -p[0];
}

int oracle_rhs(int model, double t, const double *y, const double *p, double *f) {
  switch (model) {
  case OR_MODEL_DUFFING: rhs_duffing(t, y, p, f); return 0;
  case OR_MODEL_KELLER_MIKSIS: rhs_keller_miksis(t, y, p, f); return 0;
  case OR_MODEL_RELIEF_VALVE: rhs_relief_valve(t, y, p, f); return 0;
  case OR_MODEL_BALLISTIC: rhs_ballistic(t, y, p, f); return 0;
  case OR_MODEL_DUFFING_LYAPUNOV: rhs_duffing_lyapunov(t, y, p, f); return 0;
  default: return -1;
  }
}

/* ------------------------------------------------------------------------ */
/* Integration schemes (paper Sec. 3)                                        */
/* ------------------------------------------------------------------------ */

/* Cash-Karp embedded 4(5) pair (READING R1: the paper names the method but
 * prints no coefficients; these are Cash & Karp's published values).  The
 * fifth-order solution is propagated (READING R2) and the difference to the
 * embedded fourth-order one is the local error estimate.                    */
static const double CK_C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
static const double CK_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0, 0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0, 0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0, 0}};
static const double CK_B[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
static const double CK_BSTAR[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0,
                                   13525.0 / 55296.0, 277.0 / 14336.0, 1.0 / 4.0};


/* Error weights e = b - b* (exact rationals), so that the error estimate
 * y5 - y4 = h * sum_i e_i k_i is formed without subtracting two nearly equal
 * solutions. */
static const double CK_E[6] = {-277.0 / 64512.0, 0.0, 6925.0 / 370944.0,
                               -6925.0 / 202752.0, -277.0 / 14336.0, 277.0 / 7084.0};

void oracle_cash_karp_tableau(double *c, double *a, double *b, double *bstar, double *e) {
  for (int i = 0; i < 6; ++i) {
    c[i] = CK_C[i];
    b[i] = CK_B[i];
    bstar[i] = CK_BSTAR[i];
    e[i] = CK_E[i];
    for (int j = 0; j < 6; ++j) a[i * 6 + j] = CK_A[i][j];
  }
}

/* One Cash-Karp step of length h from (t, y).  Stages whose weight is zero
 * do not enter the sums. */
static void cash_karp_step(int model, int n, double t, const double *y, const double *p,
                           double h, double *y5, double *err) {
  double k[6][OR_MAX_STATE];
  double ys[OR_MAX_STATE];
  for (int s = 0; s < 6; ++s) {
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < s; ++j) acc += CK_A[s][j] * k[j][i];
      ys[i] = y[i] + h * acc;
    }
    oracle_rhs(model, t + CK_C[s] * h, ys, p, k[s]);
  }
  for (int i = 0; i < n; ++i) {
    double s5 = 0.0, se = 0.0;
    for (int j = 0; j < 6; ++j) {
      if (CK_B[j] != 0.0) s5 += CK_B[j] * k[j][i];
      if (CK_E[j] != 0.0) se += CK_E[j] * k[j][i];
    }
    y5[i] = y[i] + h * s5;
    err[i] = h * se;
  }
}

/* One classical fourth-order Runge-Kutta step of length h from (t, y). */
static void rk4_step(int model, int n, double t, const double *y, const double *p, double h,
                     double *y_new) {
  double k1[OR_MAX_STATE], k2[OR_MAX_STATE], k3[OR_MAX_STATE], k4[OR_MAX_STATE];
  double ys[OR_MAX_STATE];
  oracle_rhs(model, t, y, p, k1);
  for (int i = 0; i < n; ++i) ys[i] = y[i] + 0.5 * h * k1[i];
  oracle_rhs(model, t + 0.5 * h, ys, p, k2);
  for (int i = 0; i < n; ++i) ys[i] = y[i] + 0.5 * h * k2[i];
  oracle_rhs(model, t + 0.5 * h, ys, p, k3);
  for (int i = 0; i < n; ++i) ys[i] = y[i] + h * k3[i];
  oracle_rhs(model, t + h, ys, p, k4);
  for (int i = 0; i < n; ++i)
    y_new[i] = y[i] + h * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]) / 6.0;
}

int oracle_step(int model, int method, double t, const double *y, const double *p, double h,
                double *y_new, double *err) {
  int n;
  if (oracle_model_dims(model, &n, NULL) != 0) return -1;
  if (method == OR_RKCK45) {
    double e[OR_MAX_STATE];
    cash_karp_step(model, n, t, y, p, h, y_new, e);
    if (err)
      for (int i = 0; i < n; ++i) err[i] = e[i];
    return 0;
  }
  if (method == OR_RK4) {
    rk4_step(model, n, t, y, p, h, y_new);
    return 0;
  }
  return -1;
}

/* A full step of the selected method (the secant iterates are full steps of
 * a shortened length from the same starting point). */
static void method_step(const or_options *o, int n, double t, const double *y, const double *p,
                        double h, double *y_new, double *err) {
  if (o->method == OR_RKCK45)
    cash_karp_step(o->model, n, t, y, p, h, y_new, err);
  else
    rk4_step(o->model, n, t, y, p, h, y_new);
}

/* ------------------------------------------------------------------------ */
/* Event handling (paper Sec. 4 and Sec. 6.6)                                */
/* ------------------------------------------------------------------------ */

enum { EV_NORMAL = 0, EV_LEAVING = 1 };
enum { DET_NONE = 0, DET_CROSSING = 1, DET_LANDING = 2 };

static double event_value(const or_event *e, const double *y) {
  return y[e->component] - e->level;
}

/* Detection from the previous accepted point (value Fo, outside the zone) to
 * the candidate point (value Fn).  READING R8: direction -1 means F
 * decreasing (a local maximum when F is the velocity), +1 increasing, 0 both.
 * READING R9: configuration "a" of the paper's figure is a crossing (the step
 * jumps over the zone); the others end inside the zone (landing).           */
static int detect(double Fo, double Fn, int dir, double tol) {
  if (dir <= 0 && Fo > tol) {
    if (Fn < -tol) return DET_CROSSING;
    if (fabs(Fn) <= tol) return DET_LANDING;
  }
  if (dir >= 0 && Fo < -tol) {
    if (Fn > tol) return DET_CROSSING;
    if (fabs(Fn) <= tol) return DET_LANDING;
  }
  return DET_NONE;
}

/* ------------------------------------------------------------------------ */
/* One system                                                               */
/* ------------------------------------------------------------------------ */

#define SECANT_MAX_ITER 50

typedef struct {
  double t, y[OR_MAX_STATE];
  double accv[OR_MAX_ACC], acct[OR_MAX_ACC];
  int window_open;
} sys_view;

static void accessories_init(const or_options *o, double t, const double *y, double *accv,
                             double *acct) {
  for (int a = 0; a < o->n_acc; ++a) {
    if (o->acc[a].kind == OR_ACC_LOG_RESET) {
      accv[a] = 0.0; /* sum of logarithms */
      acct[a] = 0.0; /* number of sections */
    } else {
      accv[a] = y[o->acc[a].component];
      acct[a] = t;
    }
  }
}

/* Ordinary accessories (paper Sec. 6.7): strict comparison, so the first
 * point that reaches an extreme keeps it (READING R16). */
static void accessories_update(const or_options *o, double t, const double *y, double *accv,
                               double *acct) {
  for (int a = 0; a < o->n_acc; ++a) {
    if (o->acc[a].kind == OR_ACC_LOG_RESET) continue; /* acts at sections only */
    double v = y[o->acc[a].component];
    if (o->acc[a].kind == OR_ACC_MAX ? (v > accv[a]) : (v < accv[a])) {
      accv[a] = v;
      acct[a] = t;
    }
  }
}

static void solve_one(const or_options *o, int n, long long s, long long ld, double *time_domain,
                      double *state, const double *params, double *acc_out, double *next_h,
                      int *status_out, long long *counts, int *event_counts,
                      double *event_records) {
  const int ne = o->n_events;
  double p[OR_MAX_PARAM];
  int np;
  oracle_model_dims(o->model, NULL, &np);
  for (int j = 0; j < np; ++j) p[j] = params[(long long)j * ld + s];

  /* Tolerances (paper Sec. 6.5).  A serving extension, not in the paper:
   * each system may carry its own, so that requests with different
   * tolerances share one solve; each system is still the paper's problem. */
  double rtol[OR_MAX_STATE], atol[OR_MAX_STATE];
  int tol_ok = 1;
  for (int i = 0; i < n; ++i) {
    rtol[i] = o->tolerances ? o->tolerances[(long long)i * ld + s] : o->rtol[i];
    atol[i] = o->tolerances ? o->tolerances[(long long)(n + i) * ld + s] : o->atol[i];
    if (o->tolerances && o->method == OR_RKCK45 &&
        !(rtol[i] >= 0.0 && atol[i] >= 0.0 && rtol[i] + atol[i] > 0.0 &&
          isfinite(rtol[i] + atol[i])))
      tol_ok = 0;
  }

  double t0 = time_domain[s], t1 = time_domain[ld + s];
  double t = t0;
  /* start of this system's recording window */
  const double t_rec = o->record_start ? o->record_start[s] : o->t_record;
  double y[OR_MAX_STATE];
  for (int i = 0; i < n; ++i) y[i] = state[(long long)i * ld + s];

  /* Initial step: no prediction (paper Sec. 6.4); a positive next_h from a
   * previous solve resumes the controller. */
  double h = o->h0;
  if (o->method == OR_RKCK45) {
    if (next_h && next_h[s] > 0.0 && isfinite(next_h[s])) h = next_h[s];
    if (h > o->h_max) h = o->h_max;
    if (h < o->h_min) h = o->h_min;
  }

  /* Every attempted step is either committed (n_acc), rejected by the error
   * test (n_rej) or spent on event location (the full step that jumped over
   * a zone and the secant iterates that missed it). */
  long long n_acc = 0, n_rej = 0, attempts = 0;
  int status = -1; /* running */
  int flags = 0;

  /* RK4 grid: the state after m steps of a segment sits at seg_start + m*dt
   * (READING R25); a segment restarts at every forced boundary and located
   * event. */
  double seg_start = t;
  long long seg_steps = 0;

  /* Events: initial point inside a zone is not detected (paper Sec. 7.2). */
  double F[OR_MAX_EVENTS];
  int evstate[OR_MAX_EVENTS], zone[OR_MAX_EVENTS];
  long long count[OR_MAX_EVENTS], wcount[OR_MAX_EVENTS];
  for (int j = 0; j < ne; ++j) {
    F[j] = event_value(&o->ev[j], y);
    evstate[j] = fabs(F[j]) <= o->ev[j].tolerance ? EV_LEAVING : EV_NORMAL;
    zone[j] = 0;
    count[j] = 0;
    wcount[j] = 0;
  }
  long long n_records = 0;

  double accv[OR_MAX_ACC], acct[OR_MAX_ACC];
  int window_open = 0;

  if (!isfinite(t0) || !isfinite(t1) || !tol_ok) status = OR_BAD_INPUT;

  /* Poincare sections (paper Sec. 2.1: t_n = n*T).  READING R29: n counts
   * from the origin of time, not from t0, so a solve split in two visits the
   * same sections; the next section is the first n*T (rounded product)
   * strictly after t0, and every section is a forced step boundary. */
  const double T = o->section_period;
  long long sec_n = 0;
  double t_sec = INFINITY;
  if (status < 0 && T > 0.0) {
    sec_n = (long long)floor(t0 / T) + 1;
    t_sec = (double)sec_n * T;
    while (t_sec <= t0) {
      sec_n++;
      t_sec = (double)sec_n * T;
    }
  }

  /* Accessory initialisation (paper Sec. 6.8) at the start of the window. */
  if (status < 0 && t_rec <= t0) {
    window_open = 1;
    accessories_init(o, t, y, accv, acct);
  }

  while (status < 0) {
    if (t >= t1) {
      status = OR_DONE;
      break;
    }
    if (attempts >= o->max_steps) {
      status = OR_MAX_STEPS;
      break;
    }
    /* The next forced boundary: the start of the recording window, then t1
     * (READING R7: steps are clipped so that t lands exactly on it). */
    double t_b = (!window_open && t_rec < t1) ? t_rec : t1;
    if (t_sec < t_b) t_b = t_sec;

    double h_try;
    int clipped = 0;
    if (o->method == OR_RK4) {
      double t_grid = seg_start + (double)(seg_steps + 1) * o->h0;
      if (t_grid >= t_b - 1e-9 * o->h0) {
        h_try = t_b - t;
        clipped = 1;
      } else {
        h_try = o->h0;
      }
    } else {
      h_try = h;
      if (h_try >= t_b - t) {
        h_try = t_b - t;
        clipped = 1;
      }
    }

    double yn[OR_MAX_STATE], err[OR_MAX_STATE];
    method_step(o, n, t, y, p, h_try, yn, err);
    attempts++;

    /* Error control (paper Sec. 6.5). */
    double h_next = h;
    if (o->method == OR_RKCK45) {
      /* READING R3: scaled max norm,
       *   E = max_i |err_i| / (atol_i + rtol_i * max(|y_i|, |y5_i|)). */
      int has_nan = 0;
      double E = 0.0;
      for (int i = 0; i < n; ++i) {
        if (isnan(yn[i])) has_nan = 1;
        double sc = atol[i] + rtol[i] * fmax(fabs(y[i]), fabs(yn[i]));
        double r = fabs(err[i]) / sc;
        if (isnan(r)) has_nan = 1;
        if (r > E) E = r;
      }
      if (has_nan) {
        /* NaN: reject and shrink; with the minimum step, stop (paper Sec. 6.5). */
        if (h_try <= o->h_min) {
          status = OR_FAIL_NAN;
          break;
        }
        h = fmax(o->h_min, o->shrink * h_try);
        n_rej++;
        continue;
      }
      /* READING R4: factor 0.9*E^(-1/5) limited to [shrink, grow]. */
      double fac = (E == 0.0) ? o->grow : 0.9 * pow(E, -0.2);
      if (fac > o->grow) fac = o->grow;
      if (fac < o->shrink) fac = o->shrink;
      h_next = fac * h_try;
      if (h_next > o->h_max) h_next = o->h_max;
      if (h_next < o->h_min) h_next = o->h_min;
      /* READING R5: at (or below) the minimum step the step is accepted
       * whatever the error (paper Sec. 6.5). */
      if (!(E <= 1.0) && h_try > o->h_min) {
        h = h_next;
        n_rej++;
        continue;
      }
    }

    /* The step passed the error test: event detection (paper Sec. 4). */
    double tn;
    int located = 0;
    int det[OR_MAX_EVENTS];
    int J = -1;
    for (int j = 0; j < ne; ++j) {
      det[j] = DET_NONE;
      if (evstate[j] != EV_NORMAL) continue;
      det[j] = detect(F[j], event_value(&o->ev[j], yn), o->ev[j].direction,
                      o->ev[j].tolerance);
      if (det[j] != DET_NONE) J = j; /* largest index wins (paper Sec. 4) */
    }

    if (J >= 0 && det[J] == DET_CROSSING) {
      /* READING R10: locate a point inside the zone of event J with a secant
       * iteration on the step length s, g(s) = F_J(step(t, y, s)), safeguarded
       * by the bracket [lo, hi] that keeps the sign change; an iterate outside
       * the bracket is replaced by its midpoint. */
      const or_event *e = &o->ev[J];
      double tol = e->tolerance;
      double lo = 0.0, glo = F[J], hi = h_try, ghi = event_value(e, yn);
      double sa = lo, ga = glo, sb = hi, gb = ghi;
      double sc = hi, yc[OR_MAX_STATE], errc[OR_MAX_STATE];
      int found = 0;
      for (int it = 0; it < SECANT_MAX_ITER; ++it) {
        sc = sb - gb * (sb - sa) / (gb - ga);
        if (!(sc > lo && sc < hi)) sc = 0.5 * (lo + hi);
        method_step(o, n, t, y, p, sc, yc, errc);
        attempts++;
        double gc = event_value(e, yc);
        if (fabs(gc) <= tol) {
          found = 1;
          break;
        }
        if ((gc > 0.0) == (glo > 0.0)) {
          lo = sc;
          glo = gc;
        } else {
          hi = sc;
          ghi = gc;
        }
        sa = sb;
        ga = gb;
        sb = sc;
        gb = gc;
      }
      if (!found) flags |= OR_FLAG_SECANT_CAP; /* keep the last iterate */
      for (int i = 0; i < n; ++i) yn[i] = yc[i];
      tn = t + sc;
      located = 1;
      /* The other events are judged again over the shortened step
       * (READING R12). */
      for (int j = 0; j < ne; ++j) {
        if (j == J) continue;
        det[j] = DET_NONE;
        if (evstate[j] != EV_NORMAL) continue;
        det[j] = detect(F[j], event_value(&o->ev[j], yn), o->ev[j].direction,
                        o->ev[j].tolerance);
      }
      det[J] = DET_CROSSING;
    } else if (clipped) {
      tn = t_b;
    } else if (o->method == OR_RK4) {
      tn = seg_start + (double)(seg_steps + 1) * o->h0;
    } else {
      tn = t + h_try;
    }

    /* Commit the accepted point. */
    t = tn;
    for (int i = 0; i < n; ++i) y[i] = yn[i];
    n_acc++;
    if (o->method == OR_RK4) {
      if (located || clipped) {
        seg_start = t;
        seg_steps = 0;
      } else {
        seg_steps++;
      }
    } else {
      /* READING R11: after a location the controller's proposal from the
       * full step is kept; after a step clipped to a boundary the next step
       * is not made shorter than the step in use before the clip. */
      if (clipped && !located && h_next < h) h_next = h;
      h = h_next;
    }

    /* Ordinary accessories, called after every accepted step (paper Sec. 6.7),
     * inside the recording window; the window opens at the forced boundary
     * t_record where the accessories are initialised from the state. */
    if (!window_open) {
      if (t >= t_rec) {
        window_open = 1;
        accessories_init(o, t, y, accv, acct);
      }
    } else {
      accessories_update(o, t, y, accv, acct);
    }

    /* Event hooks in increasing event index (READING R14): counter (1-based,
     * READING R13), in-window count and record, action, stop check. */
    for (int j = 0; j < ne; ++j) {
      if (det[j] == DET_NONE) continue;
      const or_event *e = &o->ev[j];
      count[j]++;
      if (window_open) {
        wcount[j]++;
        if (e->record_component >= 0) {
          if (n_records < o->record_cap && event_records) {
            long long slot = n_records;
            event_records[(slot * 2 + 0) * ld + s] = t;
            event_records[(slot * 2 + 1) * ld + s] = y[e->record_component];
          }
          n_records++;
        }
      }
      if (e->action_component >= 0) {
        /* Event action, e.g. the impact law y2 <- -r*y2 (paper Sec. 2.3 and
         * the action function of Sec. 6.6). */
        double coef = e->action_coef;
        if (e->action_param >= 0) coef = e->action_coef * p[e->action_param];
        y[e->action_component] = coef * y[e->action_component];
      }
      if (e->stop_after > 0 && count[j] == e->stop_after) status = OR_STOP_EVENT;
    }

    /* Poincare section reached (the step was clipped to it, so t equals the
     * section time exactly): the Lyapunov accumulators add ln y[c] if the
     * section lies after the window start, and y[c] restarts from 1 (paper
     * Sec. 2.1; READING R30: the logarithm of the reset component, averaged
     * per unit time by the caller as sum / (count * T)). */
    if (t == t_sec) {
      for (int a = 0; a < o->n_acc; ++a) {
        if (o->acc[a].kind != OR_ACC_LOG_RESET) continue;
        int c = o->acc[a].component;
        if (window_open && t > t_rec) {
          accv[a] = accv[a] + log(y[c]);
          acct[a] = acct[a] + 1.0;
        }
        y[c] = 1.0;
      }
      sec_n++;
      t_sec = (double)sec_n * T;
    }

    /* Event states after the step: a system is in the normal state for event
     * j exactly when it is outside that event's zone; while it stays inside,
     * the accepted steps are counted for the equilibrium stop (paper Sec. 4,
     * configuration d, and Sec. 6.6). */
    for (int j = 0; j < ne; ++j) {
      F[j] = event_value(&o->ev[j], y);
      int inside = fabs(F[j]) <= o->ev[j].tolerance;
      if (det[j] != DET_NONE || evstate[j] == EV_NORMAL) {
        evstate[j] = inside ? EV_LEAVING : EV_NORMAL;
        zone[j] = 0;
      } else if (inside) {
        zone[j]++;
        if (o->max_equilibrium_steps > 0 && zone[j] >= o->max_equilibrium_steps &&
            status < 0)
          status = OR_STOP_EQUILIBRIUM;
      } else {
        evstate[j] = EV_NORMAL;
        zone[j] = 0;
      }
    }
  }

  /* If the window never opened, the accessories describe the final point. */
  if (!window_open) accessories_init(o, t, y, accv, acct);

  /* Finalisation (paper Sec. 6.8): the final time replaces t0 so that a new
   * solve continues from here. */
  time_domain[s] = t;
  for (int i = 0; i < n; ++i) state[(long long)i * ld + s] = y[i];
  if (next_h) next_h[s] = h;
  status_out[s] = status | flags;
  if (counts) {
    counts[s] = n_acc;
    counts[ld + s] = n_rej;
    counts[2 * ld + s] = attempts - n_acc - n_rej;
  }
  if (acc_out)
    for (int a = 0; a < o->n_acc; ++a) {
      acc_out[(long long)(2 * a) * ld + s] = accv[a];
      acc_out[(long long)(2 * a + 1) * ld + s] = acct[a];
    }
  if (event_counts)
    for (int j = 0; j < ne; ++j) event_counts[(long long)j * ld + s] = (int)wcount[j];
}

static int options_ok(const or_options *o, int *n_state) {
  int ns, np;
  if (oracle_model_dims(o->model, &ns, &np) != 0) return 0;
  if (o->method != OR_RKCK45 && o->method != OR_RK4) return 0;
  if (!(o->h0 > 0.0)) return 0;
  if (o->method == OR_RKCK45) {
    if (!(o->h_min > 0.0) || !(o->h_max >= o->h_min)) return 0;
    if (!(o->grow >= 1.0) || !(o->shrink > 0.0 && o->shrink <= 1.0)) return 0;
    for (int i = 0; i < ns; ++i)
      if (!(o->rtol[i] >= 0.0) || !(o->atol[i] >= 0.0) || !(o->rtol[i] + o->atol[i] > 0.0))
        return 0;
  }
  if (o->max_steps <= 0) return 0;
  if (!(o->section_period >= 0.0) || !isfinite(o->section_period)) return 0;
  if (o->n_events < 0 || o->n_events > OR_MAX_EVENTS) return 0;
  if (o->n_acc < 0 || o->n_acc > OR_MAX_ACC) return 0;
  if (o->record_cap < 0) return 0;
  int n_rec = 0;
  for (int j = 0; j < o->n_events; ++j) {
    const or_event *e = &o->ev[j];
    if (e->component < 0 || e->component >= ns) return 0;
    if (e->direction < -1 || e->direction > 1) return 0;
    if (!(e->tolerance >= 0.0)) return 0;
    if (e->stop_after < 0) return 0;
    if (e->action_component >= ns) return 0;
    if (e->action_param >= np) return 0;
    if (e->record_component >= ns) return 0;
    if (e->record_component >= 0) n_rec++;
  }
  if (n_rec > 1) return 0;
  for (int a = 0; a < o->n_acc; ++a) {
    if (o->acc[a].kind != OR_ACC_MAX && o->acc[a].kind != OR_ACC_MIN &&
        o->acc[a].kind != OR_ACC_LOG_RESET)
      return 0;
    if (o->acc[a].kind == OR_ACC_LOG_RESET && !(o->section_period > 0.0)) return 0;
    if (o->acc[a].component < 0 || o->acc[a].component >= ns) return 0;
  }
  *n_state = ns;
  return 1;
}

int oracle_solve_batch(const or_options *opt, long long n, long long ld, double *time_domain,
                       double *state, const double *params, double *acc, double *next_h,
                       int *status, long long *counts, int *event_counts, double *event_records,
                       const long long *index, int threads) {
  int ns;
  if (!opt || n < 0 || ld < n || !options_ok(opt, &ns)) return -1;
  if (!time_domain || !state || !params || !status) return -1;
  if (opt->n_acc > 0 && !acc) return -1;
#ifdef _OPENMP
  int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
#else
  (void)threads;
#endif
  for (long long q = 0; q < n; ++q) {
    long long s = index ? index[q] : q;
    if (s < 0 || s >= ld) continue;
    solve_one(opt, ns, s, ld, time_domain, state, params, acc, next_h, status, counts,
              event_counts, event_records);
  }
  return 0;
}
