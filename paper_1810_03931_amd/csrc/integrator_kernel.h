// Persistent ensemble integrator kernel (paper: Hegedus, arXiv:1810.03931).
//
// One lane integrates one system at a time with its state in registers.  A
// wave pulls system indices from a device-wide queue: whenever some of its
// lanes are idle it claims that many indices with one atomic (ballot +
// popcount), hands them out by lane rank (mbcnt), and the wave leaves only
// when the queue is empty and all its lanes are idle.  Systems that finish
// early -- short horizons, event or equilibrium stops, NaN stops -- are thus
// replaced at once instead of idling until the slowest lane of the wave is
// done (the paper attributes its lower utilisation to exactly this
// divergence, Sec. 7.1.1 and Sec. 7.2-7.3).
//
// Every loop iteration performs exactly one Runge-Kutta attempt per busy
// lane: a normal step, a step the error test rejects, or one secant iterate
// of an event location.  Lanes in different phases therefore still execute
// the expensive stage evaluations together; only the cheap bookkeeping after
// the attempt diverges.
#pragma once

#include "integrator.h"
#include "model_common.h"

namespace odeens {

// Cash-Karp 4(5) coefficients (Cash & Karp 1990; the paper names the
// method in Sec. 3 without printing them).  e = b - b* are the error weights.
namespace ck {
constexpr double c2 = 1.0 / 5.0, c3 = 3.0 / 10.0, c4 = 3.0 / 5.0, c6 = 7.0 / 8.0;
constexpr double a21 = 1.0 / 5.0;
constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
constexpr double a41 = 3.0 / 10.0, a42 = -9.0 / 10.0, a43 = 6.0 / 5.0;
constexpr double a51 = -11.0 / 54.0, a52 = 5.0 / 2.0, a53 = -70.0 / 27.0, a54 = 35.0 / 27.0;
constexpr double a61 = 1631.0 / 55296.0, a62 = 175.0 / 512.0, a63 = 575.0 / 13824.0,
                 a64 = 44275.0 / 110592.0, a65 = 253.0 / 4096.0;
constexpr double b1 = 37.0 / 378.0, b3 = 250.0 / 621.0, b4 = 125.0 / 594.0, b6 = 512.0 / 1771.0;
constexpr double e1 = -277.0 / 64512.0, e3 = 6925.0 / 370944.0, e4 = -6925.0 / 202752.0,
                 e5 = -277.0 / 14336.0, e6 = 277.0 / 7084.0;
}  // namespace ck

// The same coefficients rounded to FP32 for the mixed-precision stage sums.
namespace ckf {
constexpr float a21 = 1.0f / 5.0f;
constexpr float a31 = 3.0f / 40.0f, a32 = 9.0f / 40.0f;
constexpr float a41 = 3.0f / 10.0f, a42 = -9.0f / 10.0f, a43 = 6.0f / 5.0f;
constexpr float a51 = -11.0f / 54.0f, a52 = 5.0f / 2.0f, a53 = -70.0f / 27.0f, a54 = 35.0f / 27.0f;
constexpr float a61 = 1631.0f / 55296.0f, a62 = 175.0f / 512.0f, a63 = 575.0f / 13824.0f,
                a64 = 44275.0f / 110592.0f, a65 = 253.0f / 4096.0f;
constexpr float b1 = 37.0f / 378.0f, b3 = 250.0f / 621.0f, b4 = 125.0f / 594.0f,
                b6 = 512.0f / 1771.0f;
}  // namespace ckf

enum { kMethodRKCK45 = 0, kMethodRK4 = 1 };
enum { kPrecFP64 = 0, kPrecMixed = 1 };

// y[c] for a component index c known only at run time, as a bitmask blend of
// all components.  (A chain of selects between array elements is folded by
// the compiler into one dynamically indexed load, which forces the whole array
// out of registers into scratch memory; masks do not fold that way.)
template <int N>
__device__ __forceinline__ double pick(const double (&y)[N], int c) {
  unsigned long long r = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const unsigned long long m = 0ull - (unsigned long long)(c == i);
    r |= (unsigned long long)__double_as_longlong(y[i]) & m;
  }
  return __longlong_as_double((long long)r);
}

// y[c] for the component every event and accessory of the launch watches:
// COMP >= 0 is that component known at compile time (a register read), -1 a
// run-time component (pick).  The launch chooses COMP from its specs, so the
// results are the same either way.
template <int COMP, int N>
__device__ __forceinline__ double cpick(const double (&y)[N], int c) {
  if constexpr (COMP >= 0 && COMP < N)
    return y[COMP];
  else
    return pick(y, c);
}

// y[c] <- v for a run-time component index c (bitmask blend, as in pick).
template <int N>
__device__ __forceinline__ void put(double (&y)[N], int c, double v) {
  const unsigned long long vb = (unsigned long long)__double_as_longlong(v);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const unsigned long long m = 0ull - (unsigned long long)(c == i);
    const unsigned long long yb = (unsigned long long)__double_as_longlong(y[i]);
    y[i] = __longlong_as_double((long long)((vb & m) | (yb & ~m)));
  }
}

// Stage time t + c*h rounded exactly as written (product, then sum), so that
// time arguments of the forcing terms carry no contraction-dependent ulp.
__device__ __forceinline__ double stage_time(double t, double c, double h) {
  return __dadd_rn(t, __dmul_rn(c, h));
}

// The stage weights of the FP64 attempt, read from a table in constant memory
// through an opaque scalar pointer at the start of the attempt.  As literals,
// each would be rebuilt by two scalar moves at every use; the loads are issued
// with the attempt's first instructions and the first weight is needed only
// after the first right-hand side, so their latency is hidden (27-50 fewer
// issued instructions per attempt of a lone wave, measured on the Duffing,
// relief-valve and Keller-Miksis kernels).  The stage-time fractions stay
// literals: the time-only terms that start every attempt need them at once.
enum CkWeight : int {
  kA21, kA31, kA32, kA41, kA42, kA43, kA51, kA52, kA53, kA54, kA61, kA62, kA63, kA64, kA65,
  kB1, kB3, kB4, kB6, kE1, kE3, kE4, kE5, kE6, kCkWeights
};
static __device__ __constant__ double kCkTable[kCkWeights] = {
    ck::a21, ck::a31, ck::a32, ck::a41, ck::a42, ck::a43, ck::a51, ck::a52,
    ck::a53, ck::a54, ck::a61, ck::a62, ck::a63, ck::a64, ck::a65, ck::b1,
    ck::b3,  ck::b4,  ck::b6,  ck::e1,  ck::e3,  ck::e4,  ck::e5,  ck::e6};
typedef const __attribute__((address_space(4))) double *CkTableRef;
__device__ __forceinline__ CkTableRef ck_table() {
  CkTableRef t = (CkTableRef)kCkTable;
  asm volatile("" : "+s"(t));   // opaque: the weights are loaded, not folded
  return t;
}

// One Cash-Karp step of length h from (t, y): propagated fifth-order
// solution y5 and error estimate err = h * sum e_i k_i.  The time-only terms
// of all six stages are evaluated first.
template <class M>
__device__ __forceinline__ void cash_karp_attempt(double t, const double (&y)[M::NS],
                                                  const double (&p)[M::NP], double h,
                                                  double (&y5)[M::NS], double (&err)[M::NS]) {
  constexpr int N = M::NS;
  constexpr int FW = M::NF > 0 ? M::NF : 1;
  const CkTableRef K = ck_table();
  const double ts[6] = {t, stage_time(t, ck::c2, h), stage_time(t, ck::c3, h),
                        stage_time(t, ck::c4, h), t + h, stage_time(t, ck::c6, h)};
  double F[6][FW];
  M::template forcing<6>(ts, p, F);
  double k1[N], k2[N], k3[N], k4[N], k5[N], k6[N], ys[N];
  M::rhs(y, p, F[0], k1);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(h, K[kA21] * k1[i], y[i]);
  M::rhs(ys, p, F[1], k2);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(h, fma(K[kA32], k2[i], K[kA31] * k1[i]), y[i]);
  M::rhs(ys, p, F[2], k3);
#pragma unroll
  for (int i = 0; i < N; ++i)
    ys[i] = fma(h, fma(K[kA43], k3[i], fma(K[kA42], k2[i], K[kA41] * k1[i])), y[i]);
  M::rhs(ys, p, F[3], k4);
#pragma unroll
  for (int i = 0; i < N; ++i)
    ys[i] = fma(h, fma(K[kA54], k4[i], fma(K[kA53], k3[i], fma(K[kA52], k2[i], K[kA51] * k1[i]))),
                y[i]);
  M::rhs(ys, p, F[4], k5);
#pragma unroll
  for (int i = 0; i < N; ++i)
    ys[i] = fma(h,
                fma(K[kA65], k5[i],
                    fma(K[kA64], k4[i], fma(K[kA63], k3[i], fma(K[kA62], k2[i], K[kA61] * k1[i])))),
                y[i]);
  M::rhs(ys, p, F[5], k6);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    y5[i] = fma(h, fma(K[kB6], k6[i], fma(K[kB4], k4[i], fma(K[kB3], k3[i], K[kB1] * k1[i]))), y[i]);
    err[i] = h * fma(K[kE6], k6[i],
                     fma(K[kE5], k5[i], fma(K[kE4], k4[i], fma(K[kE3], k3[i], K[kE1] * k1[i]))));
  }
}

// Mixed precision: the right-hand side and the stage sums run in FP32, the
// state, time, step and the error estimate in FP64.  Each stage input
// y + h * (FP32 sum) is formed in FP64 and handed to the model, which rounds
// to FP32 what it uses (after forming in FP64 any difference that would
// cancel in FP32, or reducing a large angle); the propagated solution adds the
// FP32 weighted sum to y in FP64; the error estimate h * sum e_i k_i is formed
// in FP64 from the FP32 stage derivatives, so it carries their rounding
// (~6e-8 relative) but no cancellation.
template <class M>
__device__ __forceinline__ void cash_karp_attempt_mixed(double t, const double (&y)[M::NS],
                                                        const double (&p)[M::NP],
                                                        const float (&q)[M::NQ], double h,
                                                        double (&y5)[M::NS],
                                                        double (&err)[M::NS]) {
  constexpr int N = M::NS;
  constexpr int FW = M::NF > 0 ? M::NF : 1;
  const double ts[6] = {t, stage_time(t, ck::c2, h), stage_time(t, ck::c3, h),
                        stage_time(t, ck::c4, h), t + h, stage_time(t, ck::c6, h)};
  float F[6][FW];
  M::template forcing32<6>(ts, p, F);
  float k1[N], k2[N], k3[N], k4[N], k5[N], k6[N];
  double ys[N];
  M::rhs32(y, q, F[0], k1);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(h, double(ckf::a21 * k1[i]), y[i]);
  M::rhs32(ys, q, F[1], k2);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(h, double(fmaf(ckf::a32, k2[i], ckf::a31 * k1[i])), y[i]);
  M::rhs32(ys, q, F[2], k3);
#pragma unroll
  for (int i = 0; i < N; ++i)
    ys[i] = fma(h, double(fmaf(ckf::a43, k3[i], fmaf(ckf::a42, k2[i], ckf::a41 * k1[i]))), y[i]);
  M::rhs32(ys, q, F[3], k4);
#pragma unroll
  for (int i = 0; i < N; ++i)
    ys[i] = fma(h,
                double(fmaf(ckf::a54, k4[i],
                            fmaf(ckf::a53, k3[i], fmaf(ckf::a52, k2[i], ckf::a51 * k1[i])))),
                y[i]);
  M::rhs32(ys, q, F[4], k5);
#pragma unroll
  for (int i = 0; i < N; ++i)
    ys[i] = fma(h,
                double(fmaf(ckf::a65, k5[i],
                            fmaf(ckf::a64, k4[i],
                                 fmaf(ckf::a63, k3[i], fmaf(ckf::a62, k2[i], ckf::a61 * k1[i]))))),
                y[i]);
  M::rhs32(ys, q, F[5], k6);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float inc = fmaf(ckf::b6, k6[i], fmaf(ckf::b4, k4[i], fmaf(ckf::b3, k3[i], ckf::b1 * k1[i])));
    y5[i] = fma(h, double(inc), y[i]);
    err[i] = h * fma(ck::e6, double(k6[i]),
                     fma(ck::e5, double(k5[i]),
                         fma(ck::e4, double(k4[i]), fma(ck::e3, double(k3[i]), ck::e1 * double(k1[i])))));
  }
}

// Classical RK4 with FP32 right-hand side and stage sums, FP64 state.
template <class M>
__device__ __forceinline__ void rk4_attempt_mixed(double t, const double (&y)[M::NS],
                                                  const double (&p)[M::NP],
                                                  const float (&q)[M::NQ], double h,
                                                  double (&yn)[M::NS]) {
  constexpr int N = M::NS;
  constexpr int FW = M::NF > 0 ? M::NF : 1;
  const double hh = 0.5 * h;
  const double ts[3] = {t, t + hh, t + h};
  float F[3][FW];
  M::template forcing32<3>(ts, p, F);
  float k1[N], k2[N], k3[N], k4[N];
  double ys[N];
  M::rhs32(y, q, F[0], k1);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(hh, double(k1[i]), y[i]);
  M::rhs32(ys, q, F[1], k2);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(hh, double(k2[i]), y[i]);
  M::rhs32(ys, q, F[1], k3);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(h, double(k3[i]), y[i]);
  M::rhs32(ys, q, F[2], k4);
  const double h6 = h * (1.0 / 6.0);
#pragma unroll
  for (int i = 0; i < N; ++i)
    yn[i] = fma(h6, double(fmaf(2.0f, k2[i] + k3[i], k1[i] + k4[i])), y[i]);
}

// One classical RK4 step of length h from (t, y).
template <class M>
__device__ __forceinline__ void rk4_attempt(double t, const double (&y)[M::NS],
                                            const double (&p)[M::NP], double h,
                                            double (&yn)[M::NS]) {
  constexpr int N = M::NS;
  constexpr int FW = M::NF > 0 ? M::NF : 1;
  const double hh = 0.5 * h;
  const double ts[3] = {t, t + hh, t + h};
  double F[3][FW];
  M::template forcing<3>(ts, p, F);
  double k1[N], k2[N], k3[N], k4[N], ys[N];
  M::rhs(y, p, F[0], k1);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(hh, k1[i], y[i]);
  M::rhs(ys, p, F[1], k2);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(hh, k2[i], y[i]);
  M::rhs(ys, p, F[1], k3);
#pragma unroll
  for (int i = 0; i < N; ++i) ys[i] = fma(h, k3[i], y[i]);
  M::rhs(ys, p, F[2], k4);
  const double h6 = h * (1.0 / 6.0);
#pragma unroll
  for (int i = 0; i < N; ++i) yn[i] = fma(h6, fma(2.0, k2[i] + k3[i], k1[i] + k4[i]), y[i]);
}

// E^(-1/5) for the step-size factor.  A single-precision seed (hardware
// log2/exp2, ~1e-7 relative) is refined by two Newton steps on x^-5 = E,
// x <- x + x (1 - E x^5) / 5, whose error goes 1e-7 -> 3e-14 -> rounding;
// outside [1e-30, 1e30] (where the factor is clamped anyway) the library
// routine replaces the result (a branch no lane normally takes, after the
// Newton steps rather than around them).
__device__ __forceinline__ double inv_fifth_root(double E) {
  const float lf = __builtin_amdgcn_logf(static_cast<float>(E));
  double x = static_cast<double>(__builtin_amdgcn_exp2f(-0.2f * lf));
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double x2 = x * x;
    const double x5 = x2 * x2 * x;
    x = fma(x * 0.2, fma(-E, x5, 1.0), x);
  }
  if (!(E >= 1e-30 && E <= 1e30)) x = pow(E, -0.2);
  return x;
}

// Event detection between the last accepted point (Fo, outside the zone) and
// the candidate (Fn): 0 none, 1 the step jumped over the zone (needs
// location), 2 the step ended inside the zone.  Direction -1 is F
// decreasing, +1 increasing, 0 both (paper Sec. 4 and Sec. 6.6).
__device__ __forceinline__ int detect(double Fo, double Fn, int dir, double tol) {
  const bool inside = fabs(Fn) <= tol;
  int r = 0;
  if (dir <= 0 && Fo > tol) r = (Fn < -tol) ? 1 : (inside ? 2 : 0);
  if (r == 0 && dir >= 0 && Fo < -tol) r = (Fn > tol) ? 1 : (inside ? 2 : 0);
  return r;
}

// Next step length of the event location: the secant root through the last
// two iterates, or the midpoint of the bracket (lo, hi) when the secant root
// leaves it.  Plain roundings, no contraction.
__device__ __forceinline__ double secant(double sa, double ga, double sb, double gb, double lo,
                                         double hi) {
  const double sc = __dsub_rn(sb, __ddiv_rn(__dmul_rn(gb, __dsub_rn(sb, sa)), __dsub_rn(gb, ga)));
  return (sc > lo && sc < hi) ? sc : __dmul_rn(0.5, __dadd_rn(lo, hi));
}

// The launch parameters seen through an opaque copy of the kernel-argument
// pointer.  Values read through it are loaded where they are used (scalar
// loads), instead of being hoisted to the kernel start and held in scalar
// registers for the whole run: the array pointers and the rarely used event
// fields would otherwise exhaust the scalar register file and spill into
// vector-register lanes inside the hot loop.
typedef const __attribute__((address_space(4))) Params *ParamsRef;
__device__ __forceinline__ ParamsRef fresh_params() {
  ParamsRef p = (ParamsRef)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return p;
}

// Field-wise copies out of the kernel-argument segment (the implicit copy
// constructors cannot bind to its address space).
__device__ __forceinline__ Arrays arrays_of(ParamsRef q) {
  Arrays a;
  a.td = q->a.td;
  a.y = q->a.y;
  a.p = q->a.p;
  a.acc = q->a.acc;
  a.next_h = q->a.next_h;
  a.status = q->a.status;
  a.counts = q->a.counts;
  a.evc = q->a.evc;
  a.rec = q->a.rec;
  a.index = q->a.index;
  a.t_rec = q->a.t_rec;
  a.tol = q->a.tol;
  a.n = q->a.n;
  a.ld = q->a.ld;
  a.queue = q->a.queue;
  a.total_waves = q->a.total_waves;
  a.avail = q->a.avail;
  a.closed = q->a.closed;
  a.req_of = q->a.req_of;
  a.req_left = q->a.req_left;
  a.req_done = q->a.req_done;
  a.n_req = q->a.n_req;
  a.idle_polls = q->a.idle_polls;
  return a;
}

// Served launches read what the host publishes while they run (copies on
// another stream, then the published count).  These loads are system-scope
// atomics, so they bypass any cache line that an earlier read of the same
// address left behind: slots and queue entries are reused for later requests.
template <class T>
__device__ __forceinline__ T load_published(const T *p) {
  return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ EventCtl event_of(ParamsRef q, int j) {
  EventCtl e;
  e.component = q->c.ev[j].component;
  e.direction = q->c.ev[j].direction;
  e.stop_after = q->c.ev[j].stop_after;
  e.action_component = q->c.ev[j].action_component;
  e.action_param = q->c.ev[j].action_param;
  e.record_component = q->c.ev[j].record_component;
  e.level = q->c.ev[j].level;
  e.tolerance = q->c.ev[j].tolerance;
  e.action_coef = q->c.ev[j].action_coef;
  return e;
}

// The launch constants that every attempt reads, held in vector registers
// for the whole launch.  Each is read once before the attempt loop and passed
// through an empty asm with a vector-register operand, so it stays in a VGPR
// as a per-lane value instead of being re-read by a scalar load where it is
// used.  Read through the kernel-argument pointer in the loop, an attempt
// waits on about ten scalar-cache round trips, a third of the time of a wave
// that runs alone on its SIMD (the slowest systems at the end of a sweep).
template <int N, int EV, int AC>
struct HotControl {
  double rtol[N], atol[N];
  double h0, h_min, h_max, grow, shrink, section_period;
  double ev_level[EV], ev_tol[EV];
  int32_t ev_comp[EV], ev_dir[EV];
  int32_t acc_kind[AC], acc_comp[AC];
  int32_t n_events, n_acc, max_eq, max_steps;
};

__device__ __forceinline__ double in_vgpr(double x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ int32_t in_vgpr(int32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int N, int EV, int AC>
__device__ __forceinline__ HotControl<N, EV, AC> hot_control(const Control &c) {
  static_assert(EV <= kMaxEvents && AC <= kMaxAcc && N <= kMaxState, "slot counts");
  HotControl<N, EV, AC> h;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    h.rtol[i] = in_vgpr(c.rtol[i]);
    h.atol[i] = in_vgpr(c.atol[i]);
  }
  h.h0 = in_vgpr(c.h0);
  h.h_min = in_vgpr(c.h_min);
  h.h_max = in_vgpr(c.h_max);
  h.grow = in_vgpr(c.grow);
  h.shrink = in_vgpr(c.shrink);
  h.section_period = in_vgpr(c.section_period);
#pragma unroll
  for (int j = 0; j < EV; ++j) {
    h.ev_level[j] = in_vgpr(c.ev[j].level);
    h.ev_tol[j] = in_vgpr(c.ev[j].tolerance);
    h.ev_comp[j] = in_vgpr(c.ev[j].component);
    h.ev_dir[j] = in_vgpr(c.ev[j].direction);
  }
#pragma unroll
  for (int k = 0; k < AC; ++k) {
    h.acc_kind[k] = in_vgpr(c.acc[k].kind);
    h.acc_comp[k] = in_vgpr(c.acc[k].component);
  }
  h.n_events = in_vgpr(c.n_events);
  h.n_acc = in_vgpr(c.n_acc);
  h.max_eq = in_vgpr(c.max_eq);
  h.max_steps = in_vgpr(c.max_steps);
  return h;
}

template <class M, int METHOD, int PREC, int NEV, int NACC, int COMP>
__global__ void __launch_bounds__(kMaxBlock) ode_integrate(const Params prm) {
  const Control &c = prm.c;
  constexpr int N = M::NS;
  constexpr int P = M::NP;
  constexpr int EV = NEV > 0 ? NEV : 1;
  constexpr int AC = NACC > 0 ? NACC : 1;
  const int lane = threadIdx.x & 63;

  // ---- per-lane system state (registers) ----
  int64_t s = -1;
  bool active = false;
  double t = 0.0, t1 = 0.0, h = 0.0;
  double t_rec = 0.0;  // start of this system's recording window
  double y[N], p[P];
  constexpr int Q = PREC == kPrecMixed ? M::NQ : 1;
  float pf[Q];  // FP32 parameters of the mixed-precision right-hand side
  int32_t attempts = 0, n_acc = 0, n_rej = 0, flags = 0, status = kRunning;
  bool window_open = false;
  double accv[AC], acct[AC];
  double seg_start = 0.0;  // RK4: the state after m steps of a segment is at seg_start + m*dt
  // index n of the next Poincare section n*T (an integer held in FP64)
  double sec_n = 0.0;
  int32_t seg_steps = 0;
  double F[EV];
  int32_t zone[EV], cnt[EV], wcnt[EV];
  uint32_t leaving = 0;    // bit j: inside the zone of event j
  int32_t n_rec = 0;
  // secant location of event J over step lengths in (lo, hi)
  bool locating = false;
  int32_t loc_it = 0, loc_c = 0;
  double loc_level = 0.0, loc_tol = 0.0;
  bool loc_pos = false;    // sign of F_J at the start of the step
  double lo = 0.0, hi = 0.0, sa = 0.0, ga = 0.0, sb = 0.0, gb = 0.0, sc = 0.0, h_keep = 0.0;
  uint32_t loc_bit = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) y[i] = 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) p[j] = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) pf[j] = 0.0f;
#pragma unroll
  for (int j = 0; j < EV; ++j) F[j] = 0.0, zone[j] = cnt[j] = wcnt[j] = 0;
#pragma unroll
  for (int k = 0; k < AC; ++k) accv[k] = acct[k] = 0.0;

  bool exhausted = false;  // wave-uniform
  bool first_fill = true;  // wave-uniform
  const uint32_t wave_id = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  uint32_t iter = 0;       // loop iterations of this wave (wave-uniform)
  int32_t idle = 0;        // served launches: empty polls in a row (wave-uniform)
  int32_t req = 0;         // served launches: request of the lane's system

  auto acc_init = [&]() {
#pragma unroll
    for (int k = 0; k < NACC; ++k)
      if (k < c.n_acc) {
        if (c.acc[k].kind == kAccLogReset) {
          accv[k] = 0.0;  // sum of ln y[c] at the sections
          acct[k] = 0.0;  // number of sections added
        } else {
          accv[k] = cpick<COMP>(y, c.acc[k].component);
          acct[k] = t;
        }
      }
  };

  auto retire = [&]() {
    if (!window_open) acc_init();  // window never opened: describe the final point
    const ParamsRef q = fresh_params();
    const Arrays a = arrays_of(q);
    const int64_t ld = a.ld;
    a.td[s] = t;
#pragma unroll
    for (int i = 0; i < N; ++i) a.y[i * ld + s] = y[i];
    if (a.next_h) a.next_h[s] = h;
    a.status[s] = status | flags;
    if (a.counts) {
      a.counts[s] = n_acc;
      a.counts[ld + s] = n_rej;
      a.counts[2 * ld + s] = attempts - n_acc - n_rej;
    }
#pragma unroll
    for (int k = 0; k < NACC; ++k)
      if (k < c.n_acc) {
        a.acc[(2 * k) * ld + s] = accv[k];
        a.acc[(2 * k + 1) * ld + s] = acct[k];
      }
    if (a.evc) {
#pragma unroll
      for (int j = 0; j < NEV; ++j)
        if (j < c.n_events) a.evc[j * ld + s] = wcnt[j];
    }
    if (a.avail) {
      // served: the results are written back before the request's count
      // drops, and the request's last system raises its flag in host memory;
      // then the position counts as finished
      __threadfence_system();
      if (req >= 0 && req < a.n_req && atomicSub(a.req_left + req, 1) == 1) {
        __threadfence_system();
        __hip_atomic_store(a.req_done + req, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      atomicAdd(a.queue + 1, 1ull);
    }
    active = false;
  };

  // per lane: a system's own tolerances replace the launch's at refill
  HotControl<N, EV, AC> hc = hot_control<N, EV, AC>(c);

  for (;;) {
    // ---- refill idle lanes from the queue (all 64 lanes are converged here) ----
    const unsigned long long need = __ballot(!active);
    if (need != 0 && !exhausted) {
      const ParamsRef q = fresh_params();
      const Arrays a = arrays_of(q);
      const int64_t ld = a.ld;
      const uint32_t k = __popcll(need);
      const bool served = a.avail != nullptr;
      unsigned long long base = 0, lim = (unsigned long long)a.n;  // positions [base, lim)
      if (served) {
        // Take up to k published positions: lane 0 advances the queue
        // counter with compare-and-swap, never beyond the published count.
        // While some lanes still integrate, poll every 16 iterations only.
        const bool all_idle = need == ~0ull;
        lim = 0;
        if (all_idle || (iter & 15u) == 0u) {
          unsigned long long b = 0, e = 0;
          if (lane == 0) {
            const unsigned long long av =
                (unsigned long long)__hip_atomic_load(const_cast<int64_t *>(a.avail), __ATOMIC_ACQUIRE,
                                                      __HIP_MEMORY_SCOPE_SYSTEM);
            unsigned long long old =
                __hip_atomic_load(a.queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int tries = 0; tries < 64; ++tries) {
              const unsigned long long want = (old + k < av) ? old + k : av;
              if (want <= old) break;
              if (__hip_atomic_compare_exchange_strong(a.queue, &old, want, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                b = old;
                e = want;
                break;
              }
            }
          }
          base = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
                 (unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)b);
          lim = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(e >> 32)) << 32) |
                (unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)e);
          if (lim > base) {
            idle = 0;
          } else if (all_idle) {
            // Nothing to take.  Leave once the host has closed the queue and
            // every published position is taken; otherwise wait while some
            // taken position is still being integrated (by other waves, each
            // within its step budget, so the wait is bounded), and leave
            // after idle_polls empty polls in a row with every published
            // position finished.  The host relaunches when work arrives
            // after that; a launch cannot be topped up while any of its
            // waves runs, so its waves must not leave while work may follow.
            int stop = 0;
            if (lane == 0) {
              const int32_t cl = __hip_atomic_load(const_cast<int32_t *>(a.closed), __ATOMIC_ACQUIRE,
                                                   __HIP_MEMORY_SCOPE_SYSTEM);
              const unsigned long long av = (unsigned long long)__hip_atomic_load(
                  const_cast<int64_t *>(a.avail), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
              const unsigned long long qv =
                  __hip_atomic_load(a.queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              const unsigned long long fv =
                  __hip_atomic_load(a.queue + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              stop = (cl != 0 && qv >= av) ? 1 : (fv < qv ? 2 : 0);
            }
            stop = __builtin_amdgcn_readfirstlane(stop);
            if (stop == 2) idle = 0;
            if (stop == 1 || (stop == 0 && ++idle >= a.idle_polls)) {
              exhausted = true;
            } else {
              __builtin_amdgcn_s_sleep(127);
            }
          }
        }
      } else if (first_fill && (unsigned long long)a.total_waves * 64ull >= (unsigned long long)a.n) {
        // Every system has a lane from the start: wave w takes queue
        // positions 64w .. 64w + 63, so the queue order decides which systems
        // share a SIMD.  The waves of the first 256 workgroups (one per CU)
        // share their SIMDs with those of the next 256, one wave each; a
        // caller that knows the systems' costs can order the queue so that
        // each SIMD gets one long and one short chunk.
        base = (unsigned long long)wave_id * 64ull;
        exhausted = true;
      } else {
        // with more systems than lanes the counter hands out positions in
        // queue order (an input sorted heaviest first stays so), and refills
        // balance the XCDs
        if (lane == 0) base = atomicAdd(a.queue, (unsigned long long)k);
        base = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
               (unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)base);
        if (base + k >= (unsigned long long)a.n) exhausted = true;
      }
      first_fill = false;
      if (!active) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
        const unsigned long long pos = base + rank;
        if (pos < lim) {
          const int64_t cand = served ? load_published(a.index + pos % (unsigned long long)ld)
                                      : (a.index ? a.index[pos] : (int64_t)pos);
          if (cand >= 0 && cand < ld) {
            s = cand;
            active = true;
            // ---- load and initialise the system ----
            if (served) {
              req = load_published(a.req_of + s);
              t = load_published(a.td + s);
              t1 = load_published(a.td + ld + s);
              t_rec = a.t_rec ? load_published(a.t_rec + s) : c.t_record;
#pragma unroll
              for (int i = 0; i < N; ++i) y[i] = load_published(a.y + i * ld + s);
#pragma unroll
              for (int j = 0; j < P; ++j) p[j] = load_published(a.p + j * ld + s);
            } else {
              t = a.td[s];
              t1 = a.td[ld + s];
              t_rec = a.t_rec ? a.t_rec[s] : c.t_record;
#pragma unroll
              for (int i = 0; i < N; ++i) y[i] = a.y[i * ld + s];
#pragma unroll
              for (int j = 0; j < P; ++j) p[j] = a.p[j * ld + s];
            }
            if constexpr (PREC == kPrecMixed) {
              M::prepare32(p, pf);
            }
            bool tol_ok = true;
            if (METHOD == kMethodRKCK45 && a.tol) {
#pragma unroll
              for (int i = 0; i < N; ++i) {
                const double rt = served ? load_published(a.tol + i * ld + s) : a.tol[i * ld + s];
                const double at =
                    served ? load_published(a.tol + (N + i) * ld + s) : a.tol[(N + i) * ld + s];
                tol_ok = tol_ok && rt >= 0.0 && at >= 0.0 && rt + at > 0.0 &&
                         rt + at < __builtin_huge_val();
                hc.rtol[i] = rt;
                hc.atol[i] = at;
              }
            }
            attempts = n_acc = n_rej = flags = 0;
            status = kRunning;
            locating = false;
            seg_start = t;
            seg_steps = 0;
            n_rec = 0;
            leaving = 0;
            if (METHOD == kMethodRK4) {
              h = c.h0;
            } else {
              h = c.h0;
              if (a.next_h) {
                const double hn = served ? load_published(a.next_h + s) : a.next_h[s];
                if (hn > 0.0 && isfinite(hn)) h = hn;
              }
              h = fmin(fmax(h, c.h_min), c.h_max);
            }
#pragma unroll
            for (int j = 0; j < NEV; ++j) {
              zone[j] = cnt[j] = wcnt[j] = 0;
              if (j < c.n_events) {
                F[j] = cpick<COMP>(y, c.ev[j].component) - c.ev[j].level;
                // an initial point inside a zone is not an event (paper Sec. 7.2)
                if (fabs(F[j]) <= c.ev[j].tolerance) leaving |= 1u << j;
              }
            }
            window_open = false;
            sec_n = 0.0;
            if (!isfinite(t) || !isfinite(t1) || !tol_ok) {
              status = kBadInput;
            } else {
              // Poincare sections n*T count from time zero; the first one is
              // the first rounded product strictly after t (paper Sec. 2.1)
              const double T = c.section_period;
              if (T > 0.0) {
                sec_n = floor(t / T) + 1.0;
                for (int it = 0; it < 3 && __dmul_rn(sec_n, T) <= t; ++it) sec_n += 1.0;
              }
              if (t_rec <= t) {
                window_open = true;
                acc_init();
              }
            }
            if (status == kRunning && t >= t1) status = kDone;
            if (status != kRunning) retire();
          } else if (served) {
            atomicAdd(a.queue + 1, 1ull);  // a ring entry naming no slot: finished
          }
        }
      }
    }
    if (__ballot(active) == 0) {
      if (exhausted) break;
      continue;
    }
    // Issue priority by remaining work, re-estimated every 64 iterations: the
    // wave's largest remaining step count at its lanes' current step sizes, in
    // four levels.  When two waves share a SIMD, the one that will run longer
    // issues first, so the longest serial chains -- which set the end of a
    // sweep whose systems are all resident -- run closer to their solo speed
    // while the other wave fills the gaps.  It orders issue only; results do
    // not depend on it.  (Duffing sweep: 4.5% faster; kernels with one wave
    // per SIMD are unaffected.)
    if ((++iter & 63u) == 1u) {
      const double rem = active ? (t1 - t) / fmax(h, 1e-300) : 0.0;
      if (__ballot(rem > 131072.0)) {
        __builtin_amdgcn_s_setprio(3);
      } else if (__ballot(rem > 32768.0)) {
        __builtin_amdgcn_s_setprio(2);
      } else if (__ballot(rem > 8192.0)) {
        __builtin_amdgcn_s_setprio(1);
      } else {
        __builtin_amdgcn_s_setprio(0);
      }
    }
    if (!active) continue;

    // ---- choose this attempt's step length ----
    double t_b = t1, h_att;
    bool clipped = false;
    if (locating) {
      h_att = sc;
    } else {
      t_b = (!window_open && t_rec < t1) ? t_rec : t1;
      if (hc.section_period > 0.0) {
        const double t_sec = __dmul_rn(sec_n, hc.section_period);
        t_b = (t_sec < t_b) ? t_sec : t_b;
      }
      if (METHOD == kMethodRK4) {
        const double t_grid = __dadd_rn(seg_start, __dmul_rn((double)(seg_steps + 1), hc.h0));
        if (t_grid >= __dsub_rn(t_b, __dmul_rn(1e-9, hc.h0))) {
          h_att = t_b - t;
          clipped = true;
        } else {
          h_att = hc.h0;
        }
      } else {
        h_att = h;
        if (h_att >= t_b - t) {
          h_att = t_b - t;
          clipped = true;
        }
      }
    }

    // ---- the attempt: one full method step from (t, y) ----
    double yn[N], err[N];
    if constexpr (PREC == kPrecMixed) {
      if (METHOD == kMethodRK4)
        rk4_attempt_mixed<M>(t, y, p, pf, h_att, yn);
      else
        cash_karp_attempt_mixed<M>(t, y, p, pf, h_att, yn, err);
    } else {
      if (METHOD == kMethodRK4)
        rk4_attempt<M>(t, y, p, h_att, yn);
      else
        cash_karp_attempt<M>(t, y, p, h_att, yn, err);
    }
    ++attempts;

    bool commit = false, located = false;
    double tn = t;
    uint32_t det = 0;  // events detected by the committed step

    if (!locating) {
      double h_next = h;
      bool passed = true;
      if (METHOD == kMethodRKCK45) {
        // Error test (paper Sec. 6.5): scaled max norm, step factor
        // 0.9*E^(-1/5) limited to [shrink, grow]; at h_min every step is
        // accepted; NaN rejects and shrinks, and stops at h_min.
        bool has_nan = false;
        double E = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          has_nan |= isnan(yn[i]);
          const double sc_i = fma(hc.rtol[i], fmax(fabs(y[i]), fabs(yn[i])), hc.atol[i]);
          const double r = fabs(err[i]) / sc_i;
          has_nan |= isnan(r);
          E = (r > E) ? r : E;
        }
        if (has_nan) {
          passed = false;
          if (h_att <= hc.h_min) {
            status = kFailNan;
          } else {
            h = fmax(hc.h_min, hc.shrink * h_att);
            ++n_rej;
          }
        } else {
          double fac = (E == 0.0) ? hc.grow : 0.9 * inv_fifth_root(E);
          fac = fmax(hc.shrink, fmin(hc.grow, fac));
          h_next = fmax(hc.h_min, fmin(hc.h_max, fac * h_att));
          if (!(E <= 1.0) && h_att > hc.h_min) {
            passed = false;
            h = h_next;
            ++n_rej;
          }
        }
      }
      if (passed) {
        uint32_t cross = 0, land = 0;
#pragma unroll
        for (int j = 0; j < NEV; ++j) {
          if (j < hc.n_events && !((leaving >> j) & 1u)) {
            const double Fn = cpick<COMP>(yn, hc.ev_comp[j]) - hc.ev_level[j];
            const int d = detect(F[j], Fn, hc.ev_dir[j], hc.ev_tol[j]);
            cross |= (d == 1 ? 1u : 0u) << j;
            land |= (d == 2 ? 1u : 0u) << j;
          }
        }
        const uint32_t any = cross | land;
        // the event specified last is the one located precisely (paper Sec. 4)
        const uint32_t top = any ? (1u << (31 - __clz(any))) : 0u;
        if (top & cross) {
          locating = true;
          loc_bit = top;
          loc_it = 0;
#pragma unroll
          for (int j = 0; j < NEV; ++j)
            if (top == (1u << j)) {
              loc_c = hc.ev_comp[j];
              loc_level = hc.ev_level[j];
              loc_tol = hc.ev_tol[j];
              ga = F[j];
            }
          gb = cpick<COMP>(yn, loc_c) - loc_level;
          loc_pos = ga > 0.0;
          lo = 0.0;
          hi = h_att;
          sa = 0.0;
          sb = h_att;
          h_keep = h_next;
          sc = secant(sa, ga, sb, gb, lo, hi);
        } else {
          commit = true;
          det = any;
          if (clipped)
            tn = t_b;
          else if (METHOD == kMethodRK4)
            tn = __dadd_rn(seg_start, __dmul_rn((double)(seg_steps + 1), hc.h0));
          else
            tn = t + h_att;
          if (METHOD == kMethodRKCK45) {
            // after a step clipped to a boundary, do not shrink below the
            // step in use before the clip
            h = (clipped && h_next < h) ? h : h_next;
          }
        }
      }
    } else {
      // one secant iterate of the location of event J
      const double gc = cpick<COMP>(yn, loc_c) - loc_level;
      ++loc_it;
      const bool found = fabs(gc) <= loc_tol;
      if (found || loc_it >= kSecantMaxIter) {
        if (!found) flags |= kFlagSecantCap;
        commit = true;
        located = true;
        locating = false;
        tn = t + sc;
        h = h_keep;  // the proposal from the full step stands
        det = loc_bit;
#pragma unroll
        for (int j = 0; j < NEV; ++j) {
          if (j < hc.n_events && (1u << j) != loc_bit && !((leaving >> j) & 1u)) {
            const double Fn = cpick<COMP>(yn, hc.ev_comp[j]) - hc.ev_level[j];
            det |= (detect(F[j], Fn, hc.ev_dir[j], hc.ev_tol[j]) != 0 ? 1u : 0u) << j;
          }
        }
      } else {
        if ((gc > 0.0) == loc_pos)
          lo = sc;
        else
          hi = sc;
        sa = sb;
        ga = gb;
        sb = sc;
        gb = gc;
        sc = secant(sa, ga, sb, gb, lo, hi);
      }
    }

    if (commit) {
      t = tn;
#pragma unroll
      for (int i = 0; i < N; ++i) y[i] = yn[i];
      ++n_acc;
      if (METHOD == kMethodRK4) {
        if (located || clipped) {
          seg_start = t;
          seg_steps = 0;
        } else {
          ++seg_steps;
        }
      }
      // ordinary accessories (paper Sec. 6.7) inside the recording window,
      // initialised when it opens (Sec. 6.8)
      if (!window_open) {
        if (t >= t_rec) {
          window_open = true;
          acc_init();
        }
      } else {
#pragma unroll
        for (int k = 0; k < NACC; ++k)
          if (k < hc.n_acc && hc.acc_kind[k] != kAccLogReset) {
            const double v = cpick<COMP>(y, hc.acc_comp[k]);
            const bool better = (hc.acc_kind[k] == kAccMax) ? (v > accv[k]) : (v < accv[k]);
            accv[k] = better ? v : accv[k];
            acct[k] = better ? t : acct[k];
          }
      }
      // event hooks in increasing index: counter, window count and record,
      // action (e.g. the impact law), stop count (paper Sec. 6.6)
#pragma unroll
      for (int j = 0; j < NEV; ++j) {
        if ((det >> j) & 1u) {
          ++cnt[j];
          if (window_open) {
            ++wcnt[j];
            if (fresh_params()->c.ev[j].record_component >= 0) {
              const ParamsRef q = fresh_params();
              if (n_rec < q->c.rec_cap) {
                const int64_t ld = q->a.ld;
                q->a.rec[(int64_t)(2 * n_rec) * ld + s] = t;
                q->a.rec[(int64_t)(2 * n_rec + 1) * ld + s] = pick(y, q->c.ev[j].record_component);
              }
              ++n_rec;
            }
          }
          const ParamsRef q = fresh_params();
          const EventCtl e = event_of(q, j);
          if (e.action_component >= 0) {
            double coef = e.action_coef;
            if (e.action_param >= 0) coef *= pick(p, e.action_param);
            put(y, e.action_component, coef * pick(y, e.action_component));
          }
          if (e.stop_after > 0 && cnt[j] == e.stop_after) status = kStopEvent;
        }
      }
      // Poincare section reached (the step was clipped to it): the Lyapunov
      // accumulators add ln y[c] for sections after the window start, and
      // y[c] restarts from 1 at every section (paper Sec. 2.1)
      if (hc.section_period > 0.0 && t == __dmul_rn(sec_n, hc.section_period)) {
#pragma unroll
        for (int k = 0; k < NACC; ++k)
          if (k < hc.n_acc && hc.acc_kind[k] == kAccLogReset) {
            const int comp = hc.acc_comp[k];
            if (window_open && t > t_rec) {
              accv[k] = accv[k] + log(pick(y, comp));
              acct[k] = acct[k] + 1.0;
            }
            put(y, comp, 1.0);
          }
        sec_n += 1.0;
      }
      // zone states: normal exactly when outside the zone; accepted steps
      // that stay inside after a detection count towards the equilibrium stop
#pragma unroll
      for (int j = 0; j < NEV; ++j) {
        if (j < hc.n_events) {
          F[j] = cpick<COMP>(y, hc.ev_comp[j]) - hc.ev_level[j];
          const bool inside = fabs(F[j]) <= hc.ev_tol[j];
          const uint32_t bit = 1u << j;
          if (((det | ~leaving) & bit) != 0) {
            leaving = inside ? (leaving | bit) : (leaving & ~bit);
            zone[j] = 0;
          } else if (inside) {
            ++zone[j];
            if (hc.max_eq > 0 && zone[j] >= hc.max_eq && status == kRunning)
              status = kStopEquilibrium;
          } else {
            leaving &= ~bit;
            zone[j] = 0;
          }
        }
      }
      if (status == kRunning && t >= t1) status = kDone;
    }
    if (status == kRunning && !locating && attempts >= hc.max_steps) status = kMaxSteps;
    if (status != kRunning) retire();
  }

  // The last wave to leave resets the queue for the next launch.  (A served
  // queue keeps its position: a later launch continues from it.)
  if (lane == 0) {
    const Arrays a = arrays_of(fresh_params());
    if (!a.avail) {
      __threadfence();
      const unsigned long long done = atomicAdd(a.queue + 1, 1ull);
      if (done + 1 == (unsigned long long)a.total_waves) {
        atomicExch(a.queue, 0ull);
        atomicExch(a.queue + 1, 0ull);
      }
    }
  }
}

// Instantiation table for one model: kernels for both methods, both
// precisions and every compiled (event slots, accessory slots) pair, each with
// run-time components; the FP64 kernels of the slot pairs the sweeps use most
// (one event, two accessories, or both) also with components 0 and 1 fixed at
// compile time.
template <class M>
struct ModelKernels {
  template <int METHOD, int PREC, int NEV, int NACC, int COMP>
  static const void *fn() {
    return reinterpret_cast<const void *>(&ode_integrate<M, METHOD, PREC, NEV, NACC, COMP>);
  }
  template <int METHOD, int PREC, int NEV, int NACC>
  static const void *by_comp(int comp) {
    if constexpr (PREC == kPrecFP64 && ((NEV == 1 && NACC <= 2) || (NEV == 0 && NACC == 2))) {
      if (comp == 0) return fn<METHOD, PREC, NEV, NACC, 0>();
      if (comp == 1) return fn<METHOD, PREC, NEV, NACC, 1>();
    }
    return fn<METHOD, PREC, NEV, NACC, -1>();
  }
  template <int METHOD, int PREC>
  static const void *by_slots(int nev, int nacc, int comp) {
    switch (nev * 10 + nacc) {
      case 0: return by_comp<METHOD, PREC, 0, 0>(comp);
      case 2: return by_comp<METHOD, PREC, 0, 2>(comp);
      case 4: return by_comp<METHOD, PREC, 0, 4>(comp);
      case 10: return by_comp<METHOD, PREC, 1, 0>(comp);
      case 12: return by_comp<METHOD, PREC, 1, 2>(comp);
      case 14: return by_comp<METHOD, PREC, 1, 4>(comp);
      case 40: return by_comp<METHOD, PREC, 4, 0>(comp);
      case 42: return by_comp<METHOD, PREC, 4, 2>(comp);
      case 44: return by_comp<METHOD, PREC, 4, 4>(comp);
      default: return nullptr;
    }
  }
  template <int PREC>
  static const void *by_method(int method, int nev, int nacc, int comp) {
    if (method == kMethodRKCK45) return by_slots<kMethodRKCK45, PREC>(nev, nacc, comp);
    if (method == kMethodRK4) return by_slots<kMethodRK4, PREC>(nev, nacc, comp);
    return nullptr;
  }
  static const void *get(int method, int prec, int nev, int nacc, int comp) {
    if (prec == kPrecFP64) return by_method<kPrecFP64>(method, nev, nacc, comp);
    if (prec == kPrecMixed) return by_method<kPrecMixed>(method, nev, nacc, comp);
    return nullptr;
  }
};

}  // namespace odeens
