// Right-hand sides f(t, y; p) of the built-in models, as device functors.
// Each model is a compile-time type, so the integrator kernel is specialised
// per model and the right-hand side is inlined into the stage loop (the paper
// keeps its device functions in the kernel's translation unit for the same
// reason, Sec. 6.9).
//
// The right-hand side is split in two: `forcing` evaluates the terms that
// depend on time only (the harmonic excitations) at all stage times of one
// attempt, before the stage chain starts, and `rhs` combines them with the
// state.  The time-only terms are then independent work the scheduler can
// overlap with the dependent stage chain, and the stage values can be formed
// from one full sine/cosine evaluation per attempt by angle addition.
#pragma once

#include <hip/hip_runtime.h>

namespace odeens {

// sin and cos of (base + delta) from sb = sin(base), cb = cos(base), for
// |delta| <= pi/4.  sin(delta) and cos(delta) - 1 are their Taylor series
// through delta^15 / delta^16 (truncation below 1e-16 relative on the
// interval); cos(delta) - 1 is formed directly so that nothing cancels.
__device__ __forceinline__ void rotate(double delta, double sb, double cb, double &s, double &c) {
  const double d2 = delta * delta;
  double ps = -1.0 / 1307674368000.0;        // -1/15!
  ps = fma(ps, d2, 1.0 / 6227020800.0);      //  1/13!
  ps = fma(ps, d2, -1.0 / 39916800.0);       // -1/11!
  ps = fma(ps, d2, 1.0 / 362880.0);          //  1/9!
  ps = fma(ps, d2, -1.0 / 5040.0);           // -1/7!
  ps = fma(ps, d2, 1.0 / 120.0);             //  1/5!
  ps = fma(ps, d2, -1.0 / 6.0);              // -1/3!
  const double sd = fma(delta * d2, ps, delta);
  double pc = 1.0 / 20922789888000.0;        //  1/16!
  pc = fma(pc, d2, -1.0 / 87178291200.0);    // -1/14!
  pc = fma(pc, d2, 1.0 / 479001600.0);       //  1/12!
  pc = fma(pc, d2, -1.0 / 3628800.0);        // -1/10!
  pc = fma(pc, d2, 1.0 / 40320.0);           //  1/8!
  pc = fma(pc, d2, -1.0 / 720.0);            // -1/6!
  pc = fma(pc, d2, 1.0 / 24.0);              //  1/4!
  pc = fma(pc, d2, -0.5);                    // -1/2!
  const double cm1 = d2 * pc;
  s = fma(cb, sd, fma(sb, cm1, sb));
  c = fma(cb, cm1, fma(-sb, sd, cb));
}

// The same rotation for |delta| <= 1/16 (steps short against the forcing
// period, the usual case): Taylor through delta^9 / delta^10, truncation
// below 2e-21.
constexpr double kShortRotate = 0.0625;
__device__ __forceinline__ void rotate_short(double delta, double sb, double cb, double &s,
                                             double &c) {
  const double d2 = delta * delta;
  double ps = 1.0 / 362880.0;                //  1/9!
  ps = fma(ps, d2, -1.0 / 5040.0);           // -1/7!
  ps = fma(ps, d2, 1.0 / 120.0);             //  1/5!
  ps = fma(ps, d2, -1.0 / 6.0);              // -1/3!
  const double sd = fma(delta * d2, ps, delta);
  double pc = -1.0 / 3628800.0;              // -1/10!
  pc = fma(pc, d2, 1.0 / 40320.0);           //  1/8!
  pc = fma(pc, d2, -1.0 / 720.0);            // -1/6!
  pc = fma(pc, d2, 1.0 / 24.0);              //  1/4!
  pc = fma(pc, d2, -0.5);                    // -1/2!
  const double cm1 = d2 * pc;
  s = fma(cb, sd, fma(sb, cm1, sb));
  c = fma(cb, cm1, fma(-sb, sd, cb));
}

// sin/cos of `arg` given sin/cos of a nearby `base`.  The difference
// arg - base is exact when the two are within a factor of two (Sterbenz), so
// the function is evaluated at exactly `arg`; far from `base` (a long step)
// the full library routine is used.
__device__ __forceinline__ void sincos_near(double arg, double base, double sb, double cb,
                                            double &s, double &c) {
  constexpr double kQuarterPi = 0.78539816339744830962;
  const double delta = __dsub_rn(arg, base);
  if (fabs(delta) <= kQuarterPi) {
    rotate(delta, sb, cb, s, c);
  } else {
    sincos(arg, &s, &c);
  }
}

// sin/cos of the stage phases arg[1..S-1] from those of arg[0] = base.  When
// every stage lies within 1/16 of the base (one decision per attempt, so the
// lanes of a wave normally agree) the short rotation serves all stages.
template <int S>
__device__ __forceinline__ void stage_sincos(const double (&arg)[S], double sb, double cb,
                                             double (&s)[S], double (&c)[S]) {
  double d[S];
  double dmax = 0.0;
#pragma unroll
  for (int k = 1; k < S; ++k) {
    d[k] = __dsub_rn(arg[k], arg[0]);
    dmax = fmax(dmax, fabs(d[k]));
  }
  s[0] = sb;
  c[0] = cb;
  if (dmax <= kShortRotate) {
#pragma unroll
    for (int k = 1; k < S; ++k) rotate_short(d[k], sb, cb, s[k], c[k]);
  } else {
#pragma unroll
    for (int k = 1; k < S; ++k) sincos_near(arg[k], arg[0], sb, cb, s[k], c[k]);
  }
}

// Mixed precision: sin/cos of a phase known in FP64, evaluated in FP32.  The
// phase is turned into revolutions and reduced to [-1/2, 1/2] in FP64 (exact
// subtraction of the nearest integer), and the hardware sine/cosine, which
// take revolutions, finish in FP32 (~1e-7 absolute).
__device__ __forceinline__ float sin_turns(double turns) {
  return __builtin_amdgcn_sinf(static_cast<float>(turns - rint(turns)));
}
__device__ __forceinline__ float cos_turns(double turns) {
  return __builtin_amdgcn_cosf(static_cast<float>(turns - rint(turns)));
}
constexpr double kInvTwoPi = 0.15915494309189533576888376337251;

// FP32 ln(1 + x) and exp(z) - 1 with small relative error also where the
// result is small (the mixed-precision Keller-Miksis pressure balance needs
// both near x = z = 0).  Near zero: ln(1 + x) = 2 atanh(s), s = x / (2 + x),
// by its odd series through s^7 (|x| < 1/4 gives |s| < 1/9, truncation
// < 3e-9 relative); exp(z) - 1 by Taylor's series through z^7 (|z| < 1/4,
// truncation < 2e-9 relative).  Elsewhere the hardware log2 / exp2.
__device__ __forceinline__ float log1p32(float x) {
  if (fabsf(x) < 0.25f) {
    const float s = x * __builtin_amdgcn_rcpf(2.0f + x);
    const float s2 = s * s;
    const float poly = fmaf(s2, fmaf(s2, fmaf(s2, 1.0f / 7.0f, 1.0f / 5.0f), 1.0f / 3.0f), 1.0f);
    return 2.0f * s * poly;
  }
  return __builtin_amdgcn_logf(1.0f + x) * 0.69314718055994530942f;
}
__device__ __forceinline__ float expm1_32(float z) {
  if (fabsf(z) < 0.25f) {
    float e = fmaf(z, 1.0f / 7.0f, 1.0f);
    e = fmaf(z * (1.0f / 6.0f), e, 1.0f);
    e = fmaf(z * (1.0f / 5.0f), e, 1.0f);
    e = fmaf(z * (1.0f / 4.0f), e, 1.0f);
    e = fmaf(z * (1.0f / 3.0f), e, 1.0f);
    e = fmaf(z * 0.5f, e, 1.0f);
    return z * e;
  }
  return __builtin_amdgcn_exp2f(z * 1.44269504088896340736f) - 1.0f;
}

// Every model's mixed-precision right-hand side receives the stage state in
// FP64 and its FP32 parameters `q` (`prepare32` derives them from the FP64
// parameters once per system).

// Duffing oscillator, paper Sec. 2.1 Eqs. (1)-(2), with linear and cubic
// stiffness as parameters: p = (k, B, omega, lin, cub),
//   y1' = y2,  y2' = -lin*y1 - cub*y1^3 - k*y2 + B*cos(omega*t).
// Time-only term per stage: cos(omega*t).
struct Duffing {
  static constexpr int NS = 2;
  static constexpr int NP = 5;
  static constexpr int NF = 1;
  static constexpr int NQ = 5;
  static constexpr int ID = 1;
  template <int S>
  __device__ __forceinline__ static void forcing(const double (&ts)[S], const double (&p)[NP],
                                                 double (&F)[S][NF]) {
    double arg[S], sn[S], cs[S];
#pragma unroll
    for (int k = 0; k < S; ++k) arg[k] = __dmul_rn(p[2], ts[k]);
    double sb, cb;
    sincos(arg[0], &sb, &cb);
    stage_sincos<S>(arg, sb, cb, sn, cs);
#pragma unroll
    for (int k = 0; k < S; ++k) F[k][0] = cs[k];
  }
  __device__ __forceinline__ static void rhs(const double (&y)[NS], const double (&p)[NP],
                                             const double (&F)[NF], double (&f)[NS]) {
    const double y1 = y[0], y2 = y[1];
    const double spring = fma(p[4] * y1 * y1, y1, fma(p[3], y1, p[0] * y2));
    f[0] = y2;
    f[1] = fma(p[1], F[0], -spring);
  }
  template <int S>
  __device__ __forceinline__ static void forcing32(const double (&ts)[S], const double (&p)[NP],
                                                   float (&F)[S][NF]) {
#pragma unroll
    for (int k = 0; k < S; ++k) F[k][0] = cos_turns(__dmul_rn(p[2], ts[k]) * kInvTwoPi);
  }
  __device__ __forceinline__ static void prepare32(const double (&p)[NP], float (&q)[NQ]) {
#pragma unroll
    for (int j = 0; j < NQ; ++j) q[j] = static_cast<float>(p[j]);
  }
  __device__ __forceinline__ static void rhs32(const double (&y)[NS], const float (&p)[NQ],
                                               const float (&F)[NF], float (&f)[NS]) {
    const float y1 = static_cast<float>(y[0]), y2 = static_cast<float>(y[1]);
    const float spring = fmaf(p[4] * y1 * y1, y1, fmaf(p[3], y1, p[0] * y2));
    f[0] = y2;
    f[1] = fmaf(p[1], F[0], -spring);
  }
};

// Duffing oscillator with its linearisation in polar coordinates attached,
// paper Sec. 2.1 Eqs. (3)-(6): the tangent vector r (cos phi, sin phi) of the
// Duffing flow evolves with g1 = dF2/dy1 = -lin - 3 cub y1^2 and
// g2 = dF2/dy2 = -k:
//   r'   = r ((1 + g1) sin(phi) cos(phi) + g2 sin(phi)^2)
//   phi' = -sin(phi)^2 + (g1 cos(phi) + g2 sin(phi)) cos(phi).
// y = (y1, y2, r, phi), p = (k, B, omega, lin, cub) as for Duffing.  The
// angle is state-dependent, so its sine and cosine are evaluated per stage
// (the paper also computes them once per evaluation and reuses them).
struct DuffingLyapunov {
  static constexpr int NS = 4;
  static constexpr int NP = 5;
  static constexpr int NF = 1;
  static constexpr int NQ = 5;
  static constexpr int ID = 5;
  template <int S>
  __device__ __forceinline__ static void forcing(const double (&ts)[S], const double (&p)[NP],
                                                 double (&F)[S][NF]) {
    Duffing::forcing<S>(ts, p, F);
  }
  __device__ __forceinline__ static void rhs(const double (&y)[NS], const double (&p)[NP],
                                             const double (&F)[NF], double (&f)[NS]) {
    const double y1 = y[0], y2 = y[1], r = y[2];
    const double spring = fma(p[4] * y1 * y1, y1, fma(p[3], y1, p[0] * y2));
    f[0] = y2;
    f[1] = fma(p[1], F[0], -spring);
    const double g1 = fma(-3.0 * p[4], y1 * y1, -p[3]);
    const double g2 = -p[0];
    double sn, cs;
    sincos(y[3], &sn, &cs);
    f[2] = r * sn * fma(1.0 + g1, cs, g2 * sn);
    f[3] = fma(fma(g1, cs, g2 * sn), cs, -sn * sn);
  }
  template <int S>
  __device__ __forceinline__ static void forcing32(const double (&ts)[S], const double (&p)[NP],
                                                   float (&F)[S][NF]) {
    Duffing::forcing32<S>(ts, p, F);
  }
  __device__ __forceinline__ static void prepare32(const double (&p)[NP], float (&q)[NQ]) {
#pragma unroll
    for (int j = 0; j < NQ; ++j) q[j] = static_cast<float>(p[j]);
  }
  __device__ __forceinline__ static void rhs32(const double (&y)[NS], const float (&p)[NQ],
                                               const float (&F)[NF], float (&f)[NS]) {
    const float y1 = static_cast<float>(y[0]), y2 = static_cast<float>(y[1]);
    const float r = static_cast<float>(y[2]);
    const float spring = fmaf(p[4] * y1 * y1, y1, fmaf(p[3], y1, p[0] * y2));
    f[0] = y2;
    f[1] = fmaf(p[1], F[0], -spring);
    const float g1 = fmaf(-3.0f * p[4], y1 * y1, -p[3]);
    const float g2 = -p[0];
    // the angle grows without bound: reduce it in FP64 (in revolutions)
    const double turns = y[3] * kInvTwoPi;
    const float sn = sin_turns(turns), cs = cos_turns(turns);
    f[2] = r * sn * fmaf(1.0f + g1, cs, g2 * sn);
    f[3] = fmaf(fmaf(g1, cs, g2 * sn), cs, -sn * sn);
  }
};

// Keller-Miksis bubble model in the paper's dimensionless form, Sec. 2.2
// (numerator N_KM, denominator D_KM, coefficients C0..C12); t is tau.
// Time-only terms per stage: sin and cos of 2*pi*tau and of
// 2*pi*C11*tau + C12, each phase rounded as the plain expression is.
struct KellerMiksis {
  static constexpr int NS = 2;
  static constexpr int NP = 13;
  static constexpr int NF = 4;
  static constexpr int NQ = 14;
  static constexpr int ID = 2;
  template <int S>
  __device__ __forceinline__ static void forcing(const double (&ts)[S], const double (&C)[NP],
                                                 double (&F)[S][NF]) {
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const double w2 = __dmul_rn(kTwoPi, C[11]);
    double a1[S], a2[S], s1[S], c1[S], s2[S], c2[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      a1[k] = __dmul_rn(kTwoPi, ts[k]);
      a2[k] = __dadd_rn(__dmul_rn(w2, ts[k]), C[12]);
    }
    double s1b, c1b, s2b, c2b;
    sincos(a1[0], &s1b, &c1b);
    sincos(a2[0], &s2b, &c2b);
    stage_sincos<S>(a1, s1b, c1b, s1, c1);
    stage_sincos<S>(a2, s2b, c2b, s2, c2);
#pragma unroll
    for (int k = 0; k < S; ++k) {
      F[k][0] = s1[k];
      F[k][1] = c1[k];
      F[k][2] = s2[k];
      F[k][3] = c2[k];
    }
  }
  __device__ __forceinline__ static void rhs(const double (&y)[NS], const double (&C)[NP],
                                             const double (&F)[NF], double (&f)[NS]) {
    const double y1 = y[0], y2 = y[1];
    const double rx = 1.0 / y1;
    const double gas = pow(rx, C[10]);
    const double u = fma(C[9], y2, 1.0);                     // 1 + C9*y2
    const double forcing_p = fma(C[5], F[0], C[6] * F[2]);   // C5 sin + C6 sin
    const double forcing_d = fma(C[7], F[1], C[8] * F[3]);   // C7 cos + C8 cos
    const double inertia = fma(-C[9] * (1.0 / 3.0), y2, 1.0) * 1.5 * y2 * y2;
    double N = fma(C[1], y2, C[0]) * gas;
    N = fma(-C[2], u, N);
    N = fma(-fma(C[4], y2, C[3]), rx, N);
    N -= inertia;
    N = fma(-forcing_p, u, N);
    N = fma(-y1, forcing_d, N);
    const double D = fma(-C[9] * y1, y2, y1) + C[4] * C[9];
    f[0] = y2;
    f[1] = N / D;
  }
  template <int S>
  __device__ __forceinline__ static void forcing32(const double (&ts)[S], const double (&C)[NP],
                                                   float (&F)[S][NF]) {
    const double off = C[12] * kInvTwoPi;   // phase offset in revolutions
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const double r2 = fma(C[11], ts[k], off);
      F[k][0] = sin_turns(ts[k]);           // 2*pi*tau is tau revolutions
      F[k][1] = cos_turns(ts[k]);
      F[k][2] = sin_turns(r2);
      F[k][3] = cos_turns(r2);
    }
  }
  // FP32 parameters: C0..C12 and, in slot 13, the pressure imbalance at rest
  // E0 = C0 - C2 - C3 (zero up to rounding: the gas pressure balances the
  // static pressure and surface tension at R = R_E).
  __device__ __forceinline__ static void prepare32(const double (&C)[NP], float (&q)[NQ]) {
#pragma unroll
    for (int j = 0; j < NP; ++j) q[j] = static_cast<float>(C[j]);
    q[13] = static_cast<float>((C[0] - C[2]) - C[3]);
  }
  // Near rest the gas term C0 (R_E/R)^C10 and the static terms C2 + C3 R_E/R
  // are large (C0 reaches ~1e6 for micrometre bubbles at 20 kHz) and nearly
  // cancel, so FP32 rounding of each would swamp the net pressure.  They are
  // regrouped as C0 ((R_E/R)^C10 - 1) - C3 (R_E/R - 1) + E0 with
  // (R_E/R)^C10 - 1 = expm1(-C10 ln(1 + d)), d = y1 - 1 formed in FP64, so the
  // FP32 rounding error is proportional to the distance from rest.
  __device__ __forceinline__ static void rhs32(const double (&y)[NS], const float (&C)[NQ],
                                               const float (&F)[NF], float (&f)[NS]) {
    const float y1 = static_cast<float>(y[0]), y2 = static_cast<float>(y[1]);
    const float d = static_cast<float>(y[0] - 1.0);
    const float rx = __builtin_amdgcn_rcpf(y1);
    const float gas_m1 = expm1_32(-C[10] * log1p32(d));    // (R_E/R)^C10 - 1
    const float rx_m1 = -d * rx;                            // R_E/R - 1
    const float u = fmaf(C[9], y2, 1.0f);
    const float forcing_p = fmaf(C[5], F[0], C[6] * F[2]);
    const float forcing_d = fmaf(C[7], F[1], C[8] * F[3]);
    const float inertia = fmaf(-C[9] * (1.0f / 3.0f), y2, 1.0f) * 1.5f * y2 * y2;
    // rest balance + the y2 terms of (C0 + C1 y2) gas - C2 (1 + C9 y2)
    float N = fmaf(C[0], gas_m1, fmaf(-C[3], rx_m1, C[13]));
    N = fmaf(y2, fmaf(C[1], 1.0f + gas_m1, -C[2] * C[9]), N);
    N = fmaf(-C[4] * y2, rx, N);
    N -= inertia;
    N = fmaf(-forcing_p, u, N);
    N = fmaf(-y1, forcing_d, N);
    const float D = fmaf(-C[9] * y1, y2, y1) + C[4] * C[9];
    f[0] = y2;
    f[1] = N * __builtin_amdgcn_rcpf(D);
  }
};

// Pressure relief valve, paper Sec. 2.3 Eqs. (29)-(31):
// p = (kappa, delta, beta, q, r); r is read by the impact action only.
struct ReliefValve {
  static constexpr int NS = 3;
  static constexpr int NP = 5;
  static constexpr int NF = 0;
  static constexpr int NQ = 5;
  static constexpr int ID = 3;
  template <int S>
  __device__ __forceinline__ static void forcing(const double (&)[S], const double (&)[NP],
                                                 double (&)[S][1]) {}
  __device__ __forceinline__ static void rhs(const double (&y)[NS], const double (&p)[NP],
                                             const double (&)[1], double (&f)[NS]) {
    f[0] = y[1];
    f[1] = fma(-p[0], y[1], y[2] - (y[0] + p[1]));
    f[2] = p[2] * fma(-y[0], sqrt(y[2]), p[3]);
  }
  template <int S>
  __device__ __forceinline__ static void forcing32(const double (&)[S], const double (&)[NP],
                                                   float (&)[S][1]) {}
  __device__ __forceinline__ static void prepare32(const double (&p)[NP], float (&q)[NQ]) {
#pragma unroll
    for (int j = 0; j < NQ; ++j) q[j] = static_cast<float>(p[j]);
  }
  __device__ __forceinline__ static void rhs32(const double (&yd)[NS], const float (&p)[NQ],
                                               const float (&)[1], float (&f)[NS]) {
    const float y[NS] = {static_cast<float>(yd[0]), static_cast<float>(yd[1]),
                         static_cast<float>(yd[2])};
    f[0] = y[1];
    f[1] = fmaf(-p[0], y[1], y[2] - (y[0] + p[1]));
    f[2] = p[2] * fmaf(-y[0], sqrtf(y[2]), p[3]);
  }
};

// Free flight under gravity (test model): y1' = y2, y2' = -g.
struct Ballistic {
  static constexpr int NS = 2;
  static constexpr int NP = 1;
  static constexpr int NF = 0;
  static constexpr int NQ = 1;
  static constexpr int ID = 4;
  template <int S>
  __device__ __forceinline__ static void forcing(const double (&)[S], const double (&)[NP],
                                                 double (&)[S][1]) {}
  __device__ __forceinline__ static void rhs(const double (&y)[NS], const double (&p)[NP],
                                             const double (&)[1], double (&f)[NS]) {
    f[0] = y[1];
    f[1] = -p[0];
  }
  template <int S>
  __device__ __forceinline__ static void forcing32(const double (&)[S], const double (&)[NP],
                                                   float (&)[S][1]) {}
  __device__ __forceinline__ static void prepare32(const double (&p)[NP], float (&q)[NQ]) {
    q[0] = static_cast<float>(p[0]);
  }
  __device__ __forceinline__ static void rhs32(const double (&y)[NS], const float (&p)[NQ],
                                               const float (&)[1], float (&f)[NS]) {
    f[0] = static_cast<float>(y[1]);
    f[1] = -p[0];
  }
};

}  // namespace odeens
