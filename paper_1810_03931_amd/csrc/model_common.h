// Building blocks shared by the model right-hand sides (model_*.h).
//
// Each model is a compile-time type, so the integrator kernel is specialised
// per model and the right-hand side is inlined into the stage loop (the paper
// keeps its device functions in the kernel's translation unit for the same
// reason, Sec. 6.9).  Each model header is included only by its own kernel
// translation unit.
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

// sin and cos of x.  Cody-Waite reduction modulo pi/2: x = k pi/2 + r, with
// pi/2 split into three doubles; the first product is exact inside the FMA
// (x - k C1 needs at most 53 bits), and the reduced argument is carried as
// r + rr.  On |r| <= pi/4 the Taylor series through r^17 (sine) and r^16
// (cosine) truncate below 1e-19; cos r = (1 - r^2/2) + ... keeps the rounding
// error of the leading subtraction.  The quadrant k mod 4 swaps and negates.
// Measured against 60-digit values: p99 0.57 ulp, at most 0.7 ulp away from
// the zeros (relative error up to 1.13 ulp right next to them, i.e. below
// 1e-29 absolute).  Beyond |x| = 1e6 the library routine is used.  Also
// compiled for the host, where a test checks these bounds against 60-digit
// values.
__host__ __device__ __forceinline__ void sincos_cw(double x, double &s, double &c) {
  if (!(fabs(x) <= 1e6)) {
    sincos(x, &s, &c);
    return;
  }
  constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
  constexpr double kC1 = 0x1.921fb54442d18p+0;    // pi/2 rounded
  constexpr double kC2 = 0x1.1a62633145c07p-54;   // pi/2 - kC1 rounded
  constexpr double kC3 = -0x1.f1976b7ed8fbcp-110; // pi/2 - kC1 - kC2 rounded
  const double k = rint(x * kTwoOverPi);
  const double rh = fma(-k, kC1, x);
  const double r = fma(-k, kC2, rh);
  const double rr = fma(-k, kC3, fma(-k, kC2, rh - r));
  // The series are summed in the power basis, smallest term first: each
  // step adds to the running sum (an FMA whose addend is not a constant, so
  // no coefficient has to be copied into the destination register first).
  const double r2 = r * r;
  const double r4 = r2 * r2, r6 = r4 * r2, r8 = r4 * r4;
  const double r10 = r8 * r2, r12 = r8 * r4, r14 = r12 * r2;
  double ps = (1.0 / 355687428096000.0) * r14;  //  1/17!
  ps = fma(-1.0 / 1307674368000.0, r12, ps);    // -1/15!
  ps = fma(1.0 / 6227020800.0, r10, ps);        //  1/13!
  ps = fma(-1.0 / 39916800.0, r8, ps);          // -1/11!
  ps = fma(1.0 / 362880.0, r6, ps);             //  1/9!
  ps = fma(-1.0 / 5040.0, r4, ps);              // -1/7!
  ps = fma(1.0 / 120.0, r2, ps);                //  1/5!
  ps = ps + (-1.0 / 6.0);                       // -1/3!
  const double sr = r + fma(r * r2, ps, fma(-0.5 * r2, rr, rr));
  double pc = (1.0 / 20922789888000.0) * r12;   //  1/16!
  pc = fma(-1.0 / 87178291200.0, r10, pc);      // -1/14!
  pc = fma(1.0 / 479001600.0, r8, pc);          //  1/12!
  pc = fma(-1.0 / 3628800.0, r6, pc);           // -1/10!
  pc = fma(1.0 / 40320.0, r4, pc);              //  1/8!
  pc = fma(-1.0 / 720.0, r2, pc);               // -1/6!
  pc = pc + 1.0 / 24.0;                         //  1/4!
  const double hr = 0.5 * r2;
  const double w = 1.0 - hr;
  const double cr = w + (((1.0 - w) - hr) + fma(r4, pc, -r * rr));
  const int q = static_cast<int>(k);
  const double s1 = (q & 1) ? cr : sr;
  const double c1 = (q & 1) ? sr : cr;
  s = (q & 2) ? -s1 : s1;
  c = ((q + 1) & 2) ? -c1 : c1;
}

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
// the full evaluation is used.
__device__ __forceinline__ void sincos_near(double arg, double base, double sb, double cb,
                                            double &s, double &c) {
  constexpr double kQuarterPi = 0.78539816339744830962;
  const double delta = __dsub_rn(arg, base);
  if (fabs(delta) <= kQuarterPi) {
    rotate(delta, sb, cb, s, c);
  } else {
    sincos_cw(arg, s, c);
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

}  // namespace odeens
