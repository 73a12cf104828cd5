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

// x^c for x > 0 as exp(c ln x), with ln x carried in two doubles so that
// the product c ln x keeps about 2^-100 relative accuracy.
//  * ln x: x = 2^e m with m in [1/sqrt 2, sqrt 2); u = (m - 1)/(m + 1) as
//    u_hi + u_lo (m + 1 is formed exactly as two doubles, the quotient is
//    corrected by its FMA residual); ln m = 2 atanh u = 2u + 2u^3 P(u^2),
//    P through u^18/21 (|u| <= 0.1716, truncation below 1e-18 relative);
//    e ln 2 with ln 2 split in a 32-bit head (exact products) and a tail.
//  * exp: z = n ln 2 + r, |r| <= ln(2)/2, r carried with its low part;
//    exp(r) = 1 + r + r^2 Q(r), Q through r^13/13! (truncation below 5e-18);
//    the result is scaled by 2^n.
// Measured against 60-digit values for x in [1e-3, 1e3] and c in [0, 8]
// (a test compiles this same source for the host): within 1 ulp, 0.26 ulp on
// average; 91% of the results equal the C library's pow at c = 4.2.
// Overflow gives infinity; results below the normal range are rounded twice
// (an error of up to one unit of the subnormal).  Other operands -- a zero,
// negative, infinite or NaN base, or a non-finite exponent -- get the values
// the C library defines (pow_special); the models' physical states never
// reach them.
__host__ __device__ __forceinline__ double pow_special(double x, double c) {
  constexpr double kInf = __builtin_huge_val();
  if (x != x || c != c) return (x == 1.0 || c == 0.0) ? 1.0 : x + c;  // NaN
  if (c == 0.0) return 1.0;
  if (fabs(c) == kInf) {
    const double ax = fabs(x);
    if (ax == 1.0) return 1.0;
    return ((ax > 1.0) == (c > 0.0)) ? kInf : 0.0;
  }
  const bool odd = c == rint(c) && rint(0.5 * c) != 0.5 * c;  // an odd integer
  if (x == 0.0) return c > 0.0 ? (odd ? x : 0.0) : (odd ? 1.0 / x : kInf);
  if (x == -kInf) return c > 0.0 ? (odd ? -kInf : kInf) : (odd ? -0.0 : 0.0);
  if (x == kInf) return c > 0.0 ? kInf : 0.0;
  return (x - x) / (x - x);                    // NaN (finite negative bases: pow_pos)
}

// The constants of pow_pos.  On the device they are read from a table in
// constant memory through an opaque scalar pointer.  An FP64 constant that is
// not an inline operand otherwise costs two scalar moves (one per 32-bit half)
// at every use, since the compiler rematerialises it rather than keep it live,
// and a wave that runs alone pays an issue slot for each: the Keller-Miksis
// right-hand side calls pow_pos at every stage, and the slowest system of that
// sweep takes 20% less time per attempt with the table (a few merged scalar
// loads per call, issued ahead of the series that need them).  The same
// treatment of the sine/cosine coefficients was slower: those loads come at the
// start of every attempt, where nothing hides their latency.  The host build
// (the tests compile this header for the CPU) reads a plain array.
#define ODE_POW_CONSTANTS(X)                                                       \
  X(kPowLn2Hi, 0x1.62e42fee00000p-1) /* ln 2, 32 significant bits */                \
  X(kPowLn2Lo, 0x1.a39ef35793c76p-33) /* ln 2 - kPowLn2Hi */                         \
  X(kPowInvLn2, 0x1.71547652b82fep+0)                                               \
  X(kPowSqrtHalf, 0x1.6a09e667f3bcdp-1)                                             \
  X(kPowOver, 709.8)                                                                \
  X(kPowUnder, -745.2)                                                              \
  X(kPowP3, 1.0 / 3.0) X(kPowP5, 1.0 / 5.0) X(kPowP7, 1.0 / 7.0) X(kPowP9, 1.0 / 9.0)  \
  X(kPowP11, 1.0 / 11.0) X(kPowP13, 1.0 / 13.0) X(kPowP15, 1.0 / 15.0)              \
  X(kPowP17, 1.0 / 17.0) X(kPowP19, 1.0 / 19.0) X(kPowP21, 1.0 / 21.0)              \
  X(kPowQ3, 1.0 / 6.0) X(kPowQ4, 1.0 / 24.0) X(kPowQ5, 1.0 / 120.0)                 \
  X(kPowQ6, 1.0 / 720.0) X(kPowQ7, 1.0 / 5040.0) X(kPowQ8, 1.0 / 40320.0)           \
  X(kPowQ9, 1.0 / 362880.0) X(kPowQ10, 1.0 / 3628800.0)                             \
  X(kPowQ11, 1.0 / 39916800.0) X(kPowQ12, 1.0 / 479001600.0)                        \
  X(kPowQ13, 1.0 / 6227020800.0)

enum PowConstant : int {
#define ODE_POW_NAME(name, value) name,
  ODE_POW_CONSTANTS(ODE_POW_NAME)
#undef ODE_POW_NAME
  kPowConstants
};

#if defined(__HIP_DEVICE_COMPILE__)
static __device__ __constant__ double kPowTable[kPowConstants] = {
#define ODE_POW_VALUE(name, value) value,
    ODE_POW_CONSTANTS(ODE_POW_VALUE)
#undef ODE_POW_VALUE
};
typedef const __attribute__((address_space(4))) double *PowTableRef;
__device__ __forceinline__ PowTableRef pow_table() {
  PowTableRef t = (PowTableRef)kPowTable;
  asm volatile("" : "+s"(t));   // opaque: every call loads, no value is folded
  return t;
}
#else
static constexpr double kPowTable[kPowConstants] = {
#define ODE_POW_VALUE(name, value) value,
    ODE_POW_CONSTANTS(ODE_POW_VALUE)
#undef ODE_POW_VALUE
};
typedef const double *PowTableRef;
inline PowTableRef pow_table() { return kPowTable; }
#endif

// 2^n * v for an integral n; n outside the int range (where the result is
// replaced anyway) is clamped first, so the conversion is always defined.
__host__ __device__ __forceinline__ double scale_by_pow2(double v, double n) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ldexp(v, static_cast<int>(n));   // the hardware conversion saturates
#else
  return ldexp(v, static_cast<int>(fmin(fmax(n, -4096.0), 4096.0)));
#endif
}

// 1/d, correctly rounded, for 1 <= d < 4.  On the device: the hardware
// reciprocal refined by two Newton steps and the quotient corrected by its
// FMA residual -- the steps of the compiler's division sequence, without the
// operand scaling and special-case fix-up that a divisor in this range never
// needs, so the result is the same as that of 1.0 / d.
__host__ __device__ __forceinline__ double recip_1_to_4(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  const double q = r;                      // 1.0 * r
  return fma(fma(-d, q, 1.0), r, q);
#else
  return 1.0 / d;
#endif
}

// The main path runs for every operand and the special cases replace its
// result at the end (selects, one branch for pow_special), so a wave pays no
// branch and exec-mask bookkeeping for cases its lanes never reach.
__host__ __device__ __forceinline__ double pow_pos(double x, double c) {
  constexpr double kInf = __builtin_huge_val();
  // a finite negative base is defined for integer exponents: |x|^c, negated
  // for odd c
  const bool neg_ok = x < 0.0 && x > -kInf && c == rint(c);
  const bool ordinary = ((x > 0.0 && x < kInf) || neg_ok) && fabs(c) < kInf;
  const bool negate = neg_ok && rint(0.5 * c) != 0.5 * c;   // an odd integer
  const double ax = ordinary ? fabs(x) : 1.0;
  const PowTableRef T = pow_table();
  const double kLn2Hi = T[kPowLn2Hi], kLn2Lo = T[kPowLn2Lo];
  int e = 0;
  double m = frexp(ax, &e);                           // m in [1/2, 1)
  if (m < T[kPowSqrtHalf]) {                          // below 1/sqrt 2
    m = m + m;
    e -= 1;
  }
  const double f = m - 1.0;                           // exact
  const double dh = m + 1.0;
  const double dl = m - (dh - 1.0);                   // m + 1 = dh + dl exactly
  const double rd = recip_1_to_4(dh);
  const double uh = f * rd;
  const double ul = (fma(-uh, dh, f) - uh * dl) * rd;
  // P(w) = sum_k w^k / (2k + 3), k = 0..9, w = u^2, in three blocks of
  // powers (each coefficient multiplies a power, so no constant has to be
  // copied into an accumulator register first)
  const double w = uh * uh, w2 = w * w, w3 = w2 * w, w4 = w2 * w2;
  const double pa = fma(T[kPowP5], w, fma(T[kPowP7], w2, T[kPowP9] * w3)) + T[kPowP3];
  const double pb = fma(T[kPowP13], w, fma(T[kPowP15], w2, T[kPowP17] * w3)) + T[kPowP11];
  const double pc = T[kPowP21] * w + T[kPowP19];
  const double p = fma(w4, fma(w4, pc, pb), pa);
  const double tail = (2.0 * uh * w) * p;             // 2u^3 P(u^2)
  const double ed = static_cast<double>(e);
  const double a = ed * kLn2Hi;                       // exact
  const double b = 2.0 * uh;
  const double s = a + b;                             // |a| >= |b| or a == 0
  const double lo = ((b - (s - a)) + fma(ed, kLn2Lo, fma(2.0, ul, tail)));
  const double lh = s + lo;
  const double ll = lo - (lh - s);
  const double zh = c * lh;
  const double zl = fma(c, lh, -zh) + c * ll;
  const double n = rint(zh * T[kPowInvLn2]);
  const double rh = fma(-n, kLn2Hi, zh);              // exact
  const double t = fma(-n, kLn2Lo, zl);
  const double r = rh + t;
  const double rl = (rh - r) + t;
  // Q(r) = sum_k r^k / (k + 2)!, k = 0..11, in blocks as P above
  const double r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
  const double qa = fma(T[kPowQ3], r, fma(T[kPowQ4], r2, T[kPowQ5] * r3)) + 0.5;
  const double qb = fma(T[kPowQ7], r, fma(T[kPowQ8], r2, T[kPowQ9] * r3)) + T[kPowQ6];
  const double qc = fma(T[kPowQ11], r, fma(T[kPowQ12], r2, T[kPowQ13] * r3)) + T[kPowQ10];
  const double q = fma(r4, fma(r4, qc, qb), qa);
  const double em1 = fma(r2, q, r);                   // exp(r) - 1
  const double v = 1.0 + fma(em1, rl, em1 + rl);      // exp(r + rl)
  double res = scale_by_pow2(v, n);
  res = (zh > T[kPowOver]) ? kInf : res;              // overflow
  res = (zh < T[kPowUnder]) ? 0.0 : res;              // below the subnormals
  res = negate ? -res : res;
  if (!ordinary) res = pow_special(x, c);
  return res;
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
// lanes of a wave normally agree) the short rotation serves all stages; it is
// evaluated unconditionally and replaced in the rare other case, so the
// common path carries no if/else around it.
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
#pragma unroll
  for (int k = 1; k < S; ++k) rotate_short(d[k], sb, cb, s[k], c[k]);
  if (!(dmax <= kShortRotate)) {
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
