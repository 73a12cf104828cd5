// Right-hand sides f(t, y; p) of the built-in models, as device functors.
// Each model is a compile-time type, so the integrator kernel is specialised
// per model and the right-hand side is inlined into the stage loop (the paper
// keeps its device functions in the kernel's translation unit for the same
// reason, Sec. 6.9).
#pragma once

#include <hip/hip_runtime.h>

namespace odeens {

// Duffing oscillator, paper Sec. 2.1 Eqs. (1)-(2), with linear and cubic
// stiffness as parameters: p = (k, B, omega, lin, cub),
//   y1' = y2,  y2' = -lin*y1 - cub*y1^3 - k*y2 + B*cos(omega*t).
struct Duffing {
  static constexpr int NS = 2;
  static constexpr int NP = 5;
  static constexpr int ID = 1;
  __device__ __forceinline__ static void rhs(double t, const double (&y)[NS], const double (&p)[NP],
                                             double (&f)[NS]) {
    const double y1 = y[0], y2 = y[1];
    const double forcing = p[1] * cos(p[2] * t);
    const double spring = fma(p[4] * y1 * y1, y1, fma(p[3], y1, p[0] * y2));
    f[0] = y2;
    f[1] = forcing - spring;
  }
};

// Keller-Miksis bubble model in the paper's dimensionless form, Sec. 2.2
// (numerator N_KM, denominator D_KM, coefficients C0..C12); t is tau.
struct KellerMiksis {
  static constexpr int NS = 2;
  static constexpr int NP = 13;
  static constexpr int ID = 2;
  __device__ __forceinline__ static void rhs(double tau, const double (&y)[NS],
                                             const double (&C)[NP], double (&f)[NS]) {
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const double y1 = y[0], y2 = y[1];
    const double rx = 1.0 / y1;
    const double gas = pow(rx, C[10]);
    double s1, c1, s2, c2;
    sincos(kTwoPi * tau, &s1, &c1);
    // phase 2*pi*C11*tau + C12 rounded as written: |phase| reaches ~1e5, where
    // one ulp of difference would already move sin/cos by ~1e-11
    sincos(__dadd_rn(__dmul_rn(__dmul_rn(kTwoPi, C[11]), tau), C[12]), &s2, &c2);
    const double u = fma(C[9], y2, 1.0);                 // 1 + C9*y2
    const double forcing_p = fma(C[5], s1, C[6] * s2);   // C5 sin + C6 sin
    const double forcing_d = fma(C[7], c1, C[8] * c2);   // C7 cos + C8 cos
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
};

// Pressure relief valve, paper Sec. 2.3 Eqs. (29)-(31):
// p = (kappa, delta, beta, q, r); r is read by the impact action only.
struct ReliefValve {
  static constexpr int NS = 3;
  static constexpr int NP = 5;
  static constexpr int ID = 3;
  __device__ __forceinline__ static void rhs(double, const double (&y)[NS], const double (&p)[NP],
                                             double (&f)[NS]) {
    f[0] = y[1];
    f[1] = fma(-p[0], y[1], y[2] - (y[0] + p[1]));
    f[2] = p[2] * fma(-y[0], sqrt(y[2]), p[3]);
  }
};

// Free flight under gravity (test model): y1' = y2, y2' = -g.
struct Ballistic {
  static constexpr int NS = 2;
  static constexpr int NP = 1;
  static constexpr int ID = 4;
  __device__ __forceinline__ static void rhs(double, const double (&y)[NS], const double (&p)[NP],
                                             double (&f)[NS]) {
    f[0] = y[1];
    f[1] = -p[0];
  }
};

}  // namespace odeens
