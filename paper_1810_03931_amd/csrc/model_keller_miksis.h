#pragma once

#include "model_common.h"

namespace odeens {

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
    sincos_cw(a1[0], s1b, c1b);
    sincos_cw(a2[0], s2b, c2b);
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
    const double gas = pow_pos(rx, C[10]);
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

}  // namespace odeens
