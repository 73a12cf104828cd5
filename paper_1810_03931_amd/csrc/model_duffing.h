#pragma once

#include "model_common.h"

namespace odeens {

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
    sincos_cw(arg[0], sb, cb);
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

}  // namespace odeens
