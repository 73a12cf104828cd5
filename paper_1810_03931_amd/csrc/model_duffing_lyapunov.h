#pragma once

#include "model_common.h"
#include "model_duffing.h"

namespace odeens {

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

}  // namespace odeens
