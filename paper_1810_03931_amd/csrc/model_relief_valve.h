#pragma once

#include "model_common.h"

namespace odeens {

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

}  // namespace odeens
