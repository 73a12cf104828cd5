#pragma once

#include "model_common.h"

namespace odeens {

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
