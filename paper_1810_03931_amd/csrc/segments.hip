// Small kernels around the solves: the next segment's end time of a
// repeated-horizon sequence, the per-segment snapshot of state and
// accessories, and the shortened time domain of an autotuning probe.  All are
// one thread per listed system with coalesced SoA accesses.
#include "integrator.h"

namespace odeens {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t system_of(const int64_t *index, int64_t q) {
  return index ? index[q] : q;
}

__global__ void __launch_bounds__(kThreads)
set_horizon(double *td, int64_t ld, int64_t n, const int64_t *index, double segment) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= n) return;
  const int64_t s = system_of(index, q);
  if (s < 0 || s >= ld) return;
  td[ld + s] = td[s] + segment;
}

__global__ void __launch_bounds__(kThreads)
probe_horizon(const double *src, double *dst, int64_t ld, int64_t n, const int64_t *index,
              double fraction) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= n) return;
  const int64_t s = system_of(index, q);
  if (s < 0 || s >= ld) return;
  const double t0 = src[s], t1 = src[ld + s];
  dst[s] = t0;
  dst[ld + s] = fraction == 1.0 ? t1 : t0 + fraction * (t1 - t0);
}

__global__ void __launch_bounds__(kThreads)
snapshot(const double *y, int n_state, const double *acc, int n_acc_rows, int64_t ld, int64_t n,
         const int64_t *index, double *out) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= n) return;
  const int64_t s = system_of(index, q);
  if (s < 0 || s >= ld) return;
  for (int i = 0; i < n_state; ++i) out[i * ld + s] = y[i * ld + s];
  for (int r = 0; r < n_acc_rows; ++r) out[(n_state + r) * ld + s] = acc[r * ld + s];
}

unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_set_horizon(double *td, int64_t ld, int64_t n, const int64_t *index,
                              double segment, hipStream_t stream) {
  hipLaunchKernelGGL(set_horizon, dim3(grid_for(n)), dim3(kThreads), 0, stream, td, ld, n, index,
                     segment);
  return hipGetLastError();
}

hipError_t launch_probe_horizon(const double *td_src, double *td_dst, int64_t ld, int64_t n,
                                const int64_t *index, double fraction, hipStream_t stream) {
  hipLaunchKernelGGL(probe_horizon, dim3(grid_for(n)), dim3(kThreads), 0, stream, td_src, td_dst,
                     ld, n, index, fraction);
  return hipGetLastError();
}

hipError_t launch_snapshot(const double *y, int n_state, const double *acc, int n_acc_rows,
                           int64_t ld, int64_t n, const int64_t *index, double *out,
                           hipStream_t stream) {
  hipLaunchKernelGGL(snapshot, dim3(grid_for(n)), dim3(kThreads), 0, stream, y, n_state, acc,
                     n_acc_rows, ld, n, index, out);
  return hipGetLastError();
}

}  // namespace odeens
