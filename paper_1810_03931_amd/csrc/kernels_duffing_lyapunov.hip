// Integrator kernels specialised for the Duffing model with its polar
// linearisation (Lyapunov exponents); one translation unit per model so the
// instantiations compile in parallel.
#include "integrator_kernel.h"
#include "model_duffing_lyapunov.h"

namespace odeens {

const void *kernels_duffing_lyapunov(int method, int prec, int nev, int nacc, int comp) {
  return ModelKernels<DuffingLyapunov>::get(method, prec, nev, nacc, comp);
}

}  // namespace odeens
