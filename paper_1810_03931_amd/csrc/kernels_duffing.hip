// Integrator kernels specialised for the Duffing model (one translation unit
// per model so the instantiations compile in parallel).
#include "integrator_kernel.h"
#include "model_duffing.h"

namespace odeens {

const void *kernels_duffing(int method, int prec, int nev, int nacc, int comp) {
  return ModelKernels<Duffing>::get(method, prec, nev, nacc, comp);
}

}  // namespace odeens
