// Integrator kernels specialised for the Ballistic model (one translation unit
// per model so the instantiations compile in parallel).
#include "integrator_kernel.h"
#include "model_ballistic.h"

namespace odeens {

const void *kernels_ballistic(int method, int prec, int nev, int nacc, int comp) {
  return ModelKernels<Ballistic>::get(method, prec, nev, nacc, comp);
}

}  // namespace odeens
