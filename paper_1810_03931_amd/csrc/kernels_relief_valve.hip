// Integrator kernels specialised for the ReliefValve model (one translation unit
// per model so the instantiations compile in parallel).
#include "integrator_kernel.h"
#include "model_relief_valve.h"

namespace odeens {

const void *kernels_relief_valve(int method, int prec, int nev, int nacc, int comp) {
  return ModelKernels<ReliefValve>::get(method, prec, nev, nacc, comp);
}

}  // namespace odeens
