// Integrator kernels specialised for the KellerMiksis model (one translation unit
// per model so the instantiations compile in parallel).
#include "integrator_kernel.h"
#include "model_keller_miksis.h"

namespace odeens {

const void *kernels_keller_miksis(int method, int prec, int nev, int nacc, int comp) {
  return ModelKernels<KellerMiksis>::get(method, prec, nev, nacc, comp);
}

}  // namespace odeens
