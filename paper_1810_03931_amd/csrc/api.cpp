// C ABI of the ensemble integrator: argument validation, handle management
// and kernel launch.  Declarations and the contract are in ode_ensemble.h.
#include "ode_ensemble.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "integrator.h"

namespace odeens {
const void *kernels_duffing(int method, int prec, int nev, int nacc);
const void *kernels_keller_miksis(int method, int prec, int nev, int nacc);
const void *kernels_relief_valve(int method, int prec, int nev, int nacc);
const void *kernels_ballistic(int method, int prec, int nev, int nacc);

const void *integrator_kernel(int model, int method, int prec, int nev, int nacc) {
  switch (model) {
    case ODE_MODEL_DUFFING: return kernels_duffing(method, prec, nev, nacc);
    case ODE_MODEL_KELLER_MIKSIS: return kernels_keller_miksis(method, prec, nev, nacc);
    case ODE_MODEL_RELIEF_VALVE: return kernels_relief_valve(method, prec, nev, nacc);
    case ODE_MODEL_BALLISTIC: return kernels_ballistic(method, prec, nev, nacc);
    default: return nullptr;
  }
}

hipError_t launch_integrator(int model, int method, int prec, int nev, int nacc,
                             const Params &prm, int grid, int block, hipStream_t stream) {
  const void *fn = integrator_kernel(model, method, prec, nev, nacc);
  if (!fn) return hipErrorInvalidDeviceFunction;
  Params pp = prm;
  void *args[] = {&pp};
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, stream);
}
}  // namespace odeens

using namespace odeens;

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int hip_fail(hipError_t err, const char *what) {
  return fail(ODE_EHIP, "%s: %s", what, hipGetErrorString(err));
}

bool model_dims(int32_t model, int32_t *ns, int32_t *np) {
  switch (model) {
    case ODE_MODEL_DUFFING: *ns = 2; *np = 5; return true;
    case ODE_MODEL_KELLER_MIKSIS: *ns = 2; *np = 13; return true;
    case ODE_MODEL_RELIEF_VALVE: *ns = 3; *np = 5; return true;
    case ODE_MODEL_BALLISTIC: *ns = 2; *np = 1; return true;
    default: return false;
  }
}

constexpr int kDefaultBlock = 256;
constexpr int kCombos = 9;  // (event slots 0/1/4) x (accessory slots 0/2/4)

int combo_index(int nev, int nacc) {
  const int e = nev == 0 ? 0 : (nev == 1 ? 1 : 2);
  const int k = nacc == 0 ? 0 : (nacc == 2 ? 1 : 2);
  return e * 3 + k;
}

}  // namespace

struct ode_ensemble {
  int32_t model, method, precision, block;
  int32_t n_state, n_param;
  int device;
  int compute_units;
  int blocks_per_cu[kCombos];  // 0 = not yet queried
  int last_blocks_per_cu, last_grid;
  unsigned long long *queue;   // device: [0] next position, [1] finished waves
};

extern "C" {

const char *ode_ensemble_last_error(void) { return g_error.c_str(); }

int ode_ensemble_model_dims(int32_t model, int32_t *n_state, int32_t *n_param) {
  int32_t ns, np;
  if (!model_dims(model, &ns, &np)) return fail(ODE_EINVAL, "unknown model %d", model);
  if (n_state) *n_state = ns;
  if (n_param) *n_param = np;
  return ODE_OK;
}

int ode_ensemble_create(const ode_ensemble_desc *desc, ode_ensemble **out) {
  if (!out) return fail(ODE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(ODE_EINVAL, "desc is NULL");
  int32_t ns, np;
  if (!model_dims(desc->model, &ns, &np)) return fail(ODE_EINVAL, "unknown model %d", desc->model);
  if (desc->method != ODE_RKCK45 && desc->method != ODE_RK4)
    return fail(ODE_EINVAL, "unknown method %d", desc->method);
  if (desc->precision != ODE_FP64 && desc->precision != ODE_FP32_STAGES)
    return fail(ODE_EINVAL, "unknown precision %d", desc->precision);
  int block = desc->block_size == 0 ? kDefaultBlock : desc->block_size;
  if (block < 64 || block > kMaxBlock || block % 64 != 0)
    return fail(ODE_EINVAL, "block_size %d must be a multiple of 64 in [64, %d]",
                desc->block_size, kMaxBlock);

  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
  int cus = 0;
  err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (err != hipSuccess) return hip_fail(err, "hipDeviceGetAttribute");

  auto *e = static_cast<ode_ensemble *>(std::calloc(1, sizeof(ode_ensemble)));
  if (!e) return fail(ODE_ENOMEM, "host allocation failed");
  e->model = desc->model;
  e->method = desc->method;
  e->precision = desc->precision;
  e->block = block;
  e->n_state = ns;
  e->n_param = np;
  e->device = dev;
  e->compute_units = cus;
  err = hipMalloc(reinterpret_cast<void **>(&e->queue), 2 * sizeof(unsigned long long));
  if (err != hipSuccess) {
    std::free(e);
    return fail(ODE_ENOMEM, "hipMalloc of the work queue: %s", hipGetErrorString(err));
  }
  // Zeroed once here; afterwards every launch leaves the counters at zero
  // (the last wave to finish resets them).
  err = hipMemset(e->queue, 0, 2 * sizeof(unsigned long long));
  if (err == hipSuccess) err = hipDeviceSynchronize();
  if (err != hipSuccess) {
    (void)hipFree(e->queue);
    std::free(e);
    return hip_fail(err, "clearing the work queue");
  }
  *out = e;
  return ODE_OK;
}

void ode_ensemble_destroy(ode_ensemble *e) {
  if (!e) return;
  if (e->queue) (void)hipFree(e->queue);
  std::free(e);
}

static int query_blocks(ode_ensemble *e, int nev, int nacc, int *out) {
  int &slot = e->blocks_per_cu[combo_index(nev, nacc)];
  if (slot == 0) {
    const void *fn = integrator_kernel(e->model, e->method, e->precision, nev, nacc);
    if (!fn) return fail(ODE_ENOTSUP, "no kernel for this model/method");
    int nb = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, e->block, 0);
    if (err != hipSuccess) return hip_fail(err, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    slot = nb > 0 ? nb : 1;
  }
  *out = slot;
  return ODE_OK;
}

int ode_ensemble_query(const ode_ensemble *e, ode_ensemble_info *info) {
  if (!e || !info) return fail(ODE_EINVAL, "NULL argument");
  auto *m = const_cast<ode_ensemble *>(e);
  int bpc = e->last_blocks_per_cu;
  if (bpc == 0) {
    int rc = query_blocks(m, 0, 0, &bpc);
    if (rc != ODE_OK) return rc;
  }
  info->block_size = e->block;
  info->blocks_per_cu = bpc;
  info->compute_units = e->compute_units;
  info->max_grid = bpc * e->compute_units;
  info->resident_systems = (int64_t)bpc * e->compute_units * e->block;
  return ODE_OK;
}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

static int validate(const ode_ensemble *e, const ode_solve_args *a) {
  const int ns = e->n_state, np = e->n_param;
  if (a->n_systems < 0) return fail(ODE_EINVAL, "n_systems < 0");
  if (a->system_index) {
    if (a->ld < 1) return fail(ODE_EINVAL, "ld must be >= 1");
  } else if (a->ld < a->n_systems) {
    return fail(ODE_EINVAL, "ld (%lld) < n_systems (%lld)", (long long)a->ld,
                (long long)a->n_systems);
  }
  if (a->ld > (int64_t(1) << 40)) return fail(ODE_EINVAL, "ld too large");
  const bool work = a->n_systems > 0;  // with no systems nothing is read or written
  if (work && (!a->time_domain || !a->state || !a->status))
    return fail(ODE_EINVAL, "time_domain, state and status are required");
  if (work && np > 0 && !a->params) return fail(ODE_EINVAL, "params is required");
  if (a->n_events < 0 || a->n_events > ODE_MAX_EVENTS)
    return fail(ODE_EINVAL, "n_events must be in [0, %d]", ODE_MAX_EVENTS);
  if (a->n_accessories < 0 || a->n_accessories > ODE_MAX_ACCESSORIES)
    return fail(ODE_EINVAL, "n_accessories must be in [0, %d]", ODE_MAX_ACCESSORIES);
  if (work && a->n_accessories > 0 && !a->accessories)
    return fail(ODE_EINVAL, "accessories array is NULL but n_accessories > 0");
  if (a->event_record_capacity < 0) return fail(ODE_EINVAL, "event_record_capacity < 0");
  if (work && (a->event_record_capacity > 0) != (a->event_records != nullptr))
    return fail(ODE_EINVAL, "event_records must be given exactly when the capacity is > 0");
  if (!finite_pos(a->h0)) return fail(ODE_EINVAL, "h0 must be finite and > 0");
  if (a->max_steps < 1 || a->max_steps > ODE_MAX_STEPS_LIMIT)
    return fail(ODE_EINVAL, "max_steps must be in [1, %lld]", (long long)ODE_MAX_STEPS_LIMIT);
  if (a->max_equilibrium_steps < 0) return fail(ODE_EINVAL, "max_equilibrium_steps < 0");
  if (std::isnan(a->t_record)) return fail(ODE_EINVAL, "t_record is NaN");
  if (e->method == ODE_RKCK45) {
    if (!finite_pos(a->h_min)) return fail(ODE_EINVAL, "h_min must be finite and > 0");
    if (!(a->h_max >= a->h_min)) return fail(ODE_EINVAL, "h_max < h_min");
    if (!(a->grow >= 1.0) || !std::isfinite(a->grow)) return fail(ODE_EINVAL, "grow must be >= 1");
    if (!(a->shrink > 0.0 && a->shrink <= 1.0)) return fail(ODE_EINVAL, "shrink must be in (0, 1]");
    for (int i = 0; i < ns; ++i) {
      if (!(a->rtol[i] >= 0.0) || !(a->atol[i] >= 0.0) || !(a->rtol[i] + a->atol[i] > 0.0) ||
          !std::isfinite(a->rtol[i]) || !std::isfinite(a->atol[i]))
        return fail(ODE_EINVAL, "tolerances of component %d must be >= 0 with a positive sum", i);
    }
  }
  int recording = 0;
  for (int j = 0; j < a->n_events; ++j) {
    const ode_event_spec &v = a->events[j];
    if (v.component < 0 || v.component >= ns)
      return fail(ODE_EINVAL, "event %d: component %d out of range", j, v.component);
    if (v.direction < -1 || v.direction > 1)
      return fail(ODE_EINVAL, "event %d: direction must be -1, 0 or 1", j);
    if (!(v.tolerance >= 0.0) || !std::isfinite(v.tolerance))
      return fail(ODE_EINVAL, "event %d: tolerance must be finite and >= 0", j);
    if (!std::isfinite(v.level)) return fail(ODE_EINVAL, "event %d: level must be finite", j);
    if (v.stop_after < 0) return fail(ODE_EINVAL, "event %d: stop_after < 0", j);
    if (v.action_component < -1 || v.action_component >= ns)
      return fail(ODE_EINVAL, "event %d: action_component out of range", j);
    if (v.action_param < -1 || v.action_param >= np)
      return fail(ODE_EINVAL, "event %d: action_param out of range", j);
    if (v.record_component < -1 || v.record_component >= ns)
      return fail(ODE_EINVAL, "event %d: record_component out of range", j);
    if (v.record_component >= 0) ++recording;
  }
  if (recording > 1) return fail(ODE_EINVAL, "at most one event may record");
  for (int k = 0; k < a->n_accessories; ++k) {
    const ode_accessory_spec &s = a->accessory_specs[k];
    if (s.kind != ODE_ACC_MAX && s.kind != ODE_ACC_MIN)
      return fail(ODE_EINVAL, "accessory %d: unknown kind %d", k, s.kind);
    if (s.component < 0 || s.component >= ns)
      return fail(ODE_EINVAL, "accessory %d: component out of range", k);
  }
  return ODE_OK;
}

int ode_ensemble_solve(ode_ensemble *e, const ode_solve_args *a, void *hip_stream) {
  if (!e || !a) return fail(ODE_EINVAL, "NULL handle or arguments");
  int rc = validate(e, a);
  if (rc != ODE_OK) return rc;
  if (a->n_systems == 0) return ODE_OK;

  Params prm;
  std::memset(&prm, 0, sizeof prm);
  Control &c = prm.c;
  for (int i = 0; i < ODE_MAX_STATE; ++i) {
    c.rtol[i] = a->rtol[i];
    c.atol[i] = a->atol[i];
  }
  c.h0 = a->h0;
  c.h_min = a->h_min;
  c.h_max = a->h_max;
  c.grow = a->grow;
  c.shrink = a->shrink;
  c.t_record = a->t_record;
  c.max_steps = static_cast<int32_t>(a->max_steps);
  c.max_eq = a->max_equilibrium_steps;
  c.n_events = a->n_events;
  c.n_acc = a->n_accessories;
  c.rec_cap = a->event_record_capacity;
  for (int j = 0; j < a->n_events; ++j) {
    const ode_event_spec &v = a->events[j];
    c.ev[j] = EventCtl{v.component, v.direction, v.stop_after, v.action_component,
                       v.action_param, v.record_component, v.level, v.tolerance, v.action_coef};
  }
  for (int k = 0; k < a->n_accessories; ++k)
    c.acc[k] = AccCtl{a->accessory_specs[k].kind, a->accessory_specs[k].component};

  const int nev = event_slots(a->n_events);
  const int nacc = acc_slots(a->n_accessories);
  int bpc = 0;
  rc = query_blocks(e, nev, nacc, &bpc);
  if (rc != ODE_OK) return rc;
  const int64_t max_grid = (int64_t)bpc * e->compute_units;
  const int64_t need = (a->n_systems + e->block - 1) / e->block;
  const int grid = static_cast<int>(need < max_grid ? need : max_grid);

  Arrays &arr = prm.a;
  arr.td = a->time_domain;
  arr.y = a->state;
  arr.p = a->params;
  arr.acc = a->accessories;
  arr.next_h = a->next_h;
  arr.status = a->status;
  arr.counts = a->counts;
  arr.evc = a->event_counts;
  arr.rec = a->event_records;
  arr.index = a->system_index;
  arr.n = a->n_systems;
  arr.ld = a->ld;
  arr.queue = e->queue;
  arr.total_waves = static_cast<uint32_t>(grid) * static_cast<uint32_t>(e->block / 64);

  hipError_t err = launch_integrator(e->model, e->method, e->precision, nev, nacc, prm, grid,
                                     e->block, static_cast<hipStream_t>(hip_stream));
  if (err != hipSuccess) return hip_fail(err, "integrator launch");
  e->last_blocks_per_cu = bpc;
  e->last_grid = grid;
  return ODE_OK;
}

}  // extern "C"
