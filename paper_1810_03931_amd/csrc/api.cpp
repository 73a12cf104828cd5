// C ABI of the ensemble integrator: argument validation, handle management
// and kernel launch.  Declarations and the contract are in ode_ensemble.h.
#include "ode_ensemble.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "integrator.h"

namespace odeens {
const void *kernels_duffing(int method, int prec, int nev, int nacc, int comp);
const void *kernels_keller_miksis(int method, int prec, int nev, int nacc, int comp);
const void *kernels_relief_valve(int method, int prec, int nev, int nacc, int comp);
const void *kernels_ballistic(int method, int prec, int nev, int nacc, int comp);
const void *kernels_duffing_lyapunov(int method, int prec, int nev, int nacc, int comp);

const void *integrator_kernel(int model, int method, int prec, int nev, int nacc, int comp) {
  switch (model) {
    case ODE_MODEL_DUFFING: return kernels_duffing(method, prec, nev, nacc, comp);
    case ODE_MODEL_KELLER_MIKSIS: return kernels_keller_miksis(method, prec, nev, nacc, comp);
    case ODE_MODEL_RELIEF_VALVE: return kernels_relief_valve(method, prec, nev, nacc, comp);
    case ODE_MODEL_BALLISTIC: return kernels_ballistic(method, prec, nev, nacc, comp);
    case ODE_MODEL_DUFFING_LYAPUNOV:
      return kernels_duffing_lyapunov(method, prec, nev, nacc, comp);
    default: return nullptr;
  }
}

hipError_t launch_integrator(int model, int method, int prec, int nev, int nacc, int comp,
                             const Params &prm, int grid, int block, hipStream_t stream) {
  const void *fn = integrator_kernel(model, method, prec, nev, nacc, comp);
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
    case ODE_MODEL_DUFFING_LYAPUNOV: *ns = 4; *np = 5; return true;
    default: return false;
  }
}

constexpr int kDefaultBlock = 256;
// (event slots 0/1/4) x (accessory slots 0/2/4) x (watched component run-time/0/1)
constexpr int kCombos = 27;

int combo_index(int nev, int nacc, int comp) {
  const int e = nev == 0 ? 0 : (nev == 1 ? 1 : 2);
  const int k = nacc == 0 ? 0 : (nacc == 2 ? 1 : 2);
  return (e * 3 + k) * 3 + (comp + 1);
}

// The component every event and every extremum accessory of a solve
// watches, when there is one and it is 0 or 1 (kernels are compiled with it
// fixed); -1 otherwise.
int watched_component(const ode_solve_args *a) {
  int c = -2;
  for (int j = 0; j < a->n_events; ++j) {
    const int cj = a->events[j].component;
    if (c != -2 && c != cj) return -1;
    c = cj;
  }
  for (int k = 0; k < a->n_accessories; ++k) {
    if (a->accessory_specs[k].kind == ODE_ACC_LOG_RESET) continue;
    const int ck = a->accessory_specs[k].component;
    if (c != -2 && c != ck) return -1;
    c = ck;
  }
  return (c == 0 || c == 1) ? c : -1;
}

}  // namespace

// Arguments and launch shape a cached repeated-horizon graph was recorded
// for (a change of block size or residency, e.g. by the autotuner, records a
// new graph).
struct SegmentsKey {
  ode_solve_args args;
  int32_t n_segments, first_snapshot;
  double segment;
  double *snapshots;
  int32_t block, cap;
};

struct ode_ensemble {
  int32_t model, method, precision, block;
  int32_t n_state, n_param;
  int device;
  int compute_units;
  int cap;                     // resident workgroups per CU at most (0: no cap)
  int blocks_per_cu[kMaxBlock / 64][kCombos];  // occupancy per block size; 0 = not queried
  int last_blocks_per_cu, last_grid;
  unsigned long long *queue;   // device: [0] next position, [1] finished waves
  // repeated horizons: private capture stream and the cached graph
  hipStream_t capture_stream;
  hipGraphExec_t segments_exec;
  SegmentsKey segments_key;
};

namespace {

// Device copies of every array a solve writes, for the autotuning probes.
struct ProbeArrays {
  double *td = nullptr, *y = nullptr, *acc = nullptr, *next_h = nullptr, *rec = nullptr;
  int32_t *status = nullptr, *evc = nullptr;
  int64_t *counts = nullptr;
  ~ProbeArrays() {
    for (void *p : {(void *)td, (void *)y, (void *)acc, (void *)next_h, (void *)rec,
                    (void *)status, (void *)evc, (void *)counts})
      if (p) (void)hipFree(p);
  }
};

template <class T>
hipError_t alloc(T **p, int64_t count) {
  return count > 0 ? hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * count) : hipSuccess;
}

}  // namespace

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
  if (desc->blocks_per_cu < 0) return fail(ODE_EINVAL, "blocks_per_cu must be >= 0");

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
  e->cap = desc->blocks_per_cu;
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
  if (e->segments_exec) (void)hipGraphExecDestroy(e->segments_exec);
  if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
  if (e->queue) (void)hipFree(e->queue);
  std::free(e);
}

// Resident workgroups per CU for a block size and slot combination, after
// the handle's cap.
static int query_blocks(ode_ensemble *e, int block, int nev, int nacc, int comp, int *out) {
  int &slot = e->blocks_per_cu[block / 64 - 1][combo_index(nev, nacc, comp)];
  if (slot == 0) {
    const void *fn = integrator_kernel(e->model, e->method, e->precision, nev, nacc, comp);
    if (!fn) return fail(ODE_ENOTSUP, "no kernel for this model/method");
    int nb = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, 0);
    if (err != hipSuccess) return hip_fail(err, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    slot = nb > 0 ? nb : 1;
  }
  *out = (e->cap > 0 && e->cap < slot) ? e->cap : slot;
  return ODE_OK;
}

int ode_ensemble_query(const ode_ensemble *e, ode_ensemble_info *info) {
  if (!e || !info) return fail(ODE_EINVAL, "NULL argument");
  auto *m = const_cast<ode_ensemble *>(e);
  int bpc = e->last_blocks_per_cu;
  if (bpc == 0) {
    int rc = query_blocks(m, e->block, 0, 0, -1, &bpc);
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
  if (!(a->section_period >= 0.0) || !std::isfinite(a->section_period))
    return fail(ODE_EINVAL, "section_period must be finite and >= 0");
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
    if (s.kind != ODE_ACC_MAX && s.kind != ODE_ACC_MIN && s.kind != ODE_ACC_LOG_RESET)
      return fail(ODE_EINVAL, "accessory %d: unknown kind %d", k, s.kind);
    if (s.kind == ODE_ACC_LOG_RESET && !(a->section_period > 0.0))
      return fail(ODE_EINVAL, "accessory %d: ODE_ACC_LOG_RESET needs section_period > 0", k);
    if (s.component < 0 || s.component >= ns)
      return fail(ODE_EINVAL, "accessory %d: component out of range", k);
  }
  return ODE_OK;
}

// Launch parameters of one solve (arguments already validated).
static int prepare_launch(ode_ensemble *e, const ode_solve_args *a, Params &prm, int &nev,
                          int &nacc, int &comp, int &grid) {
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
  c.section_period = a->section_period;
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

  nev = event_slots(a->n_events);
  nacc = acc_slots(a->n_accessories);
  comp = watched_component(a);
  int bpc = 0;
  int rc = query_blocks(e, e->block, nev, nacc, comp, &bpc);
  if (rc != ODE_OK) return rc;
  const int64_t max_grid = (int64_t)bpc * e->compute_units;
  const int64_t need = (a->n_systems + e->block - 1) / e->block;
  grid = static_cast<int>(need < max_grid ? need : max_grid);

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
  arr.t_rec = a->record_start;
  arr.tol = a->tolerances;
  arr.n = a->n_systems;
  arr.ld = a->ld;
  arr.queue = e->queue;
  arr.total_waves = static_cast<uint32_t>(grid) * static_cast<uint32_t>(e->block / 64);
  e->last_blocks_per_cu = bpc;
  e->last_grid = grid;
  return ODE_OK;
}

int ode_ensemble_solve(ode_ensemble *e, const ode_solve_args *a, void *hip_stream) {
  if (!e || !a) return fail(ODE_EINVAL, "NULL handle or arguments");
  int rc = validate(e, a);
  if (rc != ODE_OK) return rc;
  if (a->n_systems == 0) return ODE_OK;
  Params prm;
  int nev = 0, nacc = 0, comp = -1, grid = 0;
  rc = prepare_launch(e, a, prm, nev, nacc, comp, grid);
  if (rc != ODE_OK) return rc;
  hipError_t err = launch_integrator(e->model, e->method, e->precision, nev, nacc, comp, prm, grid,
                                     e->block, static_cast<hipStream_t>(hip_stream));
  if (err != hipSuccess) return hip_fail(err, "integrator launch");
  return ODE_OK;
}

// ---- Solves that allocate nothing (ode_ensemble_solve_noalloc) ----
//
// The only device memory a solve needs beyond the caller's arrays is the
// work-queue counter pair.  For callers that cannot allocate, it lives in
// this file-scope array: one copy per GPU, loaded with the code object and
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (its name is a host-side stand-in there); it uses the device address
// that hipGetSymbolAddress returns, looked up once per device with that
// device current.
namespace {

constexpr int kScratchWords = 2;  // [0] next queue position, [1] finished waves
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
unsigned long long *g_scratch_ptr[kMaxDevices];  // device address per device, or null

int scratch_of_device(int dev, unsigned long long **out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(ODE_ENOTSUP, "device %d: at most %d devices are supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return hip_fail(err, "hipGetSymbolAddress of the scratch counters");
    g_scratch_ptr[dev] = static_cast<unsigned long long *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return ODE_OK;
}

// Zeroes the counters on the stream before a launch (a kernel, not
// hipMemsetAsync, so the call can be recorded into a graph and replayed).
__global__ void clear_scratch(unsigned long long *words, int n) {
  if ((int)threadIdx.x < n) words[threadIdx.x] = 0ull;
}

}  // namespace

extern "C" int ode_ensemble_solve_noalloc(const ode_ensemble_desc *desc, const ode_solve_args *a,
                                          void *hip_stream) {
  if (!desc || !a) return fail(ODE_EINVAL, "NULL descriptor or arguments");
  ode_ensemble e;
  std::memset(&e, 0, sizeof e);
  if (!model_dims(desc->model, &e.n_state, &e.n_param))
    return fail(ODE_EINVAL, "unknown model %d", desc->model);
  if (desc->method != ODE_RKCK45 && desc->method != ODE_RK4)
    return fail(ODE_EINVAL, "unknown method %d", desc->method);
  if (desc->precision != ODE_FP64 && desc->precision != ODE_FP32_STAGES)
    return fail(ODE_EINVAL, "unknown precision %d", desc->precision);
  const int block = desc->block_size == 0 ? kDefaultBlock : desc->block_size;
  if (block < 64 || block > kMaxBlock || block % 64 != 0)
    return fail(ODE_EINVAL, "block_size %d must be a multiple of 64 in [64, %d]",
                desc->block_size, kMaxBlock);
  if (desc->blocks_per_cu < 0) return fail(ODE_EINVAL, "blocks_per_cu must be >= 0");
  e.model = desc->model;
  e.method = desc->method;
  e.precision = desc->precision;
  e.block = block;
  e.cap = desc->blocks_per_cu;
  int rc = validate(&e, a);
  if (rc != ODE_OK) return rc;
  if (a->n_systems == 0) return ODE_OK;

  hipError_t err = hipGetDevice(&e.device);
  if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
  err = hipDeviceGetAttribute(&e.compute_units, hipDeviceAttributeMultiprocessorCount, e.device);
  if (err != hipSuccess) return hip_fail(err, "hipDeviceGetAttribute");
  rc = scratch_of_device(e.device, &e.queue);
  if (rc != ODE_OK) return rc;

  Params prm;
  int nev = 0, nacc = 0, comp = -1, grid = 0;
  rc = prepare_launch(&e, a, prm, nev, nacc, comp, grid);
  if (rc != ODE_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(clear_scratch, dim3(1), dim3(64), 0, st, e.queue, kScratchWords);
  err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(err, "clearing the scratch counters");
  err = launch_integrator(e.model, e.method, e.precision, nev, nacc, comp, prm, grid, e.block, st);
  if (err != hipSuccess) return hip_fail(err, "integrator launch");
  return ODE_OK;
}

// ---- Served queues (ode_serve_*) ----

struct ode_serve {
  int device;
  int32_t max_requests;
  // device memory: [0] published positions (int64), [1] closed (int32 in the
  // low half), [2] next queue position, [3] finished positions
  int64_t *dev_words;
  int32_t *req_left;     // device [max_requests]
  int32_t *req_done;     // host, coherent and mapped [max_requests]
  int32_t *req_done_dev; // the same memory as the device addresses it
  int64_t *stage;        // host, pinned: staging words for the small copies
  // the queue's own launch and copy streams, created with a mask of every
  // compute unit: such streams get a hardware queue of their own instead of
  // sharing one round-robin with the process's other streams, where a copy
  // or a relaunch would wait behind another stream's persistent launch
  hipStream_t streams[2];
};

namespace {
constexpr int kServeWords = 4;   // published, closed, queue position, finished positions
constexpr int kStageCount = kServeWords + 1;   // + one staging word for a request's count

int serve_copy_word(ode_serve *s, int index, int64_t value, hipStream_t st) {
  // the host staging word stays unchanged until the copy has completed: the
  // call waits for the stream
  s->stage[index] = value;
  hipError_t err = hipMemcpyAsync(s->dev_words + index, s->stage + index, sizeof(int64_t),
                                  hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  if (err != hipSuccess) return hip_fail(err, "copying a served-queue word");
  return ODE_OK;
}
}  // namespace

extern "C" int ode_serve_create(int32_t max_requests, ode_serve **out) {
  if (!out) return fail(ODE_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_requests < 1 || max_requests > (1 << 24))
    return fail(ODE_EINVAL, "max_requests must be in [1, 2^24]");
  auto *s = static_cast<ode_serve *>(std::calloc(1, sizeof(ode_serve)));
  if (!s) return fail(ODE_ENOMEM, "host allocation failed");
  s->max_requests = max_requests;
  hipError_t err = hipGetDevice(&s->device);
  if (err == hipSuccess) err = hipMalloc(reinterpret_cast<void **>(&s->dev_words),
                                         kServeWords * sizeof(int64_t));
  if (err == hipSuccess) err = hipMalloc(reinterpret_cast<void **>(&s->req_left),
                                         sizeof(int32_t) * max_requests);
  if (err == hipSuccess)
    err = hipHostMalloc(reinterpret_cast<void **>(&s->req_done), sizeof(int32_t) * max_requests,
                        hipHostMallocCoherent | hipHostMallocMapped);
  if (err == hipSuccess)
    err = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->req_done_dev), s->req_done, 0);
  if (err == hipSuccess)
    err = hipHostMalloc(reinterpret_cast<void **>(&s->stage), kStageCount * sizeof(int64_t),
                        hipHostMallocDefault);
  int n_cu = 0;
  if (err == hipSuccess)
    err = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s->device);
  if (err == hipSuccess) {
    uint32_t mask[32] = {};
    const int words = n_cu <= 0 ? 0 : (n_cu > 1024 ? 32 : (n_cu + 31) / 32);
    for (int c = 0; c < words * 32 && c < n_cu; ++c) mask[c / 32] |= 1u << (c % 32);
    for (int k = 0; k < 2 && err == hipSuccess; ++k)
      err = hipExtStreamCreateWithCUMask(&s->streams[k], static_cast<uint32_t>(words), mask);
  }
  if (err == hipSuccess) err = hipMemset(s->dev_words, 0, kServeWords * sizeof(int64_t));
  if (err == hipSuccess) err = hipMemset(s->req_left, 0, sizeof(int32_t) * max_requests);
  if (err == hipSuccess) err = hipDeviceSynchronize();
  if (err != hipSuccess) {
    ode_serve_destroy(s);
    return fail(ODE_ENOMEM, "allocating a served queue: %s", hipGetErrorString(err));
  }
  std::memset(s->req_done, 0, sizeof(int32_t) * max_requests);
  *out = s;
  return ODE_OK;
}

extern "C" void ode_serve_destroy(ode_serve *s) {
  if (!s) return;
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->dev_words) (void)hipFree(s->dev_words);
  if (s->req_left) (void)hipFree(s->req_left);
  if (s->req_done) (void)hipHostFree(s->req_done);
  if (s->stage) (void)hipHostFree(s->stage);
  std::free(s);
}

extern "C" volatile int32_t *ode_serve_done_flags(ode_serve *s) {
  return s ? s->req_done : nullptr;
}

extern "C" void *ode_serve_stream(ode_serve *s, int32_t which) {
  return (s && (which == 0 || which == 1)) ? static_cast<void *>(s->streams[which]) : nullptr;
}

extern "C" int ode_serve_reset(ode_serve *s, void *copy_stream) {
  if (!s) return fail(ODE_EINVAL, "NULL served queue");
  const hipStream_t st = static_cast<hipStream_t>(copy_stream);
  for (int w = 0; w < kServeWords; ++w) {
    const int rc = serve_copy_word(s, w, 0, st);
    if (rc != ODE_OK) return rc;
  }
  std::memset(const_cast<int32_t *>(s->req_done), 0, sizeof(int32_t) * s->max_requests);
  return ODE_OK;
}

extern "C" int ode_serve_begin_request(ode_serve *s, int32_t request, int32_t n_systems,
                                       void *copy_stream) {
  if (!s) return fail(ODE_EINVAL, "NULL served queue");
  if (request < 0 || request >= s->max_requests)
    return fail(ODE_EINVAL, "request %d outside [0, %d)", request, s->max_requests);
  if (n_systems < 1) return fail(ODE_EINVAL, "a request needs at least one system");
  const hipStream_t st = static_cast<hipStream_t>(copy_stream);
  __atomic_store_n(s->req_done + request, 0, __ATOMIC_RELEASE);
  int32_t *n32 = reinterpret_cast<int32_t *>(s->stage + kServeWords);
  *n32 = n_systems;
  hipError_t err = hipMemcpyAsync(s->req_left + request, n32, sizeof(int32_t),
                                  hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  if (err != hipSuccess) return hip_fail(err, "setting a request's count");
  return ODE_OK;
}

extern "C" int ode_serve_publish(ode_serve *s, int64_t published, void *copy_stream) {
  if (!s) return fail(ODE_EINVAL, "NULL served queue");
  if (published < 0) return fail(ODE_EINVAL, "published < 0");
  return serve_copy_word(s, 0, published, static_cast<hipStream_t>(copy_stream));
}

extern "C" int ode_serve_close(ode_serve *s, void *copy_stream) {
  if (!s) return fail(ODE_EINVAL, "NULL served queue");
  return serve_copy_word(s, 1, 1, static_cast<hipStream_t>(copy_stream));
}

extern "C" int ode_serve_launch(ode_serve *s, ode_ensemble *e, const ode_solve_args *a,
                                const int32_t *request_of_slot, int32_t max_workgroups,
                                int32_t idle_polls, void *hip_stream) {
  if (!s || !e || !a) return fail(ODE_EINVAL, "NULL served queue, handle or arguments");
  if (!a->system_index) return fail(ODE_EINVAL, "a served launch needs the position ring (system_index)");
  if (!request_of_slot) return fail(ODE_EINVAL, "request_of_slot is NULL");
  if (max_workgroups < 0) return fail(ODE_EINVAL, "max_workgroups < 0");
  if (idle_polls < 1) return fail(ODE_EINVAL, "idle_polls must be >= 1");
  ode_solve_args v = *a;
  v.n_systems = a->ld;   // the ring: every slot may be taken
  int rc = validate(e, &v);
  if (rc != ODE_OK) return rc;
  if (v.ld < 1) return fail(ODE_EINVAL, "ld must be >= 1");
  Params prm;
  int nev = 0, nacc = 0, comp = -1, grid = 0;
  rc = prepare_launch(e, &v, prm, nev, nacc, comp, grid);
  if (rc != ODE_OK) return rc;
  if (max_workgroups > 0 && grid > max_workgroups) grid = max_workgroups;
  Arrays &arr = prm.a;
  arr.queue = reinterpret_cast<unsigned long long *>(s->dev_words + 2);
  arr.total_waves = static_cast<uint32_t>(grid) * static_cast<uint32_t>(e->block / 64);
  arr.avail = s->dev_words;
  arr.closed = reinterpret_cast<const int32_t *>(s->dev_words + 1);
  arr.req_of = request_of_slot;
  arr.req_left = s->req_left;
  arr.req_done = s->req_done_dev;
  arr.n_req = s->max_requests;
  arr.idle_polls = idle_polls;
  e->last_grid = grid;
  const hipError_t err = launch_integrator(e->model, e->method, e->precision, nev, nacc, comp, prm, grid,
                                           e->block, static_cast<hipStream_t>(hip_stream));
  if (err != hipSuccess) return hip_fail(err, "served launch");
  return ODE_OK;
}

// Records the whole repeated-horizon sequence on the handle's private stream.
static int record_segments(ode_ensemble *e, const ode_solve_args *a, int32_t n_segments,
                           double segment, int32_t first_snapshot, double *snapshots,
                           hipGraphExec_t *out) {
  Params prm;
  int nev = 0, nacc = 0, comp = -1, grid = 0;
  int rc = prepare_launch(e, a, prm, nev, nacc, comp, grid);
  if (rc != ODE_OK) return rc;
  const int rows = e->n_state + 2 * a->n_accessories;
  hipStream_t cs = e->capture_stream;
  hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) return hip_fail(err, "hipStreamBeginCapture");
  hipError_t first = hipSuccess;
  for (int32_t k = 0; k < n_segments && first == hipSuccess; ++k) {
    first = launch_set_horizon(a->time_domain, a->ld, a->n_systems, a->system_index, segment, cs);
    if (first == hipSuccess)
      first = launch_integrator(e->model, e->method, e->precision, nev, nacc, comp, prm, grid, e->block,
                                cs);
    if (first == hipSuccess && k >= first_snapshot)
      first = launch_snapshot(a->state, e->n_state, a->accessories, 2 * a->n_accessories, a->ld,
                              a->n_systems, a->system_index,
                              snapshots + (int64_t)(k - first_snapshot) * rows * a->ld, cs);
  }
  hipGraph_t graph = nullptr;
  err = hipStreamEndCapture(cs, &graph);
  if (first != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(first, "recording the segment launches");
  }
  if (err != hipSuccess) return hip_fail(err, "hipStreamEndCapture");
  err = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (err != hipSuccess) return hip_fail(err, "hipGraphInstantiate");
  return ODE_OK;
}

int ode_ensemble_solve_segments(ode_ensemble *e, const ode_solve_args *a, int32_t n_segments,
                                double segment, int32_t first_snapshot, double *snapshots,
                                void *hip_stream) {
  if (!e || !a) return fail(ODE_EINVAL, "NULL handle or arguments");
  int rc = validate(e, a);
  if (rc != ODE_OK) return rc;
  if (n_segments < 1) return fail(ODE_EINVAL, "n_segments must be >= 1");
  if (!finite_pos(segment)) return fail(ODE_EINVAL, "segment must be finite and > 0");
  if (first_snapshot < 0 || first_snapshot > n_segments)
    return fail(ODE_EINVAL, "first_snapshot must be in [0, n_segments]");
  if (a->n_systems > 0 && (first_snapshot < n_segments) != (snapshots != nullptr))
    return fail(ODE_EINVAL, "snapshots must be given exactly when first_snapshot < n_segments");
  if (a->n_systems > (int64_t(1) << 38)) return fail(ODE_EINVAL, "n_systems too large");
  if (a->n_systems == 0) return ODE_OK;

  SegmentsKey key;
  std::memset(&key, 0, sizeof key);
  key.args = *a;
  key.n_segments = n_segments;
  key.first_snapshot = first_snapshot;
  key.segment = segment;
  key.snapshots = snapshots;
  key.block = e->block;
  key.cap = e->cap;
  // the event and accessory arrays beyond the counts in use do not matter
  for (int j = a->n_events; j < ODE_MAX_EVENTS; ++j) std::memset(&key.args.events[j], 0, sizeof(ode_event_spec));
  for (int k = a->n_accessories; k < ODE_MAX_ACCESSORIES; ++k)
    std::memset(&key.args.accessory_specs[k], 0, sizeof(ode_accessory_spec));
  if (!e->capture_stream) {
    hipError_t err = hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking);
    if (err != hipSuccess) {
      e->capture_stream = nullptr;
      return hip_fail(err, "hipStreamCreateWithFlags");
    }
  }
  if (!e->segments_exec || std::memcmp(&key, &e->segments_key, sizeof key) != 0) {
    if (e->segments_exec) {
      (void)hipGraphExecDestroy(e->segments_exec);
      e->segments_exec = nullptr;
    }
    hipGraphExec_t exec = nullptr;
    rc = record_segments(e, a, n_segments, segment, first_snapshot, snapshots, &exec);
    if (rc != ODE_OK) return rc;
    e->segments_exec = exec;
    e->segments_key = key;
  }
  hipError_t err = hipGraphLaunch(e->segments_exec, static_cast<hipStream_t>(hip_stream));
  if (err != hipSuccess) return hip_fail(err, "hipGraphLaunch");
  return ODE_OK;
}

int ode_ensemble_tune(ode_ensemble *e, const ode_solve_args *a, double probe_fraction,
                      void *hip_stream, ode_tune_result *result) {
  if (!e || !a || !result) return fail(ODE_EINVAL, "NULL handle, arguments or result");
  int rc = validate(e, a);
  if (rc != ODE_OK) return rc;
  if (!(probe_fraction > 0.0 && probe_fraction <= 1.0))
    return fail(ODE_EINVAL, "probe_fraction must be in (0, 1]");
  std::memset(result, 0, sizeof *result);
  result->block_size = e->block;
  result->blocks_per_cu = e->cap;
  if (a->n_systems == 0) return ODE_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t ld = a->ld;

  ProbeArrays c;
  hipError_t err = hipSuccess;
  auto chk = [&](hipError_t x) { if (err == hipSuccess) err = x; };
  chk(alloc(&c.td, 2 * ld));
  chk(alloc(&c.y, (int64_t)e->n_state * ld));
  chk(alloc(&c.status, ld));
  chk(alloc(&c.counts, 3 * ld));
  if (a->n_accessories) chk(alloc(&c.acc, 2 * (int64_t)a->n_accessories * ld));
  if (a->next_h) chk(alloc(&c.next_h, ld));
  if (a->n_events) chk(alloc(&c.evc, (int64_t)a->n_events * ld));
  if (a->event_record_capacity) chk(alloc(&c.rec, 2 * (int64_t)a->event_record_capacity * ld));
  if (err != hipSuccess)
    return fail(ODE_ENOMEM, "allocating the probe copies: %s", hipGetErrorString(err));
  ode_solve_args pa = *a;
  pa.time_domain = c.td;
  pa.state = c.y;
  pa.accessories = c.acc;
  pa.next_h = c.next_h;
  pa.status = c.status;
  pa.counts = c.counts;
  pa.event_counts = c.evc;
  pa.event_records = c.rec;

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  chk(hipEventCreate(&ev0));
  chk(hipEventCreate(&ev1));
  if (err != hipSuccess) {
    if (ev0) (void)hipEventDestroy(ev0);
    return hip_fail(err, "hipEventCreate");
  }
  const int saved_block = e->block, saved_cap = e->cap;
  // one probe: fresh copies of the inputs, then the timed solve
  auto probe = [&](int block, int cap, double *ms) -> int {
    e->block = block;
    e->cap = cap;
    hipError_t x = launch_probe_horizon(a->time_domain, c.td, ld, a->n_systems, a->system_index,
                                        probe_fraction, st);
    if (x == hipSuccess)
      x = hipMemcpyAsync(c.y, a->state, sizeof(double) * e->n_state * ld,
                         hipMemcpyDeviceToDevice, st);
    if (x == hipSuccess && a->next_h)
      x = hipMemcpyAsync(c.next_h, a->next_h, sizeof(double) * ld, hipMemcpyDeviceToDevice, st);
    if (x != hipSuccess) return hip_fail(x, "preparing a probe");
    Params prm;
    int nev = 0, nacc = 0, comp = -1, grid = 0;
    int r = prepare_launch(e, &pa, prm, nev, nacc, comp, grid);
    if (r != ODE_OK) return r;
    x = hipEventRecord(ev0, st);
    if (x == hipSuccess)
      x = launch_integrator(e->model, e->method, e->precision, nev, nacc, comp, prm, grid, block, st);
    if (x == hipSuccess) x = hipEventRecord(ev1, st);
    if (x == hipSuccess) x = hipEventSynchronize(ev1);
    float f = 0.0f;
    if (x == hipSuccess) x = hipEventElapsedTime(&f, ev0, ev1);
    if (x != hipSuccess) return hip_fail(x, "timing a probe");
    *ms = f;
    return ODE_OK;
  };

  int best_block = saved_block, best_cap = saved_cap, n_tried = 0;
  double best = 0.0, base = 0.0;
  // the handle's own configuration, twice: the first run also warms up
  rc = probe(saved_block, saved_cap, &base);
  if (rc == ODE_OK) rc = probe(saved_block, saved_cap, &base);
  best = base;
  n_tried = 1;
  static const int kBlocks[] = {64, 128, 256};
  for (int b : kBlocks) {
    int full = 0;
    e->cap = 0;
    rc = query_blocks(e, b, event_slots(a->n_events), acc_slots(a->n_accessories),
                      watched_component(a), &full);
    for (int half = 0; half < 2 && rc == ODE_OK; ++half) {
      const int cap = half ? full / 2 : 0;
      if (half && cap < 1) continue;
      if (b == saved_block && cap == saved_cap) continue;
      double ms = 0.0;
      rc = probe(b, cap, &ms);
      ++n_tried;
      if (rc == ODE_OK && ms < best) {
        best = ms;
        best_block = b;
        best_cap = cap;
      }
    }
    if (rc != ODE_OK) break;
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  e->block = rc == ODE_OK ? best_block : saved_block;
  e->cap = rc == ODE_OK ? best_cap : saved_cap;
  e->last_blocks_per_cu = 0;  // describe the chosen configuration, not the last probe
  e->last_grid = 0;
  if (rc != ODE_OK) return rc;
  result->block_size = best_block;
  result->blocks_per_cu = best_cap;
  result->candidates = n_tried;
  result->best_ms = best;
  result->default_ms = base;
  return ODE_OK;
}


int ode_ensemble_plan(ode_ensemble *e, const ode_solve_args *a, double probe_fraction,
                      double probe_tolerance_scale, int64_t *index_out, int64_t capacity,
                      int64_t *n_positions, void *hip_stream) {
  if (!e || !a || !n_positions) return fail(ODE_EINVAL, "NULL handle, arguments or n_positions");
  int rc = validate(e, a);
  if (rc != ODE_OK) return rc;
  if (!(probe_fraction > 0.0 && probe_fraction <= 1.0))
    return fail(ODE_EINVAL, "probe_fraction must be in (0, 1]");
  if (!(probe_tolerance_scale >= 1.0) || !std::isfinite(probe_tolerance_scale))
    return fail(ODE_EINVAL, "probe_tolerance_scale must be finite and >= 1");
  const int64_t n = a->n_systems, ld = a->ld;
  int bpc = 0;
  rc = query_blocks(e, e->block, event_slots(a->n_events), acc_slots(a->n_accessories),
                    watched_component(a), &bpc);
  if (rc != ODE_OK) return rc;
  const int64_t max_grid = (int64_t)bpc * e->compute_units;
  const int64_t need = (n + e->block - 1) / e->block;
  const int64_t waves = std::max<int64_t>(1, std::min(need, max_grid)) * (e->block / 64);
  const int64_t round_waves = 4 * (int64_t)e->compute_units;  // one wave on every SIMD
  const int64_t total = n == 0 ? 0 : (waves * 64 >= n ? waves * 64 : n);
  *n_positions = total;
  if (!index_out || n == 0) return ODE_OK;
  if (capacity < total)
    return fail(ODE_EINVAL, "index capacity %lld < %lld positions", (long long)capacity,
                (long long)total);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);

  // the probe: the problem over the first probe_fraction of each horizon, on
  // private copies of every array the solve writes
  ProbeArrays c;
  hipError_t err = hipSuccess;
  auto chk = [&](hipError_t x) { if (err == hipSuccess) err = x; };
  chk(alloc(&c.td, 2 * ld));
  chk(alloc(&c.y, (int64_t)e->n_state * ld));
  chk(alloc(&c.status, ld));
  chk(alloc(&c.counts, 3 * ld));
  if (a->n_accessories) chk(alloc(&c.acc, 2 * (int64_t)a->n_accessories * ld));
  if (a->next_h) chk(alloc(&c.next_h, ld));
  if (a->n_events) chk(alloc(&c.evc, (int64_t)a->n_events * ld));
  if (a->event_record_capacity) chk(alloc(&c.rec, 2 * (int64_t)a->event_record_capacity * ld));
  if (err != hipSuccess)
    return fail(ODE_ENOMEM, "allocating the probe copies: %s", hipGetErrorString(err));
  ode_solve_args pa = *a;
  pa.time_domain = c.td;
  pa.state = c.y;
  pa.accessories = c.acc;
  pa.next_h = c.next_h;
  pa.status = c.status;
  pa.counts = c.counts;
  pa.event_counts = c.evc;
  pa.event_records = c.rec;
  for (int i = 0; i < ODE_MAX_STATE; ++i) {
    pa.rtol[i] = a->rtol[i] * probe_tolerance_scale;
    pa.atol[i] = a->atol[i] * probe_tolerance_scale;
  }
  hipError_t x = launch_probe_horizon(a->time_domain, c.td, ld, n, a->system_index,
                                      probe_fraction, st);
  if (x == hipSuccess)
    x = hipMemcpyAsync(c.y, a->state, sizeof(double) * e->n_state * ld, hipMemcpyDeviceToDevice, st);
  if (x == hipSuccess && a->next_h)
    x = hipMemcpyAsync(c.next_h, a->next_h, sizeof(double) * ld, hipMemcpyDeviceToDevice, st);
  if (x != hipSuccess) return hip_fail(x, "preparing the probe");
  Params prm;
  int nev = 0, nacc = 0, comp = -1, grid = 0;
  rc = prepare_launch(e, &pa, prm, nev, nacc, comp, grid);
  if (rc != ODE_OK) return rc;
  x = launch_integrator(e->model, e->method, e->precision, nev, nacc, comp, prm, grid, e->block, st);
  if (x != hipSuccess) return hip_fail(x, "launching the probe");

  // per-position cost: the probe's attempts of the position's system
  std::vector<int64_t> counts(3 * ld), queue, cost(n, 0), order(total);
  x = hipMemcpyAsync(counts.data(), c.counts, sizeof(int64_t) * 3 * ld, hipMemcpyDeviceToHost, st);
  if (x == hipSuccess && a->system_index) {
    queue.resize(n);
    x = hipMemcpyAsync(queue.data(), a->system_index, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st);
  }
  if (x == hipSuccess) x = hipStreamSynchronize(st);
  if (x != hipSuccess) return hip_fail(x, "reading the probe counts");
  for (int64_t q = 0; q < n; ++q) {
    const int64_t s = queue.empty() ? q : queue[q];
    if (s >= 0 && s < ld) cost[q] = counts[s] + counts[ld + s] + counts[2 * ld + s];
  }
  int64_t written = 0;
  if (ode_plan_order(cost.data(), queue.empty() ? nullptr : queue.data(), n, waves, round_waves,
                     order.data(), total, &written) != ODE_OK || written != total)
    return fail(ODE_EINVAL, "planner arguments");
  x = hipMemcpyAsync(index_out, order.data(), sizeof(int64_t) * total, hipMemcpyHostToDevice, st);
  if (x == hipSuccess) x = hipStreamSynchronize(st);
  if (x != hipSuccess) return hip_fail(x, "writing the plan");
  return ODE_OK;
}

}  // extern "C"
