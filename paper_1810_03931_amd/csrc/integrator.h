// Internal interface between the C ABI (api.cpp) and the integrator kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace odeens {

constexpr int kMaxState = 8;
constexpr int kMaxEvents = 4;
constexpr int kMaxAcc = 4;
constexpr int kMaxBlock = 256;
constexpr int kSecantMaxIter = 50;

enum LaneStatus : int32_t {
  kDone = 0,
  kStopEvent = 1,
  kStopEquilibrium = 2,
  kFailNan = 3,
  kMaxSteps = 4,
  kBadInput = 5,
  kRunning = -1
};
constexpr int32_t kFlagSecantCap = 0x100;

struct EventCtl {
  int32_t component, direction, stop_after, action_component, action_param, record_component;
  double level, tolerance, action_coef;
};

struct AccCtl {
  int32_t kind, component;  // kind: 1 max, 2 min, 3 log-and-reset at sections
};
constexpr int32_t kAccMax = 1, kAccMin = 2, kAccLogReset = 3;

// Solver-wide constants.  Passed by value in the kernel-argument segment.
// The kernel copies the ones every attempt reads into vector registers once
// per launch (scalar loads inside the attempt loop would stall a wave that
// runs alone); the rarely used fields are read from the argument segment
// where they are needed.
struct Control {
  double rtol[kMaxState], atol[kMaxState];
  double h0, h_min, h_max, grow, shrink, t_record;
  double section_period;  // > 0: Poincare sections n*T are forced boundaries
  int32_t max_steps;
  int32_t max_eq;
  int32_t n_events, n_acc, rec_cap, pad;
  EventCtl ev[kMaxEvents];
  AccCtl acc[kMaxAcc];
};

// Per-system arrays (structure of arrays, row r of system s at r*ld + s)
// and the persistent work queue.
struct Arrays {
  double *td;
  double *y;
  const double *p;
  double *acc;
  double *next_h;
  int32_t *status;
  int64_t *counts;
  int32_t *evc;
  double *rec;
  const int64_t *index;
  const double *t_rec;  // per-system window start, or nullptr (Control::t_record)
  const double *tol;    // per-system [2*n_state][ld] rtol, atol, or nullptr
  int64_t n, ld;
  // [0] next queue position, [1] finished waves (a served queue: finished
  // positions, i.e. systems retired plus ring entries naming no slot)
  unsigned long long *queue;
  uint32_t total_waves;
  // Served launches (avail != nullptr): queue position q holds the system in
  // slot index[q % ld]; positions below *avail are published (written by the
  // host with copies on its own stream while the launch runs).  Waves keep
  // taking published positions until *closed is set and every published
  // position is taken, or until they have polled idle_polls times in a row
  // without finding work.  A system's request (req_of[slot]) is finished when
  // req_left drops to zero; the last system of a request sets req_done[r] in
  // host-visible memory.
  const int64_t *avail;
  const int32_t *closed;
  const int32_t *req_of;
  int32_t *req_left;
  int32_t *req_done;
  int32_t n_req;
  int32_t idle_polls;
};

// Everything one launch needs, passed as the single by-value kernel argument.
struct Params {
  Control c;
  Arrays a;
};

// Compile-time variants: number of event / accessory slots compiled in.
inline int event_slots(int n_events) { return n_events == 0 ? 0 : (n_events == 1 ? 1 : 4); }
inline int acc_slots(int n_acc) { return n_acc == 0 ? 0 : (n_acc <= 2 ? 2 : 4); }

// The kernel for (model, method, precision, event slots, accessory slots,
// watched component: 0 or 1 when every event and extremum accessory watches
// that component, else -1), or nullptr.
const void *integrator_kernel(int model, int method, int prec, int nev, int nacc, int comp);

// Launch it with `grid` workgroups of `block` threads on `stream`.
hipError_t launch_integrator(int model, int method, int prec, int nev, int nacc, int comp,
                             const Params &prm, int grid, int block, hipStream_t stream);

// Repeated-horizon helpers (segments.hip): set t1 = t0 + segment for every
// listed system, and copy the state and accessories of every listed system
// into one snapshot.
hipError_t launch_set_horizon(double *td, int64_t ld, int64_t n, const int64_t *index,
                              double segment, hipStream_t stream);
// t1 of the copy = t0 + fraction * (t1 - t0) for every listed system (the
// probe horizon of the autotuner); fraction 1 copies t1 unchanged.
hipError_t launch_probe_horizon(const double *td_src, double *td_dst, int64_t ld, int64_t n,
                                const int64_t *index, double fraction, hipStream_t stream);
hipError_t launch_snapshot(const double *y, int n_state, const double *acc, int n_acc_rows,
                           int64_t ld, int64_t n, const int64_t *index, double *out,
                           hipStream_t stream);

}  // namespace odeens
