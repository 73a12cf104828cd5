"""Python binding of the C ABI in ``include/ode_ensemble.h`` (ctypes).

Argument marshalling only: every step of the integration runs in the HIP
library ``lib/libode_ensemble.so``.  PyTorch supplies device memory and the
stream.  If the library is missing or cannot be loaded, every call raises --
there is no CPU fallback.

Arrays are torch float64 (int32/int64 for status, counts and indices) CUDA
tensors shaped [rows, ld] and C-contiguous; row r of system s is element
[r, s] (paper Sec. 6.1, problem pool).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Any, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libode_ensemble.so")

MODEL = {"duffing": 1, "keller_miksis": 2, "relief_valve": 3, "ballistic": 4,
         "duffing_lyapunov": 5}
METHOD = {"rkck45": 0, "rk4": 1}
PRECISION = {"fp64": 0, "mixed": 1}
ACC_KIND = {"max": 1, "min": 2, "log_reset": 3}
MAX_STATE, MAX_EVENTS, MAX_ACC = 8, 4, 4

OK, EINVAL, ENOMEM, EHIP, ENOTSUP = 0, -1, -2, -3, -4
DONE, STOP_EVENT, STOP_EQUILIBRIUM, FAIL_NAN, MAX_STEPS, BAD_INPUT = range(6)
FLAG_SECANT_CAP = 0x100


class OdeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ode_ensemble error {code}: {msg}")
        self.code = code


class EventSpec(C.Structure):
    _fields_ = [
        ("component", C.c_int32), ("direction", C.c_int32), ("stop_after", C.c_int32),
        ("action_component", C.c_int32), ("action_param", C.c_int32),
        ("record_component", C.c_int32),
        ("level", C.c_double), ("tolerance", C.c_double), ("action_coef", C.c_double),
    ]


class AccessorySpec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("component", C.c_int32)]


class Desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("method", C.c_int32), ("precision", C.c_int32),
                ("block_size", C.c_int32), ("blocks_per_cu", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("candidates", C.c_int32), ("reserved", C.c_int32),
                ("best_ms", C.c_double), ("default_ms", C.c_double)]


class SolveArgs(C.Structure):
    _fields_ = [
        ("n_systems", C.c_int64), ("ld", C.c_int64),
        ("time_domain", C.c_void_p), ("state", C.c_void_p), ("params", C.c_void_p),
        ("accessories", C.c_void_p), ("next_h", C.c_void_p), ("status", C.c_void_p),
        ("counts", C.c_void_p), ("event_counts", C.c_void_p), ("event_records", C.c_void_p),
        ("system_index", C.c_void_p), ("record_start", C.c_void_p), ("tolerances", C.c_void_p),
        ("rtol", C.c_double * MAX_STATE), ("atol", C.c_double * MAX_STATE),
        ("h0", C.c_double), ("h_min", C.c_double), ("h_max", C.c_double),
        ("grow", C.c_double), ("shrink", C.c_double), ("t_record", C.c_double),
        ("section_period", C.c_double), ("max_steps", C.c_int64), ("max_equilibrium_steps", C.c_int32),
        ("n_events", C.c_int32), ("n_accessories", C.c_int32),
        ("event_record_capacity", C.c_int32),
        ("events", EventSpec * MAX_EVENTS), ("accessory_specs", AccessorySpec * MAX_ACC),
    ]


class Info(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("compute_units", C.c_int32), ("max_grid", C.c_int32),
                ("resident_systems", C.c_int64)]


EXPORTS = ("ode_ensemble_model_dims", "ode_ensemble_create", "ode_ensemble_solve",
           "ode_ensemble_solve_noalloc", "ode_ensemble_solve_segments", "ode_ensemble_tune",
           "ode_ensemble_plan", "ode_plan_order", "ode_serve_create", "ode_serve_done_flags",
           "ode_serve_stream", "ode_serve_reset", "ode_serve_begin_request", "ode_serve_publish", "ode_serve_close",
           "ode_serve_launch", "ode_serve_destroy", "ode_ensemble_query", "ode_ensemble_destroy",
           "ode_ensemble_last_error")

_lib = None


def plan_order(cost, waves: int, round_waves: int, queue=None):
    """Host-only queue order from per-position costs (``ode_plan_order``):
    numpy int64 ``cost`` [n] and optional ``queue`` [n] -> int64 order."""
    import numpy as np
    cost = np.ascontiguousarray(cost, dtype=np.int64)
    q = None if queue is None else np.ascontiguousarray(queue, dtype=np.int64)
    if q is not None and q.size != cost.size:
        raise ValueError("queue: need one entry per cost")
    lib = load_library()
    total = C.c_int64(0)
    args = (cost.ctypes.data, None if q is None else q.ctypes.data, cost.size, int(waves),
            int(round_waves))
    if lib.ode_plan_order(*args, None, 0, C.byref(total)) != OK:
        raise OdeError(EINVAL, "ode_plan_order: invalid arguments")
    out = np.empty(max(total.value, 1), dtype=np.int64)
    if lib.ode_plan_order(*args, out.ctypes.data, out.size, C.byref(total)) != OK:
        raise OdeError(EINVAL, "ode_plan_order: invalid arguments")
    return out[:total.value]


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OdeError(ENOTSUP, f"HIP library not built: {path} (run __graft_entry__.build())")
    L = C.CDLL(path)
    L.ode_ensemble_model_dims.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.ode_ensemble_model_dims.restype = C.c_int
    L.ode_ensemble_create.argtypes = [C.POINTER(Desc), C.POINTER(C.c_void_p)]
    L.ode_ensemble_create.restype = C.c_int
    L.ode_ensemble_solve.argtypes = [C.c_void_p, C.POINTER(SolveArgs), C.c_void_p]
    L.ode_ensemble_solve.restype = C.c_int
    L.ode_ensemble_solve_noalloc.argtypes = [C.POINTER(Desc), C.POINTER(SolveArgs), C.c_void_p]
    L.ode_ensemble_solve_noalloc.restype = C.c_int
    L.ode_ensemble_solve_segments.argtypes = [C.c_void_p, C.POINTER(SolveArgs), C.c_int32,
                                              C.c_double, C.c_int32, C.c_void_p, C.c_void_p]
    L.ode_ensemble_solve_segments.restype = C.c_int
    L.ode_ensemble_tune.argtypes = [C.c_void_p, C.POINTER(SolveArgs), C.c_double, C.c_void_p,
                                    C.POINTER(TuneResult)]
    L.ode_ensemble_tune.restype = C.c_int
    L.ode_ensemble_plan.argtypes = [C.c_void_p, C.POINTER(SolveArgs), C.c_double, C.c_double,
                                    C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_void_p]
    L.ode_ensemble_plan.restype = C.c_int
    L.ode_plan_order.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                 C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
    L.ode_plan_order.restype = C.c_int
    L.ode_serve_create.argtypes = [C.c_int32, C.POINTER(C.c_void_p)]
    L.ode_serve_create.restype = C.c_int
    L.ode_serve_done_flags.argtypes = [C.c_void_p]
    L.ode_serve_done_flags.restype = C.c_void_p
    L.ode_serve_stream.argtypes = [C.c_void_p, C.c_int32]
    L.ode_serve_stream.restype = C.c_void_p
    for f in ("ode_serve_reset", "ode_serve_close"):
        getattr(L, f).argtypes = [C.c_void_p, C.c_void_p]
        getattr(L, f).restype = C.c_int
    L.ode_serve_begin_request.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
    L.ode_serve_begin_request.restype = C.c_int
    L.ode_serve_publish.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
    L.ode_serve_publish.restype = C.c_int
    L.ode_serve_launch.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(SolveArgs), C.c_void_p,
                                   C.c_int32, C.c_int32, C.c_void_p]
    L.ode_serve_launch.restype = C.c_int
    L.ode_serve_destroy.argtypes = [C.c_void_p]
    L.ode_serve_destroy.restype = None
    L.ode_ensemble_query.argtypes = [C.c_void_p, C.POINTER(Info)]
    L.ode_ensemble_query.restype = C.c_int
    L.ode_ensemble_destroy.argtypes = [C.c_void_p]
    L.ode_ensemble_destroy.restype = None
    L.ode_ensemble_last_error.argtypes = []
    L.ode_ensemble_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise OdeError(rc, load_library().ode_ensemble_last_error().decode())


def model_dims(model: str) -> tuple[int, int]:
    ns, np_ = C.c_int32(), C.c_int32()
    _check(load_library().ode_ensemble_model_dims(MODEL[model], C.byref(ns), C.byref(np_)))
    return ns.value, np_.value


def _ptr(t, dtype, rows: int, ld: int, name: str):
    """Device pointer of a [rows, ld] tensor after checking it really is one."""
    import torch
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor")
    if t.numel() < rows * ld:
        raise ValueError(f"{name}: has {t.numel()} elements, needs {rows}*{ld}")
    if rows > 1 and (t.dim() != 2 or t.shape[1] != ld):
        raise ValueError(f"{name}: expected shape [{rows}, {ld}], got {tuple(t.shape)}")
    del torch
    return t.data_ptr()


def fill_args(args: SolveArgs, n_state: int, *, h0: float, rtol=1e-10, atol=1e-10,
              h_min: float = 1e-12, h_max: float = 1e6, grow: float = 5.0, shrink: float = 0.1,
              t_record: float = float("-inf"), section_period: float = 0.0,
              max_steps: int = 10**8,
              max_equilibrium_steps: int = 0, events: Sequence[dict] = (),
              accessories: Sequence[tuple] = (), record_cap: int = 0) -> None:
    """Scalar options and specs of one solve (paper Sec. 6.4-6.7)."""
    rt = list(rtol) if hasattr(rtol, "__len__") else [rtol] * n_state
    at = list(atol) if hasattr(atol, "__len__") else [atol] * n_state
    for i in range(n_state):
        args.rtol[i], args.atol[i] = float(rt[i]), float(at[i])
    args.h0, args.h_min, args.h_max = float(h0), float(h_min), float(h_max)
    args.grow, args.shrink, args.t_record = float(grow), float(shrink), float(t_record)
    args.section_period = float(section_period)
    args.max_steps, args.max_equilibrium_steps = int(max_steps), int(max_equilibrium_steps)
    if len(events) > MAX_EVENTS or len(accessories) > MAX_ACC:
        raise ValueError("too many events or accessories")
    args.n_events, args.n_accessories = len(events), len(accessories)
    args.event_record_capacity = int(record_cap)
    for j, e in enumerate(events):
        ev = args.events[j]
        ev.component = e["component"]
        ev.direction = e.get("direction", 0)
        ev.stop_after = e.get("stop_after", 0)
        ev.action_component = e.get("action_component", -1)
        ev.action_param = e.get("action_param", -1)
        ev.record_component = e.get("record_component", -1)
        ev.level = e.get("level", 0.0)
        ev.tolerance = e.get("tolerance", 1e-6)
        ev.action_coef = e.get("action_coef", 1.0)
    for k, (kind, comp) in enumerate(accessories):
        args.accessory_specs[k].kind = ACC_KIND[kind]
        args.accessory_specs[k].component = comp


class _Solver:
    """What a solve is for: (model, method, precision) and the launch shape;
    marshals the arguments of one solve."""

    def __init__(self, model: str, method: str, precision: str = "fp64", block_size: int = 0,
                 blocks_per_cu: int = 0):
        load_library()
        self.model, self.method = model, method
        self.n_state, self.n_param = model_dims(model)
        self._desc = Desc(MODEL[model], METHOD[method], PRECISION.get(precision, -1), block_size,
                          blocks_per_cu)

    def outputs(self, ld: int, *, n_accessories: int = 0, n_events: int = 0, record_cap: int = 0,
                device=None) -> dict:
        """Freshly allocated output tensors for a solve of leading dimension ld."""
        import torch
        dev = device or torch.device("cuda", torch.cuda.current_device())
        out = {
            "status": torch.full((ld,), -1, dtype=torch.int32, device=dev),
            "counts": torch.zeros((3, ld), dtype=torch.int64, device=dev),
            "acc": torch.full((2 * n_accessories, ld), float("nan"), dtype=torch.float64,
                              device=dev) if n_accessories else None,
            "event_counts": torch.zeros((n_events, ld), dtype=torch.int32, device=dev)
            if n_events else None,
            "event_records": torch.full((record_cap, 2, ld), float("nan"), dtype=torch.float64,
                                        device=dev) if record_cap else None,
        }
        return out

    def _args(self, time_domain, state, params, next_h, system_index, out, options):
        import torch
        options = dict(options)
        record_start = options.pop("record_start", None)
        tolerances = options.pop("tolerances", None)
        ld = int(time_domain.shape[-1])
        events = list(options.get("events", ()))
        accs = list(options.get("accessories", ()))
        cap = int(options.get("record_cap", 0)) if any(
            e.get("record_component", -1) >= 0 for e in events) else 0
        options = dict(options, record_cap=cap)
        if out is None:
            out = self.outputs(ld, n_accessories=len(accs), n_events=len(events), record_cap=cap,
                               device=time_domain.device)
        n = ld if system_index is None else int(system_index.numel())
        a = SolveArgs()
        a.n_systems, a.ld = n, ld
        f64, i32, i64 = torch.float64, torch.int32, torch.int64
        a.time_domain = _ptr(time_domain, f64, 2, ld, "time_domain")
        a.state = _ptr(state, f64, self.n_state, ld, "state")
        a.params = _ptr(params, f64, self.n_param, ld, "params")
        a.accessories = _ptr(out["acc"], f64, 2 * len(accs), ld, "acc") if accs else None
        a.next_h = _ptr(next_h, f64, 1, ld, "next_h")
        a.status = _ptr(out["status"], i32, 1, ld, "status")
        a.counts = _ptr(out["counts"], i64, 3, ld, "counts") if out.get("counts") is not None else None
        a.event_counts = (_ptr(out["event_counts"], i32, len(events), ld, "event_counts")
                          if events else None)
        if cap:
            rec = out["event_records"]
            if rec is None or rec.numel() < cap * 2 * ld or not rec.is_contiguous():
                raise ValueError("event_records: need a contiguous [cap, 2, ld] float64 tensor")
            a.event_records = rec.data_ptr()
        if system_index is not None:
            if system_index.dtype != i64 or not system_index.is_cuda or not system_index.is_contiguous():
                raise ValueError("system_index: need a contiguous int64 CUDA tensor")
            a.system_index = system_index.data_ptr() if n else None
        if record_start is not None:
            a.record_start = _ptr(record_start, torch.float64, 1, ld, "record_start")
        if tolerances is not None:
            a.tolerances = _ptr(tolerances, torch.float64, 2 * self.n_state, ld, "tolerances")
        fill_args(a, self.n_state, **options)
        return a, out, len(accs)


class Ensemble(_Solver):
    """A solver handle for one (model, method, precision) on the current
    device (paper Sec. 6.2)."""

    def __init__(self, model: str, method: str, precision: str = "fp64", block_size: int = 0,
                 blocks_per_cu: int = 0):
        super().__init__(model, method, precision, block_size, blocks_per_cu)
        h = C.c_void_p()
        _check(load_library().ode_ensemble_create(C.byref(self._desc), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().ode_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = Info()
        _check(load_library().ode_ensemble_query(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def solve(self, time_domain, state, params, *, next_h=None, system_index=None, out=None,
              stream=None, **options: Any) -> dict:
        """Enqueue one integration on ``stream`` (default: torch's current
        stream) and return the output tensors (written asynchronously).

        ``time_domain`` [2, ld], ``state`` [n_state, ld] and ``next_h`` [ld]
        are updated in place; ``params`` [n_param, ld] is read.  Options:
        h0, rtol, atol, h_min, h_max, grow, shrink, t_record, section_period,
        max_steps, max_equilibrium_steps, events, accessories, record_cap.
        """
        import torch
        a, out, _ = self._args(time_domain, state, params, next_h, system_index, out, options)
        if stream is None:
            stream = torch.cuda.current_stream(time_domain.device)
        _check(load_library().ode_ensemble_solve(self._h, C.byref(a), C.c_void_p(stream.cuda_stream)))
        return out

    def tune(self, time_domain, state, params, *, probe_fraction: float = 1.0, next_h=None,
             system_index=None, stream=None, **options: Any) -> dict:
        """Time the candidate launch configurations on private copies of the
        problem (the arguments are only read) and keep the fastest on this
        handle; returns the choice and the probe times."""
        import torch
        a, _, _ = self._args(time_domain, state, params, next_h, system_index, None, options)
        if stream is None:
            stream = torch.cuda.current_stream(time_domain.device)
        r = TuneResult()
        _check(load_library().ode_ensemble_tune(self._h, C.byref(a), float(probe_fraction),
                                                C.c_void_p(stream.cuda_stream), C.byref(r)))
        return {f: getattr(r, f) for f, _ in TuneResult._fields_ if f != "reserved"}

    def plan(self, time_domain, state, params, *, probe_fraction: float = 0.02,
             probe_tolerance_scale: float = 1000.0, next_h=None, system_index=None, stream=None,
             **options: Any):
        """Queue order for a solve of this problem on this handle: a probe on
        private copies over the first ``probe_fraction`` of each horizon, with
        the tolerances multiplied by ``probe_tolerance_scale``, measures every
        system's cost, and 64-system chunks are dealt so that the waves
        sharing a SIMD get a long and a short one.  Returns a CUDA int64
        tensor to pass as ``system_index`` to :meth:`solve` (same other
        arguments); results are bit-identical to the unplanned solve."""
        import torch
        a, _, _ = self._args(time_domain, state, params, next_h, system_index, None, options)
        if stream is None:
            stream = torch.cuda.current_stream(time_domain.device)
        lib = load_library()
        total = C.c_int64(0)
        frac, scale = float(probe_fraction), float(probe_tolerance_scale)
        _check(lib.ode_ensemble_plan(self._h, C.byref(a), frac, scale, None, 0, C.byref(total),
                                     C.c_void_p(stream.cuda_stream)))
        index = torch.empty(max(total.value, 1), dtype=torch.int64, device=time_domain.device)
        _check(lib.ode_ensemble_plan(self._h, C.byref(a), frac, scale,
                                     C.c_void_p(index.data_ptr()), index.numel(), C.byref(total),
                                     C.c_void_p(stream.cuda_stream)))
        return index[:total.value]

    def solve_segments(self, time_domain, state, params, n_segments: int, segment: float, *,
                       first_snapshot: int = 0, snapshots=None, next_h=None, system_index=None,
                       out=None, stream=None, **options: Any) -> dict:
        """``n_segments`` consecutive solves, each from the current time over
        ``segment`` more time units, recorded once as a HIP graph (paper
        Sec. 7: a sweep advanced one excitation period per solve).  Snapshots
        [n_segments - first_snapshot, n_state + 2*n_accessories, ld] of the
        state and the accessories after each segment from ``first_snapshot``
        on are returned in ``out["snapshots"]``."""
        import torch
        a, out, n_acc = self._args(time_domain, state, params, next_h, system_index, out, options)
        ld = int(time_domain.shape[-1])
        n_snap = int(n_segments) - int(first_snapshot)
        rows = self.n_state + 2 * n_acc
        valid = 0 <= int(first_snapshot) <= int(n_segments)   # else the library says EINVAL
        if snapshots is None and n_snap > 0 and valid:
            snapshots = torch.full((n_snap, rows, ld), float("nan"), dtype=torch.float64,
                                   device=time_domain.device)
        if valid and snapshots is not None and (
                snapshots.dtype != torch.float64 or not snapshots.is_contiguous()
                or snapshots.numel() < n_snap * rows * ld):
            raise ValueError("snapshots: need a contiguous float64 tensor of "
                             f"[{n_snap}, {rows}, {ld}]")
        if stream is None:
            stream = torch.cuda.current_stream(time_domain.device)
        snap_ptr = C.c_void_p(snapshots.data_ptr() if (snapshots is not None and n_snap > 0) else None)
        _check(load_library().ode_ensemble_solve_segments(
            self._h, C.byref(a), int(n_segments), float(segment), int(first_snapshot), snap_ptr,
            C.c_void_p(stream.cuda_stream)))
        out["snapshots"] = snapshots
        return out


class NoAllocSolver(_Solver):
    """Solves through ``ode_ensemble_solve_noalloc``: no handle and no device
    allocation in the library (the work-queue counters are the library's
    static device array).  For callers that cannot allocate, e.g. code under
    HIP graph capture; pass preallocated outputs (``outputs``) to allocate
    nothing here either.  Calls whose work overlaps on one GPU race on the
    shared counters: keep them on one stream."""

    def solve(self, time_domain, state, params, *, next_h=None, system_index=None, out=None,
              stream=None, **options: Any) -> dict:
        """As :meth:`Ensemble.solve`."""
        import torch
        a, out, _ = self._args(time_domain, state, params, next_h, system_index, out, options)
        if stream is None:
            stream = torch.cuda.current_stream(time_domain.device)
        _check(load_library().ode_ensemble_solve_noalloc(C.byref(self._desc), C.byref(a),
                                                         C.c_void_p(stream.cuda_stream)))
        return out


class ServedQueue:
    """A served queue (``ode_serve_*``): continuous admission of systems into
    a running persistent launch.  The caller owns the slot pool; this object
    owns the queue's counters and the requests' done flags."""

    def __init__(self, max_requests: int):
        import numpy as np
        L = load_library()
        h = C.c_void_p()
        _check(L.ode_serve_create(int(max_requests), C.byref(h)))
        self._h = h
        self.max_requests = int(max_requests)
        flags = L.ode_serve_done_flags(h)
        self.done = np.ctypeslib.as_array(C.cast(flags, C.POINTER(C.c_int32)),
                                          shape=(self.max_requests,))

    def streams(self, device=None):
        """The queue's own (launch, copy) streams as torch external streams:
        each has a hardware queue of its own, so neither waits behind another
        stream's persistent launch."""
        import torch
        L = load_library()
        return tuple(torch.cuda.ExternalStream(L.ode_serve_stream(self._h, k), device=device)
                     for k in (0, 1))

    def close_queue(self, stream):
        _check(load_library().ode_serve_close(self._h, C.c_void_p(stream.cuda_stream)))

    def reset(self, stream):
        _check(load_library().ode_serve_reset(self._h, C.c_void_p(stream.cuda_stream)))

    def begin_request(self, request: int, n_systems: int, stream):
        _check(load_library().ode_serve_begin_request(self._h, int(request), int(n_systems),
                                                      C.c_void_p(stream.cuda_stream)))

    def publish(self, published: int, stream):
        _check(load_library().ode_serve_publish(self._h, int(published),
                                                C.c_void_p(stream.cuda_stream)))

    def launch(self, ens: "Ensemble", time_domain, state, params, ring, request_of_slot, *,
               out, next_h=None, max_workgroups: int = 0, idle_polls: int = 2000, stream=None,
               **options: Any):
        """Enqueue a served launch of ``ens`` over the slot pool (``ring``:
        int64 position ring [ld]; ``request_of_slot``: int32 [ld])."""
        import torch
        ld = int(time_domain.shape[-1])
        if ring is None or ring.numel() < ld:
            raise ValueError("ring: need an int64 CUDA tensor of one entry per slot")
        a, out, _ = ens._args(time_domain, state, params, next_h, ring, out, options)
        rq = _ptr(request_of_slot, torch.int32, 1, ld, "request_of_slot")
        if stream is None:
            stream = torch.cuda.current_stream(time_domain.device)
        _check(load_library().ode_serve_launch(self._h, ens._h, C.byref(a), C.c_void_p(rq),
                                               int(max_workgroups), int(idle_polls),
                                               C.c_void_p(stream.cuda_stream)))
        return out

    def destroy(self):
        if getattr(self, "_h", None):
            load_library().ode_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy2DAsync.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t,
                                          C.c_size_t, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpy2DAsync.restype = C.c_int
        _hip.hipExtStreamCreateWithCUMask.argtypes = [C.POINTER(C.c_void_p), C.c_uint32,
                                                      C.POINTER(C.c_uint32)]
        _hip.hipExtStreamCreateWithCUMask.restype = C.c_int
    return _hip


def dedicated_stream(device=None):
    """A new stream with a hardware queue of its own, as a torch external
    stream: created over every compute unit with a CU mask
    (hipExtStreamCreateWithCUMask).  Streams without one share the device's
    few hardware queues round-robin, and work on a stream that shares a queue
    with a running persistent launch waits for that launch to end.  The
    stream lives until the process ends."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None \
        else torch.device(device)
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    words = (n_cu + 31) // 32
    mask = (C.c_uint32 * words)(*[(1 << min(32, n_cu - 32 * w)) - 1 for w in range(words)])
    hip = _hip_runtime()
    s = C.c_void_p()
    with torch.cuda.device(dev):
        rc = hip.hipExtStreamCreateWithCUMask(C.byref(s), C.c_uint32(words), mask)
    if rc != 0:
        raise OdeError(EHIP, f"hipExtStreamCreateWithCUMask failed ({rc})")
    return torch.cuda.ExternalStream(s.value, device=dev)


def copy_columns(dst, dst_col: int, src, src_col: int, ncols: int, stream) -> None:
    """Columns [src_col, src_col + ncols) of every row of ``src`` into columns
    [dst_col, dst_col + ncols) of ``dst``, as one strided copy
    (hipMemcpy2DAsync) on ``stream``.  Both are C-contiguous tensors of one
    dtype and the same number of rows (the last axis is the column axis, the
    others are rows); host tensors must be pinned.  Asynchronous."""
    if dst.dtype != src.dtype or not dst.is_contiguous() or not src.is_contiguous():
        raise ValueError("copy_columns: need contiguous tensors of one dtype")
    rows_d, rows_s = dst.numel() // dst.shape[-1], src.numel() // src.shape[-1]
    if rows_d != rows_s:
        raise ValueError(f"copy_columns: {rows_d} rows into {rows_s}")
    if ncols <= 0:
        return
    if dst_col < 0 or src_col < 0 or dst_col + ncols > dst.shape[-1] or src_col + ncols > src.shape[-1]:
        raise ValueError("copy_columns: columns out of range")
    es = dst.element_size()
    rc = _hip_runtime().hipMemcpy2DAsync(
        dst.data_ptr() + dst_col * es, dst.shape[-1] * es, src.data_ptr() + src_col * es,
        src.shape[-1] * es, ncols * es, rows_d, 4, C.c_void_p(stream.cuda_stream))  # 4: by address
    if rc != 0:
        raise OdeError(EHIP, f"hipMemcpy2DAsync failed ({rc})")


def solve_problem(pb, *, device="cuda", block_size: int = 0, stream=None, ens=None):
    """Copy a seeded ``inputs.Problem`` to the device, solve it, and return
    (time_domain, state, outputs) as CUDA tensors (asynchronously written)."""
    import torch
    td = torch.as_tensor(pb.time_domain, device=device).contiguous()
    y = torch.as_tensor(pb.state, device=device).contiguous()
    p = torch.as_tensor(pb.params, device=device).contiguous()
    ens = ens or Ensemble(pb.model, pb.method, block_size=block_size)
    out = ens.solve(td, y, p, stream=stream, **pb.options)
    return td, y, out
