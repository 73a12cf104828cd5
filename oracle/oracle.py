"""Python access to the CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``liboracle.so`` (built by
``oracle/build.py``) and marshals numpy arrays; it shares nothing with the HIP
library or its binding.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# The same source with fused multiply-adds: calibrates parity bars only.
LIB_FMA_PATH = os.path.join(HERE, "liboracle_fma.so")

MODEL = {"duffing": 1, "keller_miksis": 2, "relief_valve": 3, "ballistic": 4,
         "duffing_lyapunov": 5}
METHOD = {"rkck45": 0, "rk4": 1}
ACC = {"max": 1, "min": 2, "log_reset": 3}
DIMS = {"duffing": (2, 5), "keller_miksis": (2, 13), "relief_valve": (3, 5), "ballistic": (2, 1),
        "duffing_lyapunov": (4, 5)}

DONE, STOP_EVENT, STOP_EQUILIBRIUM, FAIL_NAN, MAX_STEPS, BAD_INPUT = range(6)
FLAG_SECANT_CAP = 0x100


class _Event(C.Structure):
    _fields_ = [
        ("component", C.c_int), ("level", C.c_double), ("direction", C.c_int),
        ("tolerance", C.c_double), ("stop_after", C.c_int),
        ("action_component", C.c_int), ("action_coef", C.c_double),
        ("action_param", C.c_int), ("record_component", C.c_int),
    ]


class _Acc(C.Structure):
    _fields_ = [("kind", C.c_int), ("component", C.c_int)]


class _Options(C.Structure):
    _fields_ = [
        ("model", C.c_int), ("method", C.c_int),
        ("rtol", C.c_double * 8), ("atol", C.c_double * 8),
        ("h0", C.c_double), ("h_min", C.c_double), ("h_max", C.c_double),
        ("grow", C.c_double), ("shrink", C.c_double), ("t_record", C.c_double),
        ("section_period", C.c_double), ("record_start", C.POINTER(C.c_double)),
        ("tolerances", C.POINTER(C.c_double)),
        ("max_equilibrium_steps", C.c_int), ("max_steps", C.c_longlong),
        ("n_events", C.c_int), ("n_acc", C.c_int), ("record_cap", C.c_int),
        ("ev", _Event * 4), ("acc", _Acc * 4),
    ]


_lib = None
_lib_fma = None


def lib(variant: str = "plain"):
    """The oracle library; ``variant="fma"`` gives the contracted calibration
    build instead."""
    global _lib, _lib_fma
    if variant == "fma":
        if _lib_fma is None:
            _lib_fma = _load(LIB_FMA_PATH)
        return _lib_fma
    if variant != "plain":
        raise ValueError(f"unknown oracle variant {variant!r}")
    if _lib is None:
        _lib = _load(LIB_PATH)
    return _lib


def _load(path):
    if not os.path.exists(path):
        from oracle import build as _b  # noqa: WPS433
        _b.build()
    L = C.CDLL(path)
    dp, lp, ip = C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.POINTER(C.c_int)
    L.oracle_solve_batch.argtypes = [C.POINTER(_Options), C.c_longlong, C.c_longlong,
                                     dp, dp, dp, dp, dp, ip, lp, ip, dp, lp, C.c_int]
    L.oracle_solve_batch.restype = C.c_int
    L.oracle_rhs.argtypes = [C.c_int, C.c_double, dp, dp, dp]
    L.oracle_rhs.restype = C.c_int
    L.oracle_step.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp, C.c_double, dp, dp]
    L.oracle_step.restype = C.c_int
    L.oracle_cash_karp_tableau.argtypes = [dp, dp, dp, dp, dp]
    L.oracle_model_dims.argtypes = [C.c_int, ip, ip]
    return L


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def tableau():
    """(c[6], a[6,6], b[6], bstar[6], e[6]) exactly as the oracle stores them."""
    c, a, b, bs, e = (np.zeros(6), np.zeros(36), np.zeros(6), np.zeros(6), np.zeros(6))
    lib().oracle_cash_karp_tableau(_ptr(c, C.c_double), _ptr(a, C.c_double), _ptr(b, C.c_double),
                                   _ptr(bs, C.c_double), _ptr(e, C.c_double))
    return c, a.reshape(6, 6), b, bs, e


def rhs(model, t, y, p):
    y = np.ascontiguousarray(y, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    f = np.zeros_like(y)
    rc = lib().oracle_rhs(MODEL[model], float(t), _ptr(y, C.c_double), _ptr(p, C.c_double),
                          _ptr(f, C.c_double))
    assert rc == 0
    return f


def step(model, method, t, y, p, h):
    """One method step; returns (y_new, err) (err is None for RK4)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    yn = np.zeros_like(y)
    err = np.zeros_like(y)
    rc = lib().oracle_step(MODEL[model], METHOD[method], float(t), _ptr(y, C.c_double),
                           _ptr(p, C.c_double), float(h), _ptr(yn, C.c_double),
                           _ptr(err, C.c_double))
    assert rc == 0
    return yn, (err if method == "rkck45" else None)


def make_options(model, method, *, h0, rtol=1e-10, atol=1e-10, h_min=1e-12, h_max=1e6,
                 grow=5.0, shrink=0.1, t_record=-np.inf, section_period=0.0,
                 max_equilibrium_steps=0,
                 max_steps=10**9, events=(), accessories=(), record_cap=0):
    o = _Options()
    o.model, o.method = MODEL[model], METHOD[method]
    ns = DIMS[model][0]
    rt = np.broadcast_to(np.asarray(rtol, dtype=np.float64), (ns,))
    at = np.broadcast_to(np.asarray(atol, dtype=np.float64), (ns,))
    for i in range(ns):
        o.rtol[i], o.atol[i] = float(rt[i]), float(at[i])
    o.h0, o.h_min, o.h_max, o.grow, o.shrink = h0, h_min, h_max, grow, shrink
    o.t_record, o.section_period = t_record, section_period
    o.max_equilibrium_steps, o.max_steps = max_equilibrium_steps, max_steps
    o.n_events, o.n_acc, o.record_cap = len(events), len(accessories), record_cap
    for j, e in enumerate(events):
        ev = o.ev[j]
        ev.component = e["component"]
        ev.level = e.get("level", 0.0)
        ev.direction = e.get("direction", 0)
        ev.tolerance = e.get("tolerance", 1e-6)
        ev.stop_after = e.get("stop_after", 0)
        ev.action_component = e.get("action_component", -1)
        ev.action_coef = e.get("action_coef", 1.0)
        ev.action_param = e.get("action_param", -1)
        ev.record_component = e.get("record_component", -1)
    for a, spec in enumerate(accessories):
        kind, comp = spec
        o.acc[a].kind, o.acc[a].component = ACC[kind], comp
    return o


def solve(model, method, time_domain, state, params, *, next_h=None, index=None, threads=0,
          record_start=None, tolerances=None, variant="plain", **opts):
    """Integrate every system (or those in ``index``) in place.

    ``time_domain`` [2, ld], ``state`` [n_state, ld] and ``params``
    [n_param, ld] are float64 SoA arrays; ``time_domain`` and ``state`` are
    overwritten with the final time and state (and so is ``next_h`` if given).
    Returns a dict with status, counts, acc, event_counts, event_records.
    ``variant="fma"`` runs the contracted calibration build.
    """
    o = make_options(model, method, **opts)
    if record_start is not None:
        record_start = np.ascontiguousarray(record_start, dtype=np.float64)
        assert record_start.shape == (time_domain.shape[1],)
        o.record_start = _ptr(record_start, C.c_double)
    if tolerances is not None:
        tolerances = np.ascontiguousarray(tolerances, dtype=np.float64)
        assert tolerances.shape == (2 * DIMS[model][0], time_domain.shape[1])
        o.tolerances = _ptr(tolerances, C.c_double)
    td = np.ascontiguousarray(time_domain, dtype=np.float64)
    st = np.ascontiguousarray(state, dtype=np.float64)
    pr = np.ascontiguousarray(params, dtype=np.float64)
    assert td is time_domain and st is state, "time_domain/state must be C-contiguous float64"
    ld = td.shape[1]
    n = ld if index is None else len(index)
    idx = None if index is None else np.ascontiguousarray(index, dtype=np.int64)
    acc = np.full((max(2 * o.n_acc, 1), ld), np.nan)
    status = np.full(ld, -1, dtype=np.int32)
    counts = np.zeros((3, ld), dtype=np.int64)
    evc = np.zeros((max(o.n_events, 1), ld), dtype=np.int32)
    rec = np.full((max(o.record_cap, 1), 2, ld), np.nan)
    rc = lib(variant).oracle_solve_batch(
        C.byref(o), n, ld, _ptr(td, C.c_double), _ptr(st, C.c_double), _ptr(pr, C.c_double),
        _ptr(acc, C.c_double), _ptr(next_h, C.c_double), _ptr(status, C.c_int),
        _ptr(counts, C.c_longlong), _ptr(evc, C.c_int), _ptr(rec, C.c_double),
        _ptr(idx, C.c_longlong), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the options")
    return {
        "status": status, "counts": counts, "acc": acc[: 2 * o.n_acc],
        "event_counts": evc[: o.n_events], "event_records": rec[: o.record_cap],
    }
