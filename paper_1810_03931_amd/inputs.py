"""Seeded synthetic inputs for the four parameter-sweep workloads.

This module only builds inputs: structure-of-arrays float64 arrays (component
``i`` of system ``s`` at ``[i, s]``, paper Sec. 6.1) plus the solver options.
It performs none of the integration arithmetic, so the HIP path and the CPU
oracle can both consume what it returns.  The paper measures on parameter
sweeps it defines itself (Sec. 7: Duffing damping scan, Keller-Miksis
frequency/amplitude scan, relief-valve flow-rate scan); the sweeps below are
synthetic stand-ins with the same models, tolerances and structure, sized as
the workloads this library is measured on.

The Keller-Miksis coefficient map C0..C12 (paper Sec. 2.2, coefficient list)
is host-side input preparation, as in the paper, where the coefficients are
precomputed so the kernel does less work.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Any

import numpy as np

TWO_PI = 2.0 * math.pi
SEED_BASE = 1810_03931

# Material constants of water at 25 C and the gas (paper Sec. 2.2).
RHO_L = 997.1          # kg/m^3
C_L = 1497.3           # m/s
P_V = 3166.8           # Pa
SIGMA = 0.072          # N/m
MU_L = 8.902e-4        # Pa s (the paper prints "8.902^{-4}"; read as 8.902e-4)
P_INF = 1.0e5          # Pa (1 bar)
GAMMA = 1.4            # polytropic exponent

MODELS = {"duffing": (2, 5), "keller_miksis": (2, 13), "relief_valve": (3, 5), "ballistic": (2, 1),
          "duffing_lyapunov": (4, 5)}


@dataclasses.dataclass
class Problem:
    """One sweep: SoA arrays plus the solver options shared by every system."""

    name: str
    model: str
    method: str
    time_domain: np.ndarray   # [2, N]  (t0, t1)
    state: np.ndarray         # [n_state, N]
    params: np.ndarray        # [n_param, N]
    options: dict[str, Any]

    @property
    def n(self) -> int:
        return self.time_domain.shape[1]

    def copy(self) -> "Problem":
        return dataclasses.replace(
            self, time_domain=self.time_domain.copy(), state=self.state.copy(),
            params=self.params.copy(), options=dict(self.options))

    def subset(self, index) -> "Problem":
        """The systems ``index`` (in that order) as a new, contiguous problem."""
        idx = np.asarray(index, dtype=np.int64)
        return dataclasses.replace(
            self, time_domain=np.ascontiguousarray(self.time_domain[:, idx]),
            state=np.ascontiguousarray(self.state[:, idx]),
            params=np.ascontiguousarray(self.params[:, idx]), options=dict(self.options))

    def with_horizon(self, t1: float, t_record: float | None = None) -> "Problem":
        """Same systems with a different end time (and recording window)."""
        p = self.copy()
        p.time_domain[1, :] = t1
        if t_record is not None:
            p.options["t_record"] = t_record
        return p


def keller_miksis_coefficients(R_E, P_A1, P_A2, f1, f2, theta=0.0, *, paper_literal_c8=False):
    """C0..C12 of the dimensionless Keller-Miksis equation (paper Sec. 2.2).

    Inputs are SI (m, Pa, Hz, rad); ``omega = 2*pi*f``.  The returned array is
    [13, N].  READING: the paper's C8 carries omega_1; differentiating the
    second forcing term p_A2*sin(omega_2 t + theta) gives omega_2, which is what
    is used unless ``paper_literal_c8``.
    """
    R_E, P_A1, P_A2, f1, f2, theta = np.broadcast_arrays(
        *(np.asarray(x, dtype=np.float64) for x in (R_E, P_A1, P_A2, f1, f2, theta)))
    w1 = TWO_PI * f1
    w2 = TWO_PI * f2
    s = TWO_PI / (R_E * w1)            # 2 pi / (R_E omega_1)
    s2 = s * s
    pg0 = P_INF - P_V + 2.0 * SIGMA / R_E
    C = np.empty((13,) + R_E.shape)
    C[0] = pg0 / RHO_L * s2
    C[1] = (1.0 - 3.0 * GAMMA) / (RHO_L * C_L) * pg0 * s
    C[2] = (P_INF - P_V) / RHO_L * s2
    C[3] = 2.0 * SIGMA / (RHO_L * R_E) * s2
    C[4] = 4.0 * MU_L / (RHO_L * R_E * R_E) * (TWO_PI / w1)
    C[5] = P_A1 / RHO_L * s2
    C[6] = P_A2 / RHO_L * s2
    C[7] = R_E * w1 * P_A1 / (RHO_L * C_L) * s2
    C[8] = R_E * (w1 if paper_literal_c8 else w2) * P_A2 / (RHO_L * C_L) * s2
    C[9] = R_E * w1 / (TWO_PI * C_L)
    C[10] = 3.0 * GAMMA
    C[11] = w2 / w1
    C[12] = theta
    return C


def _rng(cfg: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + cfg))


def duffing_rk4_sweep(n: int = 1024) -> Problem:
    """Duffing x'' + k x' + x + x^3 = B cos(w t), RK4 with dt = T/200.

    k = 0.2, w = 1, B on a uniform grid over [0.2, 2]; initial state a seeded
    +-1e-3 jitter around rest; 64 transient + 32 recorded forcing periods; max
    and min of x with their times over the recorded periods.
    """
    g = _rng(1)
    i = np.arange(n, dtype=np.float64)
    B = 0.2 + 1.8 * i / max(n - 1, 1)
    params = np.stack([np.full(n, 0.2), B, np.ones(n), np.ones(n), np.ones(n)])
    state = g.uniform(-1e-3, 1e-3, size=(2, n))
    T = TWO_PI
    td = np.stack([np.zeros(n), np.full(n, 96 * T)])
    opts = dict(h0=T / 200.0, t_record=64 * T, accessories=[("max", 0), ("min", 0)],
                max_steps=2 * 10**7)
    return Problem("duffing_rk4", "duffing", "rk4", td, state, params, opts)


def duffing_rkck45_sweep(n_k: int = 512, n_B: int = 256) -> Problem:
    """Duffing x'' + k x' + x + x^3 = B cos(t), Cash-Karp at rtol = atol = 1e-10.

    2-D grid: k log-uniform over [0.01, 1] (fast index, so neighbouring lanes
    have similar parameters), B uniform over [0.1, 10]; starts at rest;
    1024 transient + 64 recorded periods; local maxima of x located by the
    event x' = 0 with x' decreasing and recorded as (t, x).
    """
    i = np.arange(n_k, dtype=np.float64)
    j = np.arange(n_B, dtype=np.float64)
    k = 10.0 ** (-2.0 + 2.0 * i / max(n_k - 1, 1))
    B = 0.1 + 9.9 * j / max(n_B - 1, 1)
    kk, BB = np.meshgrid(k, B)            # [n_B, n_k]: lane s = j*n_k + i
    n = n_k * n_B
    params = np.stack([kk.ravel(), BB.ravel(), np.ones(n), np.ones(n), np.ones(n)])
    state = np.zeros((2, n))
    T = TWO_PI
    td = np.stack([np.zeros(n), np.full(n, 1088 * T)])
    ev = dict(component=1, level=0.0, direction=-1, tolerance=1e-6, stop_after=0,
              record_component=0)
    opts = dict(h0=1e-3, rtol=1e-10, atol=1e-10, h_min=1e-12, h_max=1e6, grow=5.0, shrink=0.1,
                t_record=1024 * T, events=[ev], record_cap=256, max_steps=2 * 10**7)
    return Problem("duffing_rkck45", "duffing", "rkck45", td, state, params, opts)


def duffing_lyapunov_sweep(n: int = 61440) -> Problem:
    """Largest Lyapunov exponent of the double-well Duffing oscillator
    x'' + k x' - x + x^3 = 0.3 cos(t) (paper Sec. 2.1 and its Duffing4 test),
    Cash-Karp at rtol = atol = 1e-9.

    k on a uniform grid over [0.2, 0.3]; initial state a seeded +-1e-3 jitter
    around the origin, tangent vector r = 1 at angle 0; Poincare sections
    every period 2 pi, where r is reset to 1; 1024 transient + 32 recorded
    periods; the accumulator (sum ln r, count) over the recorded sections.
    """
    g = _rng(5)
    i = np.arange(n, dtype=np.float64)
    k = 0.2 + 0.1 * i / max(n - 1, 1)
    params = np.stack([k, np.full(n, 0.3), np.ones(n), np.full(n, -1.0), np.ones(n)])
    state = np.concatenate([g.uniform(-1e-3, 1e-3, size=(2, n)),
                            np.ones((1, n)), np.zeros((1, n))])
    T = TWO_PI
    td = np.stack([np.zeros(n), np.full(n, 1056 * T)])
    opts = dict(h0=1e-3, rtol=1e-9, atol=1e-9, h_min=1e-12, h_max=1e6, grow=5.0, shrink=0.1,
                t_record=1024 * T, section_period=T, accessories=[("log_reset", 2)],
                max_steps=2 * 10**7)
    return Problem("duffing_lyapunov", "duffing_lyapunov", "rkck45", td, state, params, opts)


def duffing_poincare_sweep(n: int = 30720) -> Problem:
    """The paper's Duffing1/Duffing2 workflow (Sec. 7.1): the double-well
    Duffing oscillator (lin = -1, cub = 1, B = 0.3, omega = 1), k uniform over
    [0.2, 0.3], RK4 with the paper's fixed step 1e-2, advanced one excitation
    period per solve; 1024 transient + 32 kept periods, each kept period
    storing the Poincare point (y1, y2) and the maximum of y1 in the period.

    ``time_domain`` spans one period; ``segments`` = (periods, period,
    first kept period)."""
    g = _rng(6)
    i = np.arange(n, dtype=np.float64)
    k = 0.2 + 0.1 * i / max(n - 1, 1)
    params = np.stack([k, np.full(n, 0.3), np.ones(n), np.full(n, -1.0), np.ones(n)])
    state = g.uniform(-1e-3, 1e-3, size=(2, n))
    T = TWO_PI
    td = np.stack([np.zeros(n), np.full(n, T)])
    opts = dict(h0=1e-2, accessories=[("max", 0)], max_steps=10**6)
    pb = Problem("duffing_poincare", "duffing", "rk4", td, state, params, opts)
    pb.segments = (1056, T, 1024)  # type: ignore[attr-defined]
    return pb


def keller_miksis_sweep(n: int = 1 << 18, *, cluster: bool = True) -> Problem:
    """Dual-frequency Keller-Miksis bubble, Cash-Karp at rtol = atol = 1e-10.

    Independent samples: R_E log-uniform over [1, 10] um, P_A1 and P_A2
    uniform over [0, 2] bar, f1 and f2 log-uniform over [20 kHz, 2 MHz],
    theta = 0; starts at rest (y = (1, 0)); tau in [0, 128] (forcing periods of
    f1) with the last 32 recorded: max and min of R/R_E and their times.
    With ``cluster`` the systems are ordered by R_E*f1 so that neighbouring
    lanes behave alike (paper Sec. 7.2, clustering remark).
    """
    g = _rng(3)
    R_E = 10.0 ** g.uniform(-6.0, -5.0, n)
    P_A1 = g.uniform(0.0, 2.0e5, n)
    P_A2 = g.uniform(0.0, 2.0e5, n)
    lo, hi = math.log10(2.0e4), math.log10(2.0e6)
    f1 = 10.0 ** g.uniform(lo, hi, n)
    f2 = 10.0 ** g.uniform(lo, hi, n)
    if cluster:
        order = np.argsort(R_E * f1, kind="stable")
        R_E, P_A1, P_A2, f1, f2 = (a[order] for a in (R_E, P_A1, P_A2, f1, f2))
    params = keller_miksis_coefficients(R_E, P_A1, P_A2, f1, f2, 0.0)
    state = np.stack([np.ones(n), np.zeros(n)])
    td = np.stack([np.zeros(n), np.full(n, 128.0)])
    opts = dict(h0=1e-4, rtol=1e-10, atol=1e-10, h_min=1e-12, h_max=1e6, grow=5.0, shrink=0.1,
                t_record=96.0, accessories=[("max", 0), ("min", 0)], max_steps=2 * 10**7)
    pb = Problem("keller_miksis", "keller_miksis", "rkck45", td, state, params, opts)
    pb.physical = dict(R_E=R_E, P_A1=P_A1, P_A2=P_A2, f1=f1, f2=f2)  # type: ignore[attr-defined]
    return pb


def relief_valve_sweep(n: int = 1 << 17) -> Problem:
    """Pressure relief valve with impacts, Cash-Karp at rtol = atol = 1e-10.

    q uniform over [0.2, 10]; kappa = 1.25, delta = 10, beta = 20, r = 0.8
    (paper Sec. 2.3); starts closed at rest with y3 = delta; 1024 transient +
    64 recorded units of 2*pi; the impact event y1 = 0 with y1 decreasing
    applies y2 <- -r*y2 (r read from the parameters); max and min of y1 and
    the number of impacts over the recorded interval.
    """
    i = np.arange(n, dtype=np.float64)
    q = 0.2 + 9.8 * i / max(n - 1, 1)
    params = np.stack([np.full(n, 1.25), np.full(n, 10.0), np.full(n, 20.0), q, np.full(n, 0.8)])
    state = np.stack([np.zeros(n), np.zeros(n), np.full(n, 10.0)])
    T = TWO_PI
    td = np.stack([np.zeros(n), np.full(n, 1088 * T)])
    ev = dict(component=0, level=0.0, direction=-1, tolerance=1e-6, stop_after=0,
              action_component=1, action_coef=-1.0, action_param=4)
    opts = dict(h0=1e-3, rtol=1e-10, atol=1e-10, h_min=1e-12, h_max=1e6, grow=5.0, shrink=0.1,
                t_record=1024 * T, events=[ev], accessories=[("max", 0), ("min", 0)],
                max_steps=2 * 10**7)
    return Problem("relief_valve", "relief_valve", "rkck45", td, state, params, opts)


CONFIGS = {
    "duffing_rk4": duffing_rk4_sweep,
    "duffing_rkck45": duffing_rkck45_sweep,
    "keller_miksis": keller_miksis_sweep,
    "relief_valve": relief_valve_sweep,
    "duffing_lyapunov": duffing_lyapunov_sweep,
    "duffing_poincare": duffing_poincare_sweep,
}


def short_horizon(pb: Problem) -> Problem:
    """The same sweep over a short horizon with the window open from t0:
    one forcing period for RK4 Duffing and Keller-Miksis, two for the others
    (two Poincare sections for the Lyapunov sweep)."""
    periods = {"duffing_rk4": 1, "keller_miksis": 1}.get(pb.name, 2)
    T = 1.0 if pb.model == "keller_miksis" else TWO_PI
    return pb.with_horizon(periods * T, t_record=0.0)


def with_tolerance(pb: Problem, tol: float) -> Problem:
    """The same sweep at relative and absolute tolerance ``tol``."""
    p = pb.copy()
    if p.method == "rkck45":
        p.options["rtol"] = tol
        p.options["atol"] = tol
    return p


def stratified_sample(n: int, k: int, seed: int = 0) -> np.ndarray:
    """k distinct system indices spread over [0, n): one per stratum."""
    k = min(k, n)
    g = np.random.Generator(np.random.PCG64(SEED_BASE + 100 + seed))
    edges = np.linspace(0, n, k + 1).astype(np.int64)
    return np.array([g.integers(edges[m], max(edges[m + 1], edges[m] + 1)) for m in range(k)],
                    dtype=np.int64)


# ---------------------------------------------------------------------------
# Served mix: a stream of parameter-sweep requests of mixed model, size and
# horizon.  Each request is a contiguous slice of one of the sweeps of the
# first three workloads (RK4 Duffing, Cash-Karp Duffing, Keller-Miksis), with
# its own horizon; arrival times are a Poisson process.
# ---------------------------------------------------------------------------

SERVED_MODELS = ("duffing_rk4", "duffing_rkck45", "keller_miksis")


@dataclasses.dataclass
class Request:
    rid: int
    problem: Problem
    periods: int


def _served_base(name: str) -> Problem:
    if name == "duffing_rk4":
        return duffing_rk4_sweep(1 << 16)
    if name == "duffing_rkck45":
        return duffing_rkck45_sweep(256, 256)
    return keller_miksis_sweep(1 << 16)


def served_mix(n_requests: int = 600, *, seed: int = 0, tol=(1e-7, 1e-6),
               sizes=(256, 65536), periods=(64, 2048)) -> list[Request]:
    """Requests: model uniform over the three sweeps; size log-uniform over
    ``sizes`` systems (a contiguous slice at a uniform offset); horizon
    log-uniform over ``periods`` forcing periods, the last 1/16 (at least one)
    recorded; adaptive requests at rtol = atol = ``tol``, or, for a range
    (lo, hi), at a tolerance log-uniform over it drawn per request."""
    g = np.random.default_rng(SEED_BASE + 100 + seed)
    bases = {name: _served_base(name) for name in SERVED_MODELS}
    out = []
    for rid in range(n_requests):
        name = SERVED_MODELS[int(g.integers(len(SERVED_MODELS)))]
        base = bases[name]
        m = int(round(10.0 ** g.uniform(math.log10(sizes[0]), math.log10(sizes[1]))))
        m = max(1, min(m, base.n))
        a = int(g.integers(0, base.n - m + 1))
        P = int(round(10.0 ** g.uniform(math.log10(periods[0]), math.log10(periods[1]))))
        T = 1.0 if base.model == "keller_miksis" else TWO_PI
        pb = base.subset(np.arange(a, a + m))
        pb = pb.with_horizon(P * T, t_record=(P - max(1, P // 16)) * T)
        if np.ndim(tol):
            t = float(10.0 ** g.uniform(math.log10(tol[0]), math.log10(tol[1])))
        else:
            t = float(tol)
        pb = with_tolerance(pb, t)
        pb.name = f"{name}#{rid}"
        out.append(Request(rid, pb, P))
    return out


def poisson_arrivals(n: int, qps: float, *, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of rate ``qps``, from 0."""
    g = np.random.default_rng(SEED_BASE + 200 + seed)
    gaps = g.exponential(1.0 / qps, size=n)
    return np.cumsum(gaps) - gaps[0]
