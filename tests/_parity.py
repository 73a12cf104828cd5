"""Shared helpers of the GPU parity tests: run the oracle and the HIP path on
the same seeded inputs and compare element by element.

The bars below are fixed by the oracle alone, before any GPU result is looked
at, and their constants are calibrated on the CPU.

1. Integers (status, step counts, event counts) are identical on every system
   whose step sequence matches the oracle's ("same-step" systems).

2. Every floating-point output of a same-step system has its own bar,
       |gpu - oracle| <= max(1e-11, FACTOR * floor)          (relative),
   where ``floor`` is that output's conditioning floor, measured with the
   oracle alone: the largest change of the output among four twin runs whose
   inputs move by rounding-level amounts -- the initial state moved by
   +-1e-15 * max(1, |y0|) (two sign patterns), and every parameter scaled by
   (1 + 2^-52) and by (1 - 2^-53), about one ulp, which changes the rounding
   of the right-hand side at every step.  Final states, the final time,
   accessory values, accessory times, record times and record values each
   have a floor of their own, so an output that is sensitive to a tie-break
   (which of two nearly equal maxima comes first) cannot loosen the bar of
   another.  "Relative" is per system against the size of its state vector:
   |a_i - b_i| <= rel * max(|b_i|, max_j |b_j|), since a component that passes
   through zero is judged against the state's magnitude, as the integrator's
   own error control does; times are relative to max(1, |t1|).
   A system is "held" when FACTOR * floor of its final state is at most 1e-11,
   i.e. it is judged at exactly 1e-11.
   FACTOR = 100 is calibrated with the FMA-contracted build of the oracle (the
   same source, other roundings at every operation): on the 4999-system
   short-horizon subsets of all four sweeps its final states stay within 21x
   the floor (init twins alone) and within 6x (all four twins).

3. "Loose" systems are flips (unequal step counts, status or event counts:
   a decision that rounding tipped) and fragile systems (a twin already
   changes the step counts or the status).  Their number is capped at
   max(ceil(0.1% n), 3 L), where L is the number of systems the FMA build
   takes off the oracle's step sequence on the same inputs (computed beside
   the oracle).  Their final states must agree within
       min(LOOSE_CAP, max(100 * tol, FACTOR * floor))
   with tol the problem's largest tolerance: two valid step sequences each
   keep the local error below tol, so over a short horizon they differ by a
   small multiple of it, amplified as the twins show.  A system whose bar would
   exceed LOOSE_CAP = 1e-3 is "undetermined": the twins show that the plain
   definition does not fix its answer to 1e-3, so it is checked for validity
   only (status, finiteness, final time) and counts towards the cap.  No
   floor-based raise goes above 1e-3.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle import oracle as O

REL = 1e-11
FACTOR = 100.0
LOOSE_CAP = 1e-3


def run_oracle(pb, threads: int = 0, variant: str = "plain") -> dict:
    td, y = pb.time_domain.copy(), pb.state.copy()
    r = O.solve(pb.model, pb.method, td, y, pb.params, threads=threads, variant=variant,
                **pb.options)
    r["t"], r["y"], r["t1"] = td[0], y, td[1]
    return r


def run_gpu(pb, *, block_size: int = 0, index=None, ens=None, precision: str = "fp64",
            next_h=None) -> dict:
    import torch
    from paper_1810_03931_amd import ensemble as E
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(pb.time_domain, device=dev).contiguous()
    y = torch.as_tensor(pb.state, device=dev).contiguous()
    p = torch.as_tensor(pb.params, device=dev).contiguous()
    hn = None if next_h is None else torch.as_tensor(next_h, device=dev).contiguous()
    ens = ens or E.Ensemble(pb.model, pb.method, precision=precision, block_size=block_size)
    sidx = None if index is None else torch.as_tensor(np.asarray(index, dtype=np.int64), device=dev)
    out = ens.solve(td, y, p, system_index=sidx, next_h=hn, **pb.options)
    torch.cuda.synchronize()
    r = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    r["t"], r["y"], r["t1"] = td[0].cpu().numpy(), y.cpu().numpy(), td[1].cpu().numpy()
    if hn is not None:
        r["next_h"] = hn.cpu().numpy()
    if r.get("acc") is None:
        r["acc"] = np.zeros((0, pb.n))
    if r.get("event_counts") is None:
        r["event_counts"] = np.zeros((0, pb.n), dtype=np.int32)
    if r.get("event_records") is None:
        r["event_records"] = np.zeros((0, 2, pb.n))
    return r


def adiff(a, b):
    """|a - b| where NaN on both sides counts as equal and NaN on one side as
    infinitely far."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        d = np.abs(a - b)
    d = np.where(np.isnan(a) & np.isnan(b), 0.0, d)
    return np.where(np.isnan(d), np.inf, d)


def rel_err(a, b, scale):
    return adiff(a, b) / np.maximum(np.maximum(np.abs(np.nan_to_num(b)), scale), 1e-300)


def scales(o):
    """Per-system magnitude of the final state and of the time axis."""
    scale = np.maximum(np.max(np.abs(np.nan_to_num(o["y"])), axis=0), 1e-300)
    tscale = np.maximum(np.abs(o["t1"]), 1.0)
    return scale, tscale


def distances(a: dict, o: dict) -> dict:
    """Relative distance of result ``a`` from result ``o`` per output and per
    system: final state ``y`` [n], final time ``t`` [n], accessory values
    ``accv`` and times ``acct`` [n_acc, n], record times ``rect`` and values
    ``recv`` [n] (largest over the record slots)."""
    scale, tscale = scales(o)
    n = o["y"].shape[1]
    d = {"y": np.max(rel_err(a["y"], o["y"], scale[None, :]), axis=0),
         "t": adiff(a["t"], o["t"]) / tscale,
         # each component against its own size (at least 1)
         "yc": adiff(a["y"], o["y"]) / np.maximum(np.abs(np.nan_to_num(o["y"])), 1.0)}
    if o["acc"].shape[0]:
        d["accv"] = rel_err(a["acc"][0::2], o["acc"][0::2], scale[None, :])
        d["acct"] = adiff(a["acc"][1::2], o["acc"][1::2]) / tscale[None, :]
        # accessory values against their own size (at least 1)
        d["accl"] = adiff(a["acc"][0::2], o["acc"][0::2]) / np.maximum(
            np.abs(np.nan_to_num(o["acc"][0::2])), 1.0)
    else:
        d["accv"] = d["acct"] = d["accl"] = np.zeros((0, n))
    if o["event_records"].shape[0]:
        rec_a, rec_o = a["event_records"], o["event_records"]
        d["rect"] = np.max(adiff(rec_a[:, 0], rec_o[:, 0]) / tscale[None, :], axis=0)
        d["recv"] = np.max(rel_err(rec_a[:, 1], rec_o[:, 1], scale[None, :]), axis=0)
    else:
        d["rect"] = d["recv"] = np.zeros(n)
    return d


def same_path(a: dict, o: dict) -> np.ndarray:
    """Systems on which ``a`` took the step sequence of ``o``: equal step
    counts (accepted, rejected, location), status and event counts."""
    m = np.all(a["counts"] == o["counts"], axis=0) & (a["status"] == o["status"])
    if o["event_counts"].shape[0]:
        m &= np.all(a["event_counts"] == o["event_counts"], axis=0)
    return m


def short_twins(pb) -> list:
    """The four rounding-level twins of a problem (see the module notes)."""
    ns = pb.state.shape[0]
    size = np.maximum(np.max(np.abs(pb.state), axis=0), 1.0)
    out = []
    for pattern in (np.ones(ns), (-1.0) ** np.arange(ns)):
        tw = pb.copy()
        tw.state = tw.state + 1e-15 * pattern[:, None] * size[None, :]
        out.append(tw)
    for f in (1.0 + 2.0 ** -52, 1.0 - 2.0 ** -53):
        tw = pb.copy()
        tw.params = tw.params * f
        out.append(tw)
    return out


def tolerance_of(pb) -> float:
    """The largest of the problem's tolerances (0 for fixed-step RK4)."""
    if pb.method != "rkck45":
        return 0.0
    return float(max(np.max(pb.options.get("rtol", 1e-10)), np.max(pb.options.get("atol", 1e-10))))


@dataclasses.dataclass
class Reference:
    """The oracle's result with everything the bars need."""

    o: dict
    floor: dict           # per output, as returned by distances()
    fragile: np.ndarray   # a twin left the oracle's step sequence
    cap: int              # most loose systems allowed
    tol: float
    fma_loose: int        # systems the FMA build took off the step sequence


def reference(pb, threads: int = 0, calibrate: bool = True) -> Reference:
    """Oracle run, per-output conditioning floors from the four twins, and the
    loose-system cap from the FMA calibration build."""
    o = run_oracle(pb, threads)
    floor = {k: np.zeros(np.shape(v)) for k, v in distances(o, o).items()}
    fragile = np.zeros(pb.n, dtype=bool)
    for tw in short_twins(pb):
        ot = run_oracle(tw, threads)
        fragile |= ~same_path(ot, o)
        for k, v in distances(ot, o).items():
            bad = ~np.isfinite(v)
            fragile |= bad if v.ndim == 1 else np.any(bad, axis=0)
            floor[k] = np.maximum(floor[k], np.where(np.isfinite(v), v, 0.0))
    fma_loose = 0
    if calibrate:
        of = run_oracle(pb, threads, variant="fma")
        fma_loose = int(np.sum(~same_path(of, o) | fragile))
    cap = max(int(np.ceil(1e-3 * pb.n)), 3 * fma_loose)
    return Reference(o, floor, fragile, cap, tolerance_of(pb), fma_loose)


def check(pb, g, *, label: str = "", **kw) -> dict:
    """Oracle reference of ``pb``, then compare the GPU result ``g`` with it."""
    return compare(g, reference(pb), label=label, **kw)


def take(r: dict, idx) -> dict:
    """The systems idx of a result (columns of every array)."""
    idx = np.asarray(idx)
    out = {}
    for k, v in r.items():
        if v is None:
            out[k] = None
        elif v.ndim == 1:
            out[k] = v[idx]
        elif v.ndim == 2:
            out[k] = v[:, idx]
        else:
            out[k] = v[..., idx]
    return out


def compare(g: dict, ref: Reference, *, rel: float = REL, min_held: float = 0.0,
            label: str = "") -> dict:
    """Element-wise parity of a GPU result ``g`` with the oracle reference."""
    o, fl, fragile = ref.o, ref.floor, ref.fragile
    n = o["y"].shape[1]
    steady = ~fragile
    wrong = np.flatnonzero(steady & (g["status"] != o["status"]))
    same = same_path(g, o) & steady
    loose = ~same
    d = distances(g, o)
    bars = {k: np.maximum(rel, FACTOR * v) for k, v in fl.items()}
    held = same & (FACTOR * fl["y"] <= rel)
    lbar = np.maximum(max(100.0 * ref.tol, rel), FACTOR * fl["y"])
    undetermined = loose & (lbar > LOOSE_CAP)
    checked_loose = loose & ~undetermined & (g["status"] == o["status"])
    stats = {"n": n, "same_steps": int(same.sum()), "flips": int(np.sum(loose & steady)),
             "fragile": int(fragile.sum()), "undetermined": int(undetermined.sum()),
             "loose_cap": ref.cap, "fma_loose": ref.fma_loose,
             "held_1e-11": int(held.sum()),
             "max_rel_y_held": float(d["y"][held].max(initial=0)),
             "max_rel_y": float(d["y"][same].max(initial=0)),
             "max_bar_y": float(bars["y"][same].max(initial=0)),
             "max_rel_t": float(d["t"][same].max(initial=0))}
    if d["accv"].shape[0]:
        stats["max_rel_accv"] = float(d["accv"][:, same].max(initial=0))
        stats["max_rel_acct"] = float(d["acct"][:, same].max(initial=0))
    if o["event_records"].shape[0]:
        stats["max_rel_rec"] = float(np.maximum(d["rect"], d["recv"])[same].max(initial=0))
    if checked_loose.any():
        stats["max_rel_y_loose"] = float(d["y"][checked_loose].max())
    assert wrong.size == 0, f"{label}: status differs on {wrong.size} systems: {wrong[:5]}"
    assert int(loose.sum()) <= ref.cap, \
        f"{label}: {int(loose.sum())} systems off the oracle's step sequence (cap {ref.cap}): {stats}"
    for k in ("y", "t", "accv", "acct", "rect", "recv"):
        e, b = d[k], bars[k]
        over = (e > b) & same if e.ndim == 1 else np.any((e > b) & same[None, :], axis=0)
        bad = np.flatnonzero(over)
        assert bad.size == 0, (f"{label}: output {k} beyond its bar on {bad.size} same-step "
                               f"systems: first {bad[:5]}, err "
                               f"{(e[bad[:5]] if e.ndim == 1 else e[:, bad[:5]].max(axis=0))}, "
                               f"bar {(b[bad[:5]] if b.ndim == 1 else b[:, bad[:5]].min(axis=0))}")
    bad = np.flatnonzero(checked_loose & (d["y"] > lbar))
    assert bad.size == 0, (f"{label}: loose systems beyond min(1e-3, max(100 tol, "
                           f"{FACTOR:g} floor)): {bad[:5]}, err {d['y'][bad[:5]]}, "
                           f"bar {lbar[bad[:5]]}")
    eq = loose & (g["status"] == o["status"])
    assert np.array_equal(np.isfinite(g["y"][:, eq]), np.isfinite(o["y"][:, eq])), \
        f"{label}: finiteness differs on loose systems"
    done = eq & (o["status"] == 0)
    assert np.array_equal(g["t"][done], o["t"][done]), f"{label}: final time of loose systems"
    assert held.sum() >= min_held * n, \
        f"{label}: only {int(held.sum())} of {n} systems held at {rel:g} (minimum {min_held:.2%})"
    return stats


# ---------------------------------------------------------------------------
# Long horizons (the full transient and recording window), on a sample.
#
# Only systems whose answer the definition fixes are compared: "stable"
# systems, for which four oracle twins -- the initial state moved by a
# relative 1e-9, every parameter scaled by (1 + 2^-52), and the state at the
# window start moved by +-1e-15 -- end within 1e-9 of the oracle in the final
# state and the accessory values, with the same event counts.  The screen
# uses the oracle alone and is the same for every sweep.
#
# Restart parity: a decision flip in the transient moves a system to another,
# equally valid step grid, and on a long horizon the grids never meet again.
# Both the oracle and the GPU therefore integrate in two solves, split at the
# window start (a split solve continues exactly as the single one would).  The
# recording window is compared against the oracle's own window run when the
# GPU's transient took the oracle's step sequence, and otherwise against the
# oracle's window run restarted from the GPU's checkpoint (time, state, next
# step).  Inside the window, stable same-step systems are held to 1e-8 on the
# final state, the accessory values, the record times and values, and the
# accessory times -- or, for a time off by more than that, the oracle's own
# trajectory must reach the extremum at the GPU's time within 2e-8 (a maximum
# that recurs every period up to rounding has no unique first time).  Flips inside the window
# are capped in number and bounded by a bar calibrated with the FMA build run
# over the window from the oracle's checkpoint: max(ceil(1% stable), 3 F) flips
# for the F the FMA build makes, within min(1e-3, max(1e-8, 10 x the FMA
# flips' largest error)).
# ---------------------------------------------------------------------------

LONG_REL = 1e-8
STABLE_REL = 1e-9


def long_twins(pb) -> list:
    a = pb.copy()
    a.state = a.state * (1.0 + 1e-9) + 1e-12
    b = pb.copy()
    b.params = b.params * (1.0 + 2.0 ** -52)
    return [a, b]


def transient_part(pb, t_split):
    """The problem up to the window start (t1 clipped to ``t_split``)."""
    pre = pb.copy()
    pre.time_domain[1] = np.minimum(pre.time_domain[1], t_split)
    return pre


def window_part(pb, t, y):
    """The problem from the checkpoint (t, y) to the original end."""
    w = pb.copy()
    w.time_domain = np.ascontiguousarray(np.stack([t, pb.time_domain[1]]))
    w.state = np.ascontiguousarray(y)
    return w


def oracle_solve(pb, next_h, threads: int = 0, variant: str = "plain") -> dict:
    """One oracle solve that continues from (and updates) ``next_h``."""
    td, y = pb.time_domain.copy(), pb.state.copy()
    r = O.solve(pb.model, pb.method, td, y, pb.params, next_h=next_h, threads=threads,
                variant=variant, **pb.options)
    r["t"], r["y"], r["t1"], r["next_h"] = td[0], y, td[1], next_h.copy()
    return r


@dataclasses.dataclass
class LongReference:
    o1: dict                 # oracle over the transient
    o2: dict                 # oracle over the window from its own checkpoint
    stable: np.ndarray
    window_cap: int
    flip_bar_y: float
    flip_bar_acc: float
    fma_window_flips: int


def long_reference(pb, threads: int = 0) -> LongReference:
    t_rec = float(pb.options.get("t_record", -np.inf))
    hn = np.zeros(pb.n)
    o1 = oracle_solve(transient_part(pb, t_rec), hn, threads)
    ck_t, ck_y, ck_h = o1["t"].copy(), o1["y"].copy(), o1["next_h"].copy()
    o2 = oracle_solve(window_part(pb, ck_t, ck_y), ck_h.copy(), threads)
    evc = o1["event_counts"] + o2["event_counts"]
    stable = o2["status"] == 0
    for tw in long_twins(pb):
        ot = run_oracle(tw, threads)
        d = distances(ot, o2)
        dist = np.maximum(d["y"], d["accv"].max(axis=0, initial=0))
        stable &= (ot["status"] == o2["status"]) & (dist <= STABLE_REL)
        if evc.shape[0]:
            stable &= np.all(ot["event_counts"] == evc, axis=0)
    # Window-start twins: the checkpoint moved by +-1e-15 * max(1, |y|).  On a
    # contracting orbit the twins above have decayed back onto the oracle's
    # arithmetic by the window start, so they cannot see how rounding inside
    # the window moves a grid extremum (the minimum radius of a violent
    # collapse moves by up to 1e-5 for a 1e-15 change of the state there).
    size = np.maximum(np.abs(ck_y), 1.0)
    for sgn in (1.0, -1.0):
        ow = oracle_solve(window_part(pb, ck_t, ck_y + sgn * 1e-15 * size), ck_h.copy(), threads)
        d = distances(ow, o2)
        dist = np.maximum(d["y"], d["accv"].max(axis=0, initial=0))
        stable &= (ow["status"] == o2["status"]) & (dist <= STABLE_REL)
        if o2["event_counts"].shape[0]:
            stable &= np.all(ow["event_counts"] == o2["event_counts"], axis=0)
    f2 = oracle_solve(window_part(pb, ck_t, ck_y), ck_h.copy(), threads, variant="fma")
    fw = stable & ~same_path(f2, o2)
    d = distances(f2, o2)
    ey = float(d["y"][fw].max(initial=0))
    ea = float(d["accv"][:, fw].max(initial=0))
    cap = max(int(np.ceil(0.01 * stable.sum())), 3 * int(fw.sum()))
    bar_y = min(LOOSE_CAP, max(LONG_REL, 10.0 * ey))
    bar_a = min(LOOSE_CAP, max(LONG_REL, 10.0 * ea))
    return LongReference(o1, o2, stable, cap, bar_y, bar_a, int(fw.sum()))


def restart_reference(pb, ref: LongReference, g1: dict, threads: int = 0):
    """The window reference for every system: the oracle's own window run, or,
    where the GPU's transient left the oracle's step sequence, the oracle's
    window run from the GPU's checkpoint.  Returns (reference, restarted)."""
    restarted = ~same_path(g1, ref.o1)
    r2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ref.o2.items()}
    # the checkpoint each window reference starts from
    r2["ck_t"], r2["ck_y"], r2["ck_h"] = ref.o1["t"].copy(), ref.o1["y"].copy(), \
        ref.o1["next_h"].copy()
    idx = np.flatnonzero(restarted)
    if idx.size:
        sub = pb.subset(idx)
        w = window_part(sub, g1["t"][idx], g1["y"][:, idx])
        rr = oracle_solve(w, np.ascontiguousarray(g1["next_h"][idx]), threads)
        for k, v in rr.items():
            if isinstance(v, np.ndarray) and k in r2 and v.size:
                r2[k][..., idx] = v
        r2["ck_t"][idx], r2["ck_y"][:, idx] = g1["t"][idx], g1["y"][:, idx]
        r2["ck_h"][idx] = g1["next_h"][idx]
    return r2, restarted


# The bar of a tied time follows from the two bars the GPU is held to inside
# the window: its value at its time is within LONG_REL of the reference's
# extremum, and its trajectory within LONG_REL of the reference's, so at the
# GPU's time the reference is within 2 LONG_REL of its extremum.
# (Rounding-level ties sit far below it -- periodic RK4 maxima within 4e-15;
# located impact minima of the valve, set by the secant's last iterate,
# within 7e-11 -- and one grid step off a maximum is 3e-4.)
TIE_REL = 2.0 * LONG_REL


def tied_time_check(pb, g2: dict, r2: dict, ref: LongReference, threads: int = 0) -> dict:
    """An accessory time is the first accepted point at which the extremum is
    reached (strict > / <).  Where the extremum recurs up to rounding -- once
    per period of a periodic orbit sampled on a phase-locked grid -- which
    recurrence comes "first" is a rounding decision, and two evaluations of
    the same definition can pick different periods.  So a stable same-step
    system whose accessory time differs from the reference's beyond 1e-8 is
    checked for what the definition does fix: at the GPU's time, the
    reference's own trajectory reaches the extremum within TIE_REL (relative
    to the state's size), the sum of the value's and the trajectory's bars.  The oracle integrates from the reference's
    checkpoint to the GPU's time (the last step clipped to land on it)."""
    same = same_path(g2, r2) & ref.stable
    d = distances(g2, r2)
    kinds = pb.options.get("accessories", [])
    scale, _ = scales(r2)
    checked, worst = 0, 0.0
    for k, (kind, comp) in enumerate(kinds):
        if kind not in ("max", "min"):
            continue
        idx = np.flatnonzero(same & (d["acct"][k] > LONG_REL))
        if not idx.size:
            continue
        sub = pb.subset(idx)
        w = window_part(sub, r2["ck_t"][idx], r2["ck_y"][:, idx])
        w.time_domain[1] = g2["acc"][2 * k + 1, idx]
        w.options["accessories"] = []
        # events stay (their actions shape the trajectory); records are not needed
        w.options["events"] = [dict(e, record_component=-1) for e in w.options.get("events", [])]
        w.options["record_cap"] = 0
        at = oracle_solve(w, np.ascontiguousarray(r2["ck_h"][idx]), threads)
        gap = adiff(at["y"][comp], r2["acc"][2 * k, idx]) / scale[idx]
        checked += idx.size
        worst = max(worst, float(gap.max()))
        bad = idx[gap > TIE_REL]
        assert bad.size == 0, (f"accessory {k}: at the GPU's time the oracle is "
                               f"{gap[gap > TIE_REL][:5]} away from its extremum on systems {bad[:5]}")
    return {"tied_times_checked": checked, "max_rel_tie_gap": worst}


def compare_window(g2: dict, r2: dict, ref: LongReference, *, label: str = "", pb=None) -> dict:
    """Parity of the GPU's window run with the window reference (see above)."""
    st_mask = ref.stable
    same = same_path(g2, r2) & st_mask
    flips = st_mask & ~same
    d = distances(g2, r2)
    stats = {"stable": int(st_mask.sum()), "same_steps": int(same.sum()),
             "window_flips": int(flips.sum()), "window_cap": ref.window_cap,
             "fma_window_flips": ref.fma_window_flips,
             "max_rel_y": float(d["y"][same].max(initial=0)),
             "max_rel_accv": float(d["accv"][:, same].max(initial=0)),
             "acc_times_equal_1e-8": int(np.sum((d["acct"] <= LONG_REL) & same[None, :])),
             "max_rel_rec": float(np.maximum(d["rect"], d["recv"])[same].max(initial=0)),
             "flip_bar_y": ref.flip_bar_y, "flip_bar_acc": ref.flip_bar_acc,
             "max_rel_y_flips": float(d["y"][flips].max(initial=0)),
             "max_rel_accv_flips": float(d["accv"][:, flips].max(initial=0))}
    assert np.array_equal(g2["status"][st_mask], r2["status"][st_mask]), f"{label}: status"
    assert int(flips.sum()) <= ref.window_cap, f"{label}: window flips {stats}"
    for k, mask in (("y", same), ("t", same), ("rect", same), ("recv", same)):
        bad = np.flatnonzero(mask & (d[k] > LONG_REL))
        assert bad.size == 0, f"{label}: {k} beyond 1e-8 on {bad[:5]}: {d[k][bad[:5]]} ({stats})"
    over = np.any((d["accv"] > LONG_REL) & same[None, :], axis=0)
    assert not over.any(), f"{label}: accessory values beyond 1e-8 on {np.flatnonzero(over)[:5]} ({stats})"
    # accessory times: equal within 1e-8, or a tie the definition leaves open
    over = np.any((d["acct"] > LONG_REL) & same[None, :], axis=0)
    if pb is None:
        assert not over.any(), f"{label}: accessory times beyond 1e-8 on {np.flatnonzero(over)[:5]} ({stats})"
    else:
        stats.update(tied_time_check(pb, g2, r2, ref))
    assert np.all(d["y"][flips] <= ref.flip_bar_y), f"{label}: flipped final states ({stats})"
    assert np.all(d["accv"][:, flips] <= ref.flip_bar_acc), f"{label}: flipped accessories ({stats})"
    return stats
