"""Throughput benchmark of the ensemble integrator on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config NAME] [--no-cpu-baseline]

A step is one full solve of a parameter sweep (every system integrated over
its whole horizon, all events, accessories and records), starting from the
same seeded inputs already resident in HBM.  Prints ONE JSON line with
accepted system-steps/s over the timed steps, the FP64 roofline position of
the integrator kernel (timed with HIP events on the stream it runs on) and
the CPU oracle timed on a bounded sample of the same sweep.

Default workload: Duffing x'' + k x' + x + x^3 = B cos t, Cash-Karp at
rtol = atol = 1e-10, 2^17 systems on a (k, B) grid, 1088 forcing periods,
local maxima of x located by events and recorded over the last 64.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1810_03931_amd import inputs as I  # noqa: E402  (input generators only)

METRIC = "system-steps/s + % FP64 VALU peak (RKCK45 sweep); p50/p99 sweep latency"
FP64_PEAK_TFLOPS = 78.6     # MI355X: 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk/CU

# FP64 FLOP per attempted step of one system (the roofline's per-unit figure).
# Calibrated with hardware counters on a lock-step input (bench.py --uniform S:
# every lane has the parameters of system S, so no lane is masked):
#   FLOP = 64*(ADD + MUL + TRANS) + 128*FMA of SQ_INSTS_VALU_*_F64, / attempts.
# The figure includes the FP64 work the math library does inside cos/sin/pow.
# It is read from profiles/<workload>_fp64_counters.txt ("uniform" block).
# Workloads without a calibration fall back to a count from the formulas
# (FMA = 2, add/mul/div/sqrt = 1) plus 40 FLOP per library transcendental.
FLOPS_ESTIMATE = {
    ("duffing", "rk4"): 70 + 4 * 40,
    ("duffing", "rkck45"): 191 + 7 * 40,
    ("keller_miksis", "rkck45"): 359 + 19 * 40,
    ("relief_valve", "rkck45"): 237 + 7 * 40,
    ("duffing_lyapunov", "rkck45"): 875,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="duffing_rkck45",
                    choices=sorted(I.CONFIGS))
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="cap on resident workgroups per compute unit (0: all that fit)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch configuration (untimed) before the warmup")
    ap.add_argument("--eager", action="store_true",
                    help="repeated-horizon workloads: time the host loop of solve calls "
                         "instead of the recorded graph")
    ap.add_argument("--plan", type=float, default=-1.0, metavar="FRACTION",
                    help="plan the queue order inside every timed step from a probe over this "
                         "fraction of the horizon at S times the tolerances (ode_ensemble_plan); "
                         "-1: 0.02 when every system is resident and two or more waves share "
                         "each SIMD, 0: never")
    ap.add_argument("--plan-tol-scale", type=float, default=1000.0, metavar="S",
                    help="the plan's probe runs at S times the tolerances")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--tol", type=float, default=0.0,
                    help="override rtol = atol of the sweep (0: the sweep's own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", dest="served", action="store_false",
                    help="leave the served-mix record out of the default run")
    ap.add_argument("--no-sub-records", dest="sub_records", action="store_false",
                    help="time the headline workload only (by default the Keller-Miksis, "
                         "relief-valve and RK4 Duffing sweeps follow, in sub-records)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--uniform", type=int, default=-1, metavar="SYSTEM",
                    help="give every system the parameters and initial state of SYSTEM, so all "
                         "lanes step in lockstep (FLOP-per-attempt calibration with counters)")
    ap.add_argument("--single", type=int, default=-1, metavar="SYSTEM",
                    help="integrate only system SYSTEM of the sweep, alone (one lane of one "
                         "wave): the time per attempt of its serial chain, which bounds a sweep "
                         "whose end is its slowest system")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the kernel sources and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration)")
    return ap.parse_args()


def copy_calibration(nbytes):
    """A plain device-to-device copy of known size: what HBM byte counters read
    for it scales the integrator's counter readings to bytes."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                      "launches": 3}), flush=True)


def cpu_baseline(pb, target_s, threads=0):
    """The oracle, as it is, on a stratified sample of the same sweep over the
    full horizon, on all host cores (or ``threads``); accepted system-steps/s.
    The sample grows until one run takes at least half of target_s."""
    from oracle import oracle as O
    from paper_1810_03931_amd import inputs as I
    threads = threads or int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    k = min(pb.n, 4 * threads)
    while True:
        sample = pb.subset(I.stratified_sample(pb.n, k, seed=22))
        t0 = time.perf_counter()
        r = O.solve(sample.model, sample.method, sample.time_domain.copy(), sample.state.copy(),
                    sample.params, threads=threads, **sample.options)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or k >= pb.n:
            break
        k = int(min(pb.n, max(2 * k, k * target_s / max(dt, 1e-3))))
    acc = int(r["counts"][0].sum())
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": acc / dt, "unit": "system-steps/s", "cores": threads, "kind": "oracle",
            "cpu": cpu,
            "sample": f"{k} of {pb.n} systems (stratified), full horizon, {acc} accepted steps "
                      f"in {dt:.1f} s"}


# Sources that make up each workload's integrator kernel (besides the common
# ones): counter summaries stay valid while these are unchanged.  (The host
# code that validates arguments and launches the kernel is not among them: it
# does not change what an attempt computes or which bytes a launch moves.)
COMMON_SOURCES = ("integrator.h", "integrator_kernel.h", "model_common.h")
MODEL_SOURCES = {
    "duffing": ("model_duffing.h", "kernels_duffing.hip"),
    "keller_miksis": ("model_keller_miksis.h", "kernels_keller_miksis.hip"),
    "relief_valve": ("model_relief_valve.h", "kernels_relief_valve.hip"),
    "duffing_lyapunov": ("model_duffing.h", "model_duffing_lyapunov.h",
                         "kernels_duffing_lyapunov.hip"),
}


def device_facts(torch, info):
    """Name, compute units and peak clock of the device (the FP64 peak is
    CUs x clock x 128 FLOP/clk)."""
    import ctypes
    clock_khz = 0
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), 5, 0) == 0:   # hipDeviceAttributeClockRate
            clock_khz = v.value
    except OSError:
        pass
    cus = int(info["compute_units"])
    return {"name": torch.cuda.get_device_name(0), "compute_units": cus,
            "peak_clock_mhz": clock_khz / 1e3,
            "fp64_peak_tflops_from_clock": cus * clock_khz * 1e3 * 128 / 1e12 if clock_khz else None}


def kernel_source_hash(workload="duffing_rkck45"):
    """Hash of the sources of one workload's integrator kernel and the build
    flags: counter readings taken for another version of that kernel are not
    reported."""
    import hashlib
    from paper_1810_03931_amd import build
    model = I.CONFIGS[workload]().model if workload in I.CONFIGS else workload
    h = hashlib.sha256()
    for name in COMMON_SOURCES + MODEL_SOURCES[model]:
        with open(os.path.join(build.CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
        extra = getattr(build, "TU_FLAGS", {}).get(name)
        if extra:
            h.update(" ".join(extra).encode())
    h.update(" ".join(build.FLAGS[:-4]).encode())
    return h.hexdigest()[:16]


def calibrated_flops(workload, kind="fp64"):
    """(FLOP per attempt, source) from the committed counter summary of this
    workload's lock-step run, or None.  kind "fp64": FP64 FLOP of the FP64
    kernel at the workload's own tolerance; kind "mixed": FP32 + FP64 FLOP of
    the mixed-precision kernel at tolerance 1e-7."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{kind}_counters.txt")
    if not os.path.exists(path):
        return None
    key = "fp64_flop_per_attempt:" if kind == "fp64" else "flop_per_attempt:"
    block, val, src_hash = None, None, None
    for line in open(path):
        if line.startswith("# kernel sources hash"):
            src_hash = line.split()[-1]
        elif line.startswith("["):
            block = line[1:line.index("]")]
        elif block == "uniform" and line.strip().startswith(key):
            val = float(line.split(":", 1)[1])
    if val is None:
        return None
    note = "counter calibration, uniform lanes" + ("" if kind == "fp64" else
                                                   ", FP32 + FP64 FLOP")
    if src_hash != kernel_source_hash(workload):
        note += " (taken on an earlier build of the kernel sources)"
    return val, note


def measured_traffic(workload):
    """HBM bytes per launch from the committed counter summary of this
    workload, if it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash(workload):
        return None
    return float(vals["bytes_per_launch"])


# Further single-GPU workloads timed in the default run, each in a sub-record of
# the same JSON line: (name, timed steps, warmup steps).
SUB_WORKLOADS = (("keller_miksis", 2, 1), ("relief_valve", 3, 1), ("duffing_rk4", 10, 2))

# The served mix in the default run: the first requests of the seeded mix (three
# models, 256-65536 systems, 64-2048 periods, tolerances 1e-7-1e-6), all
# arriving at once, on the resident server, in FP64 and with FP32 stages.
SERVED_REQUESTS = 40


def served_record(args):
    from paper_1810_03931_amd import inputs as I, serve as S
    reqs = I.served_mix(SERVED_REQUESTS)
    state = {"last": None}

    def progress(done, total, admitted):
        step = (done // 10, admitted // 10)
        if step != state["last"] or done == total:
            state["last"] = step
            print(f"[bench] served mix: {admitted}/{total} admitted, {done}/{total} done",
                  file=sys.stderr, flush=True)

    runs = S.serve_mix(reqs, "resident", ("fp64", "mixed"), (), progress=progress)
    return {"requests": len(reqs), "arrivals": "all at t = 0 (saturation)",
            "models": list(I.SERVED_MODELS), "sizes": [256, 65536], "periods": [64, 2048],
            "tolerance": [1e-7, 1e-6], "server": "resident (continuous admission)",
            "runs": runs}


def bench_workload(torch, E, name, args, steps, warmup):
    """Time ``steps`` full solves of workload ``name`` after ``warmup``
    untimed ones; return the measurements (the JSON record without the CPU
    baseline)."""
    dev = torch.device("cuda", 0)
    pb = I.CONFIGS[name]()
    if args.tol > 0:
        pb = I.with_tolerance(pb, args.tol)
    if args.uniform >= 0:
        pb.params[:] = pb.params[:, args.uniform:args.uniform + 1]
        pb.state[:] = pb.state[:, args.uniform:args.uniform + 1]
        pb.time_domain[:] = pb.time_domain[:, args.uniform:args.uniform + 1]
    ens = E.Ensemble(pb.model, pb.method, precision=args.precision, block_size=args.block_size,
                     blocks_per_cu=args.blocks_per_cu)
    td0 = torch.as_tensor(pb.time_domain, device=dev).contiguous()
    y0 = torch.as_tensor(pb.state, device=dev).contiguous()
    p = torch.as_tensor(pb.params, device=dev).contiguous()
    td, y = td0.clone(), y0.clone()
    ev = pb.options.get("events", [])
    cap = pb.options.get("record_cap", 0) if any(e.get("record_component", -1) >= 0 for e in ev) else 0
    out = ens.outputs(pb.n, n_accessories=len(pb.options.get("accessories", [])),
                      n_events=len(ev), record_cap=cap, device=dev)
    stream = torch.cuda.current_stream(dev)
    tuned = None
    if args.tune:
        tuned = ens.tune(td0, y0, p, probe_fraction=0.25, stream=stream, **pb.options)
        print(f"tuned launch configuration: {tuned}", file=sys.stderr, flush=True)

    segments = getattr(pb, "segments", None)
    snaps = None
    if segments is not None:
        n_seg, seg_len, first = segments
        snaps = torch.empty((n_seg - first, pb.state.shape[0] + 2 * len(pb.options["accessories"]),
                             pb.n), dtype=torch.float64, device=dev)

    def run_segments():
        """The paper's loop of solves, one period each: one recorded graph, or
        (--eager) the same loop of launches from the host."""
        if not args.eager:
            ens.solve_segments(td, y, p, n_seg, seg_len, first_snapshot=first, snapshots=snaps,
                               out=out, stream=stream, **pb.options)
            return
        for k in range(n_seg):
            td[1] = td[0] + seg_len
            ens.solve(td, y, p, out=out, stream=stream, **pb.options)
            if k >= first:
                snaps[k - first, :2].copy_(y)
                snaps[k - first, 2:].copy_(out["acc"])

    plan_frac = 0.0
    plan_ms = []

    def step():
        td.copy_(td0)
        y.copy_(y0)
        index = None
        if plan_frac > 0:
            t_plan = time.perf_counter()
            index = ens.plan(td, y, p, probe_fraction=plan_frac,
                             probe_tolerance_scale=args.plan_tol_scale, stream=stream,
                             **pb.options)
            plan_ms.append((time.perf_counter() - t_plan) * 1e3)
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        if segments is None:
            ens.solve(td, y, p, out=out, system_index=index, stream=stream, **pb.options)
        else:
            run_segments()
        k1.record(stream)
        return k0, k1

    if args.plan > 0:
        plan_frac = args.plan
    elif args.plan < 0 and segments is None and args.uniform < 0 and pb.method == "rkck45":
        # an untimed launch first tells the residency: plan when every system
        # has a lane from the start and two or more waves share each SIMD
        step()
        torch.cuda.synchronize()
        info0 = ens.info()
        waves_per_simd = pb.n / (64.0 * 4 * max(info0["compute_units"], 1))
        if pb.n <= info0["resident_systems"] and waves_per_simd >= 2:
            plan_frac = 0.02
    print(f"[bench] {name}: {warmup} warmup + {steps} timed steps", file=sys.stderr, flush=True)
    for _ in range(warmup):
        step()
        torch.cuda.synchronize()
    plan_ms.clear()
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    kernel_events, wall = [], []
    s0.record(stream)
    for _ in range(steps):
        w0 = time.perf_counter()
        kernel_events.append(step())
        torch.cuda.synchronize()
        wall.append(time.perf_counter() - w0)
    s1.record(stream)
    torch.cuda.synchronize()
    total_ms = s0.elapsed_time(s1)
    kernel_ms = np.array([a.elapsed_time(b) for a, b in kernel_events])

    per_system = out["counts"].sum(dim=0).cpu().numpy()     # attempts of each system
    counts = out["counts"].sum(dim=1).cpu().numpy()        # accepted, rejected, location
    if segments is not None:
        # the counts describe the last segment; RK4 takes the same number of
        # steps in every period
        per_system = per_system * n_seg
        counts = counts * n_seg
    status = np.bincount(out["status"].cpu().numpy() & 0xFF, minlength=6)
    accepted, attempts = int(counts[0]), int(counts.sum())
    ms_per_step = total_ms / steps
    value = accepted / (ms_per_step / 1e3)

    # the repeated-horizon workload runs the RK4 Duffing kernel of duffing_rk4
    cal_name = "duffing_rk4" if pb.name == "duffing_poincare" else pb.name
    if args.precision == "fp64":
        cal = calibrated_flops(cal_name) if args.tol <= 0 else None
    else:
        cal = calibrated_flops(cal_name, "mixed") if args.tol == 1e-7 else None
    flops_attempt, flops_src = cal or (FLOPS_ESTIMATE[(pb.model, pb.method)],
                                       "estimate from the formulas")
    kern_s = float(kernel_ms.mean()) / 1e3
    achieved = attempts * flops_attempt / kern_s / 1e12
    traffic = measured_traffic(pb.name) if (args.uniform < 0 and args.precision == "fp64"
                                            and args.tol <= 0) else None
    info = ens.info()
    rec = {
        "value": value, "unit": "system-steps/s", "steps": steps, "warmup": warmup,
        "ms_per_step": ms_per_step,
        "config": {"workload": pb.name + ("/uniform" if args.uniform >= 0 else ""),
                   "systems": pb.n, "equation": pb.model, "method": pb.method,
                   "horizon": float(pb.time_domain[1, 0]) * (n_seg if segments else 1),
                   "t_record": pb.options.get("t_record"),
                   "rtol": pb.options.get("rtol"), "precision": args.precision,
                   "block_size": info["block_size"], "blocks_per_cu": info["blocks_per_cu"],
                   "resident_systems": info["resident_systems"], "tuned": tuned,
                   "queue_plan": ({"probe_fraction": plan_frac,
                                   "probe_tolerance_scale": args.plan_tol_scale,
                                   "plan_ms": float(np.mean(plan_ms)) if plan_ms else None,
                                   "timed": True} if plan_frac > 0 else None),
                   **({"segments": n_seg, "launch": "host loop" if args.eager else "HIP graph"}
                      if segments is not None else {})},
        "attempted_steps_per_s": attempts / (ms_per_step / 1e3),
        "reject_frac": float(counts[1] / attempts), "location_frac": float(counts[2] / attempts),
        "status_counts": status.tolist(),
        "attempts_per_system": {"p50": float(np.percentile(per_system, 50)),
                                "p99": float(np.percentile(per_system, 99)),
                                "max": int(per_system.max())},
        "p50_ms": float(np.percentile(np.array(wall) * 1e3, 50)),
        "p99_ms": float(np.percentile(np.array(wall) * 1e3, 99)),
        "kernel_ms": float(kernel_ms.mean()),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic,
                     "hbm_gb_s": traffic / kern_s / 1e9 if traffic else None,
                     "hbm_frac_of_8_tb_s": traffic / kern_s / 8e12 if traffic else None,
                     "flops_per_attempt": flops_attempt, "flops_per_attempt_source": flops_src,
                     "attempts_per_launch": attempts},
    }
    return rec, pb, info


def single_system(torch, E, args):
    """One system of the sweep integrated alone; one JSON line."""
    pb = I.CONFIGS[args.config]().subset([args.single])
    if args.tol > 0:
        pb = I.with_tolerance(pb, args.tol)
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(pb.time_domain, device=dev).contiguous()
    y = torch.as_tensor(pb.state, device=dev).contiguous()
    p = torch.as_tensor(pb.params, device=dev).contiguous()
    ens = E.Ensemble(pb.model, pb.method, precision=args.precision)
    stream = torch.cuda.current_stream(dev)
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    out = ens.solve(td, y, p, stream=stream, **pb.options)
    k1.record(stream)
    torch.cuda.synchronize()
    ms = k0.elapsed_time(k1)
    attempts = int(out["counts"].sum())
    print(json.dumps({"workload": pb.name, "system": args.single, "precision": args.precision,
                      "status": int(out["status"][0]), "attempts": attempts, "kernel_ms": ms,
                      "us_per_attempt": ms * 1e3 / attempts}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.source_hash:
        print(kernel_source_hash(args.config))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the systems are independent, so the single-GPU "
              "kernel is what is measured (the design notes describe how it would shard).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1810_03931_amd import ensemble as E

    if not os.path.exists(E.LIB_PATH):
        from paper_1810_03931_amd import build
        build.build()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.single >= 0:
        single_system(torch, E, args)
        return
    rec, pb, info = bench_workload(torch, E, args.config, args, args.steps, args.warmup)
    line = {"metric": METRIC, "value": rec["value"], "unit": rec["unit"], "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if args.precision == "fp64" else "f32 stages / f64 state",
            "data": "synthetic (seeded parameter sweep)"}
    line.update({k: v for k, v in rec.items() if k not in line})
    line["device"] = device_facts(torch, info)
    if args.sub_records and args.config == "duffing_rkck45" and args.uniform < 0:
        subs = {}
        for name, k, w in SUB_WORKLOADS:
            r, _, _ = bench_workload(torch, E, name, args, k, w)
            subs[name] = {key: r[key] for key in ("value", "unit", "steps", "warmup",
                                                  "ms_per_step", "kernel_ms",
                                                  "attempted_steps_per_s", "attempts_per_system",
                                                  "status_counts", "config")}
            subs[name]["roofline"] = {key: r["roofline"][key] for key in (
                "bound", "achieved", "peak", "unit", "frac", "traffic", "flops_per_attempt",
                "flops_per_attempt_source", "attempts_per_launch")}
            torch.cuda.empty_cache()
        line["workloads"] = subs
        if args.served:
            line["served_mix"] = served_record(args)
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pb, args.cpu_seconds)
        line["cpu_baseline_1core"] = cpu_baseline(pb, args.cpu_seconds, threads=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
