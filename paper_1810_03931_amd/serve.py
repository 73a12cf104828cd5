"""Serving loop: continuous admission of parameter-sweep requests.

Requests (``inputs.Request``: a sweep of systems with its model, method,
horizon and options) arrive at given times.  The loop admits a waiting
request as soon as a slot is free and the device-memory budget has room for
its arrays.  A slot is a HIP stream with its own solver handles, so one
handle never runs two solves at once.  On admission the loop copies the
request's inputs to the device on the slot's stream and enqueues its solve.
It polls completion events, copies the results back, releases the memory and
admits the next requests.

Waiting requests that can share a launch (same model, method, events and
accessories; horizons within a factor of two) are batched into one solve:
their systems sit side by side, each with its own window start
(``record_start``) and its own tolerances (``tolerances``), so requests with
different windows and tolerances run in one persistent kernel.
Launches on different slots run concurrently.  When one launch's workgroups
retire, the freed compute units take workgroups of the others, so requests
arriving while others run start right away, up to the slot and memory
limits.  No system's arithmetic depends on its neighbours or on the launch
shape, so a result is bit-identical alone and in the mix.

Latency is measured from arrival to the results being on the host, p50/p99
over the requests.  Throughput is the accepted steps of all requests divided
by the time from the first arrival to the last completion.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time
from collections import deque
from typing import Optional

import numpy as np

from . import ensemble as E
from . import inputs as I


def request_bytes(pb: I.Problem) -> int:
    """Device bytes a request holds while resident."""
    n = pb.n
    n_acc = len(pb.options.get("accessories", ()))
    evs = pb.options.get("events", ())
    cap = pb.options.get("record_cap", 0) if any(e.get("record_component", -1) >= 0
                                                 for e in evs) else 0
    ns = pb.state.shape[0]
    rows = 2 + ns + pb.params.shape[0] + 2 * n_acc + 2 * cap + 1 + 2 * ns
    return n * (8 * rows + 4 + 3 * 8 + 4 * len(evs))


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    steps: int
    outputs: dict

    @property
    def latency(self) -> float:
        return self.done - self.arrival


# Options that become per-system arrays of a batched launch.
PER_SYSTEM = ("t_record", "rtol", "atol")


def _batch_key(pb: I.Problem) -> str:
    """Requests with equal keys can share one launch: same model, method and
    options except the window start and the tolerances, which become per
    system."""
    opts = {k: v for k, v in pb.options.items() if k not in PER_SYSTEM}
    return json.dumps([pb.model, pb.method, opts], sort_keys=True, default=str)


def _tolerances(pb: I.Problem) -> np.ndarray:
    """[2*n_state, n] relative then absolute tolerance of every system."""
    ns = pb.state.shape[0]
    rt = np.broadcast_to(np.asarray(pb.options.get("rtol", 1e-10), dtype=np.float64), (ns,))
    at = np.broadcast_to(np.asarray(pb.options.get("atol", 1e-10), dtype=np.float64), (ns,))
    return np.repeat(np.concatenate([rt, at])[:, None], pb.n, axis=1)


class _Slot:
    def __init__(self, torch, device, precision, block_size):
        self.torch = torch
        self.stream = E.dedicated_stream(device)   # never waits behind another slot's launch
        self.device = device
        self.precision = precision
        self.block_size = block_size
        self.handles = {}
        self.busy = None

    def handle(self, model, method):
        key = (model, method)
        if key not in self.handles:
            self.handles[key] = E.Ensemble(model, method, precision=self.precision,
                                           block_size=self.block_size)
        return self.handles[key]

    def launch(self, batch: list, nbytes: int, now: float):
        """One solve for the requests of ``batch`` [(request, arrival)], their
        systems side by side, each system with its request's window start."""
        torch = self.torch
        pbs = [req.problem for req, _ in batch]
        first = pbs[0]
        cat = lambda f: np.ascontiguousarray(np.concatenate([f(pb) for pb in pbs], axis=-1))
        td = cat(lambda pb: pb.time_domain)
        y = cat(lambda pb: pb.state)
        p = cat(lambda pb: pb.params)
        rec = cat(lambda pb: np.full(pb.n, pb.options.get("t_record", -np.inf)))
        tol = cat(_tolerances)
        opts = {k: v for k, v in first.options.items() if k not in PER_SYSTEM}
        with torch.cuda.stream(self.stream):
            hosts = [torch.from_numpy(a).pin_memory() for a in (td, y, p, rec, tol)]
            dev = [h.to(self.device, non_blocking=True) for h in hosts]
            ens = self.handle(first.model, first.method)
            per_system = {"record_start": dev[3]}
            if first.method == "rkck45":
                per_system["tolerances"] = dev[4]
            out = ens.solve(dev[0], dev[1], dev[2], stream=self.stream, **per_system, **opts)
            res = {"t": dev[0][0], "y": dev[1], "status": out["status"], "counts": out["counts"]}
            if out.get("acc") is not None:
                res["acc"] = out["acc"]
            if out.get("event_counts") is not None:
                res["event_counts"] = out["event_counts"]
            host = {k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True)
                    for k, v in res.items()}
            for k, v in res.items():
                host[k].copy_(v, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.busy = (batch, now, nbytes, (hosts, dev, out, res), host, ev)


class Server:
    """Admits requests into ``slots`` concurrent streams within a device
    memory budget of ``memory_budget`` bytes; waiting requests that can
    share a launch are batched (up to ``max_batch_systems`` systems, horizons
    within ``horizon_ratio`` of the oldest waiting request's)."""

    def __init__(self, *, precision: str = "fp64", slots: int = 4,
                 memory_budget: int = 8 << 30, block_size: int = 0, device: int = 0,
                 max_batch_systems: int = 1 << 17, horizon_ratio: float = 2.0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.budget = int(memory_budget)
        self.max_batch = int(max_batch_systems)
        self.ratio = float(horizon_ratio)
        self.slots = [_Slot(torch, self.device, precision, block_size) for _ in range(slots)]

    def _take_batch(self, waiting: deque, free_bytes: int):
        """The oldest waiting request and the later ones that can join it."""
        span = lambda r: float(np.max(r.problem.time_domain[1] - r.problem.time_domain[0]))
        head, arr = waiting.popleft()
        key, h0 = _batch_key(head.problem), span(head)
        batch = [(head, arr)]
        size, nbytes = head.problem.n, request_bytes(head.problem)
        keep = deque()
        while waiting:
            req, arr = waiting.popleft()
            b = request_bytes(req.problem)
            if (_batch_key(req.problem) == key and h0 / self.ratio <= span(req) <= h0 * self.ratio
                    and size + req.problem.n <= self.max_batch and nbytes + b <= free_bytes):
                batch.append((req, arr))
                size += req.problem.n
                nbytes += b
            else:
                keep.append((req, arr))
        waiting.extend(keep)
        return batch, nbytes

    def run(self, requests: list, arrivals: Optional[np.ndarray] = None,
            poll_s: float = 5e-5) -> list:
        """Serve ``requests`` arriving at ``arrivals`` (seconds from the start;
        None: all at once).  Returns one Result per request, in request
        order."""
        if arrivals is None:
            arrivals = np.zeros(len(requests))
        order = np.argsort(arrivals, kind="stable")
        for r in requests:
            if request_bytes(r.problem) > self.budget:
                raise ValueError(f"request {r.rid} needs more than the memory budget")
        waiting = deque()
        future = deque((requests[i], float(arrivals[i])) for i in order)
        results = {}
        used = 0
        t0 = time.perf_counter()
        while future or waiting or any(s.busy for s in self.slots):
            now = time.perf_counter() - t0
            while future and future[0][1] <= now:
                waiting.append(future.popleft())
            # retire finished launches
            for s in self.slots:
                if s.busy and s.busy[-1].query():
                    batch, adm, nbytes, _dev, host, _ev = s.busy
                    done = time.perf_counter() - t0
                    out = {k: v.numpy() for k, v in host.items()}
                    lo = 0
                    for req, arr in batch:
                        hi = lo + req.problem.n
                        part = {k: v[..., lo:hi] for k, v in out.items()}
                        results[req.rid] = Result(req.rid, arr, adm, done,
                                                  int(part["counts"][0].sum()), part)
                        lo = hi
                    used -= nbytes
                    s.busy = None
            # admit, oldest first, while a slot and memory are free
            while waiting:
                slot = next((s for s in self.slots if not s.busy), None)
                if slot is None or used + request_bytes(waiting[0][0].problem) > self.budget:
                    break
                batch, nbytes = self._take_batch(waiting, self.budget - used)
                used += nbytes
                slot.launch(batch, nbytes, time.perf_counter() - t0)
            if not waiting and future and not any(s.busy for s in self.slots):
                time.sleep(max(0.0, min(future[0][1] - now, 1e-3)))
            else:
                time.sleep(poll_s)
        return [results[r.rid] for r in requests]


class _Resident:
    """The served launch of one kernel class (model, method, events and
    accessories): a pool of ``capacity`` slots on the device, its position
    ring and a served queue.  Requests are copied into free slots and
    published while the launch runs, and their systems start on the lanes
    that free up; a request's slots are released once its results are back.
    Event records are not part of a served result, so the pool keeps none."""

    def __init__(self, torch, device, first: I.Problem, *, capacity: int, precision: str,
                 block_size: int, max_workgroups: int, idle_polls: int, max_requests: int):
        self.torch = torch
        self.model, self.method = first.model, first.method
        opts = {k: v for k, v in first.options.items() if k not in PER_SYSTEM}
        opts["events"] = [dict(e, record_component=-1) for e in opts.get("events", [])]
        opts["record_cap"] = 0
        self.options = opts
        ns, npar = first.state.shape[0], first.params.shape[0]
        self.cap = C = int(capacity)
        f64 = torch.float64
        self.td = torch.zeros((2, C), dtype=f64, device=device)
        self.y = torch.zeros((ns, C), dtype=f64, device=device)
        self.p = torch.zeros((npar, C), dtype=f64, device=device)
        self.rec = torch.zeros(C, dtype=f64, device=device)
        self.tol = torch.ones((2 * ns, C), dtype=f64, device=device)
        self.ring = torch.zeros(C, dtype=torch.int64, device=device)
        self.req_of = torch.zeros(C, dtype=torch.int32, device=device)
        self.ens = E.Ensemble(self.model, self.method, precision=precision, block_size=block_size)
        self.out = self.ens.outputs(C, n_accessories=len(opts.get("accessories", [])),
                                    n_events=len(opts["events"]), device=device)
        self.queue = E.ServedQueue(max_requests)
        # the queue's own streams: a class's copies and relaunches never wait
        # behind another class's running launch
        self.stream, self.copy = self.queue.streams(device)
        self.max_requests = int(max_requests)
        self.max_workgroups = int(max_workgroups)
        self.idle_polls = int(idle_polls)
        self.launches = 0
        self.reset()

    def reset(self):
        """A new session (no launch may be running)."""
        self.queue.reset(self.copy)
        self.free = [(0, self.cap)]        # free slot ranges (start, length), sorted
        self.ids = list(range(self.max_requests - 1, -1, -1))
        self.published = 0
        self.launched = None               # completion event of the latest launch
        self.inflight = {}                 # request id -> (request, arrival, admitted, start)

    def _alloc(self, m: int):
        for i, (a, length) in enumerate(self.free):
            if length >= m:
                self.free[i:i + 1] = [] if length == m else [(a + m, length - m)]
                return a
        return None

    def _release(self, a: int, m: int):
        merged = []
        for s, length in sorted(self.free + [(a, m)]):
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + length)
            else:
                merged.append((s, length))
        self.free = merged

    def admit(self, req, arrival: float, now: float) -> bool:
        """Copy a request into free slots and publish its systems; False when
        no slot range or request id is free."""
        pb = req.problem
        m = pb.n
        if not self.ids or m > self.cap:
            return False
        a = self._alloc(m)
        if a is None:
            return False
        rid = self.ids.pop()
        torch = self.torch
        pin = lambda x: torch.from_numpy(np.ascontiguousarray(x)).pin_memory()
        host = [(self.td, pin(pb.time_domain)), (self.y, pin(pb.state)), (self.p, pin(pb.params)),
                (self.rec, pin(np.full(m, pb.options.get("t_record", -np.inf)))),
                (self.req_of, pin(np.full(m, rid, dtype=np.int32)))]
        if self.method == "rkck45":
            host.append((self.tol, pin(_tolerances(pb))))
        for dst, src in host:
            E.copy_columns(dst, a, src, 0, m, self.copy)
        # ring entries of queue positions P .. P+m-1 (wrapping at the pool size)
        P, C = self.published, self.cap
        slots = pin(a + np.arange(m, dtype=np.int64))
        first = min(m, C - P % C)
        E.copy_columns(self.ring, P % C, slots, 0, first, self.copy)
        if first < m:
            E.copy_columns(self.ring, 0, slots, first, m - first, self.copy)
        self.queue.begin_request(rid, m, self.copy)    # waits for the copies above
        self.published += m
        self.queue.publish(self.published, self.copy)
        self.inflight[rid] = (req, arrival, now, a)
        self.ensure_running()
        return True

    def ensure_running(self):
        """Launch again when requests are in flight and the latest launch has
        left (its waves leave after idle_polls empty polls)."""
        if not self.inflight or (self.launched is not None and not self.launched.query()):
            return
        opts = dict(self.options, record_start=self.rec)
        if self.method == "rkck45":
            opts["tolerances"] = self.tol
        self.queue.launch(self.ens, self.td, self.y, self.p, self.ring, self.req_of, out=self.out,
                          max_workgroups=self.max_workgroups, idle_polls=self.idle_polls,
                          stream=self.stream, **opts)
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self.launched = ev
        self.launches += 1

    def collect(self, t0: float) -> list:
        """Results of the requests whose done flag is set; their slots and
        request ids are released."""
        torch = self.torch
        results = []
        for rid in [r for r in self.inflight if self.queue.done[r] == 1]:
            req, arrival, admitted, a = self.inflight.pop(rid)
            m = req.problem.n
            dev = {"t": self.td[0], "y": self.y, "status": self.out["status"],
                   "counts": self.out["counts"]}
            for k in ("acc", "event_counts"):
                if self.out.get(k) is not None:
                    dev[k] = self.out[k]
            host = {}
            for k, v in dev.items():
                h = torch.empty(tuple(v.shape[:-1]) + (m,), dtype=v.dtype, pin_memory=True)
                E.copy_columns(h, 0, v, a, m, self.copy)
                host[k] = h
            self.copy.synchronize()
            done = time.perf_counter() - t0
            part = {k: v.numpy().copy() for k, v in host.items()}
            self._release(a, m)
            self.ids.append(rid)
            results.append(Result(req.rid, arrival, admitted, done, int(part["counts"][0].sum()),
                                  part))
        self.ensure_running()
        return results

    def close(self):
        """Close the queue and wait for the launch to leave."""
        self.queue.close_queue(self.copy)
        self.stream.synchronize()


class ResidentServer:
    """Continuous batching inside running launches: one served launch per
    kernel class (model, method, events, accessories), each on at most
    ``max_workgroups`` workgroups so the classes share the device, each with a
    pool of ``capacity`` slots (the device-memory budget of its class).  A
    request is admitted as soon as its class has a free slot range: its
    systems are copied in and published, and the running launch's lanes take
    them as they free up.  Arrival order is kept within a class; a request
    that does not fit does not hold back the other classes."""

    def __init__(self, *, precision: str = "fp64", capacity: int = 1 << 21,
                 max_workgroups: int = 128, idle_polls: int = 2000, block_size: int = 0,
                 device: int = 0, max_requests: int = 4096):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.kw = dict(capacity=capacity, precision=precision, block_size=block_size,
                       max_workgroups=max_workgroups, idle_polls=idle_polls,
                       max_requests=max_requests)
        self.classes = {}

    def _class(self, pb: I.Problem) -> _Resident:
        key = _batch_key(pb)
        if key not in self.classes:
            self.classes[key] = _Resident(self.torch, self.device, pb, **self.kw)
        return self.classes[key]

    def run(self, requests: list, arrivals: Optional[np.ndarray] = None,
            poll_s: float = 5e-5, stall_s: float = 600.0, progress=None) -> list:
        """Serve ``requests`` arriving at ``arrivals`` (seconds from the start;
        None: all at once); one Result per request, in request order.  Raises
        if no request completes for ``stall_s`` seconds while some are in
        flight.  ``progress(done, total, admitted)`` is called after every
        admission and every completed request."""
        if arrivals is None:
            arrivals = np.zeros(len(requests))
        for r in requests:
            if r.problem.n > self.kw["capacity"]:
                raise ValueError(f"request {r.rid} has more systems than a pool holds")
        order = np.argsort(arrivals, kind="stable")
        future = deque((requests[i], float(arrivals[i])) for i in order)
        waiting = deque()
        for c in self.classes.values():
            c.reset()
        results = {}
        t0 = time.perf_counter()
        last = t0
        admitted = 0
        while future or waiting or any(c.inflight for c in self.classes.values()):
            now = time.perf_counter() - t0
            while future and future[0][1] <= now:
                waiting.append(future.popleft())
            for c in list(self.classes.values()):
                for r in c.collect(t0):
                    results[r.rid] = r
                    last = time.perf_counter()
                    if progress:
                        progress(len(results), len(requests), admitted)
            if any(c.inflight for c in self.classes.values()) and \
                    time.perf_counter() - last > stall_s:
                for c in self.classes.values():
                    c.close()
                raise RuntimeError(f"served queues: no request finished in {stall_s} s")
            blocked = set()
            keep = deque()
            while waiting:
                req, arr = waiting.popleft()
                c = self._class(req.problem)
                if id(c) in blocked or not c.admit(req, arr, time.perf_counter() - t0):
                    blocked.add(id(c))
                    keep.append((req, arr))
                else:
                    admitted += 1
                    if progress:
                        progress(len(results), len(requests), admitted)
            waiting = keep
            if not waiting and future and not any(c.inflight for c in self.classes.values()):
                time.sleep(max(0.0, min(future[0][1] - now, 1e-3)))
            else:
                time.sleep(poll_s)
        for c in self.classes.values():
            c.close()
        return [results[r.rid] for r in requests]

    def stats(self) -> dict:
        return {"classes": len(self.classes),
                "launches": sum(c.launches for c in self.classes.values())}

    def shutdown(self):
        for c in self.classes.values():
            c.close()
            c.queue.destroy()
        self.classes = {}


def summarize(results: list, label: str) -> dict:
    lat = np.array([r.latency for r in results])
    span = max(r.done for r in results) - min(r.arrival for r in results)
    steps = sum(r.steps for r in results)
    return {"mode": label, "requests": len(results),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "system_steps_per_s": steps / span, "span_s": span, "accepted_steps": steps}


def make_server(mode: str, precision: str, *, slots: int = 4, capacity: int = 1 << 21,
                max_workgroups: int = 128):
    """A server of either kind: "resident" (requests admitted into running
    served launches, one per kernel class) or "launch" (one launch per batch
    of requests on ``slots`` streams)."""
    if mode == "resident":
        return ResidentServer(precision=precision, capacity=capacity,
                              max_workgroups=max_workgroups)
    return Server(precision=precision, slots=slots)


def serve_mix(reqs: list, mode: str, precisions, loads, *, slots: int = 4,
              capacity: int = 1 << 21, max_workgroups: int = 128, log=None,
              progress=None) -> list:
    """Saturation (every request at t = 0) and Poisson loads at fractions of
    the measured saturation rate, per precision; one summary per run.
    ``progress(done, total, admitted)`` reports admissions and completions
    (resident mode)."""
    lines = []
    kw = {"progress": progress} if (progress and mode == "resident") else {}
    for prec in precisions:
        srv = make_server(mode, prec, slots=slots, capacity=capacity,
                          max_workgroups=max_workgroups)
        srv.run(reqs[: min(8, len(reqs))])                     # warm up handles and kernels
        sat = summarize(srv.run(reqs, **kw), f"{prec}/saturation")   # all requests at once
        sat_qps = len(reqs) / sat["span_s"]
        sat["qps"] = sat_qps
        lines.append(sat)
        if log:
            log(sat)
        for load in loads:
            arr = I.poisson_arrivals(len(reqs), load * sat_qps)
            st = summarize(srv.run(reqs, arr, **kw), f"{prec}/load{load}")
            st["qps"] = load * sat_qps
            lines.append(st)
            if log:
                log(st)
        if mode == "resident":
            srv.shutdown()
    return lines


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="served mix: Poisson arrivals of sweep requests")
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--tol", type=float, nargs=2, default=[1e-7, 1e-6], metavar=("LO", "HI"),
                    help="per-request tolerance, log-uniform over [LO, HI]")
    ap.add_argument("--mode", choices=["resident", "launch"], default="resident",
                    help="resident: requests join running served launches; launch: one launch "
                         "per batch on --slots streams")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--capacity", type=int, default=1 << 21,
                    help="resident mode: slots of each kernel class's pool")
    ap.add_argument("--max-workgroups", type=int, default=128,
                    help="resident mode: workgroups of each class's served launch")
    ap.add_argument("--load", type=float, nargs="+", default=[0.5, 0.8],
                    help="offered load as fractions of the measured saturation rate")
    ap.add_argument("--precision", nargs="+", default=["fp64", "mixed"])
    ap.add_argument("--periods", type=int, nargs=2, default=[64, 2048], metavar=("LO", "HI"),
                    help="per-request horizon in forcing periods, log-uniform over [LO, HI]")
    args = ap.parse_args(argv)
    reqs = I.served_mix(args.requests, tol=tuple(args.tol), periods=tuple(args.periods))
    print(json.dumps({"served_mix": {"requests": len(reqs), "tolerance": args.tol,
                                     "periods": args.periods, "sizes": [256, 65536],
                                     "models": list(I.SERVED_MODELS), "mode": args.mode,
                                     "slots": args.slots, "capacity": args.capacity,
                                     "max_workgroups": args.max_workgroups}}), flush=True)
    state = {"last": (-1, -1)}

    def progress(done, total, admitted):
        step = (done // 10, admitted // 10)
        if step != state["last"] or done == total:
            state["last"] = step
            print(f"[serve] {admitted}/{total} admitted, {done}/{total} done", file=sys.stderr,
                  flush=True)

    serve_mix(reqs, args.mode, args.precision, args.load, slots=args.slots,
              capacity=args.capacity, max_workgroups=args.max_workgroups,
              log=lambda st: print(json.dumps(st), flush=True), progress=progress)
    return 0


if __name__ == "__main__":
    sys.exit(main())
