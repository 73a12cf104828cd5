"""Serving loop: per-system window starts (what lets requests share a launch)
against the oracle, results bit-identical alone and in the mix, and served
results against the oracle."""
import numpy as np
import pytest

from _parity import compare, reference
from paper_1810_03931_amd import inputs as I

pytestmark = pytest.mark.gpu


def _small_mix(n=18, seed=3):
    return I.served_mix(n, seed=seed, sizes=(64, 1500), periods=(2, 12))


def test_record_start_matches_oracle(ode, oracle):
    import torch
    from paper_1810_03931_amd import ensemble as E
    pb = I.short_horizon(I.duffing_rkck45_sweep()).subset(np.arange(0, 1 << 17, 131))
    pb.time_domain[1] = 3 * I.TWO_PI
    starts = np.linspace(-1.0, 3.5 * I.TWO_PI, pb.n)
    starts[::7] = np.nan                  # NaN: the window never opens
    # the oracle with the same per-system starts
    pb.options["record_start"] = starts
    ref = reference(pb)
    dev = torch.device("cuda", 0)
    tdg = torch.as_tensor(pb.time_domain, device=dev).clone()
    yg = torch.as_tensor(pb.state, device=dev).clone()
    pg = torch.as_tensor(pb.params, device=dev).clone()
    ens = E.Ensemble(pb.model, pb.method)
    opts = dict(pb.options, record_start=torch.as_tensor(starts, device=dev))
    out = ens.solve(tdg, yg, pg, **opts)
    torch.cuda.synchronize()
    g = {"y": yg.cpu().numpy(), "t": tdg[0].cpu().numpy(), "status": out["status"].cpu().numpy(),
         "counts": out["counts"].cpu().numpy(), "acc": np.zeros((0, pb.n)),
         "event_counts": out["event_counts"].cpu().numpy(),
         "event_records": out["event_records"].cpu().numpy()}
    st = compare(g, ref, label="record_start")
    print(f"[serve] per-system window start vs oracle: {st}", flush=True)


def test_results_same_alone_and_in_mix(ode):
    from paper_1810_03931_amd.serve import Server
    for prec in ("fp64", "mixed"):
        reqs = _small_mix()
        alone = Server(precision=prec, slots=1, max_batch_systems=0)
        ref = [alone.run([r])[0] for r in reqs]
        srv = Server(precision=prec, slots=4)
        arr = I.poisson_arrivals(len(reqs), 400.0, seed=1)
        mixed = srv.run(reqs, arr)
        batched = Server(precision=prec, slots=2).run(reqs)      # all at once: batches form
        for a, b, c in zip(ref, mixed, batched):
            for k in a.outputs:
                assert np.array_equal(a.outputs[k], b.outputs[k], equal_nan=True), (prec, a.rid, k)
                assert np.array_equal(a.outputs[k], c.outputs[k], equal_nan=True), (prec, a.rid, k)
        lat = np.array([r.latency for r in mixed])
        print(f"[serve] {prec}: {len(reqs)} requests identical alone, under Poisson arrivals and "
              f"batched; latency p50 {np.median(lat) * 1e3:.1f} ms", flush=True)


def test_served_results_match_oracle(ode, oracle):
    from paper_1810_03931_amd.serve import Server
    reqs = _small_mix(9, seed=4)
    res = Server(precision="fp64", slots=3).run(reqs)
    for req, r in zip(reqs, res):
        pb = req.problem
        ref = reference(pb)
        g = dict(r.outputs)
        g.setdefault("acc", np.zeros((0, pb.n)))
        g.setdefault("event_counts", np.zeros((0, pb.n), dtype=np.int32))
        g["event_records"] = np.zeros((0, 2, pb.n))
        ref.o["event_records"] = np.zeros((0, 2, pb.n))
        # The same bars as the sweeps' parity tests; at the served tolerance
        # (1e-7) a flip's final state must agree within 1e-5 (100 tol), and no
        # system is judged looser than 1e-3.
        st = compare(g, ref, label=pb.name)
        print(f"[serve] {pb.name} n={pb.n} periods={req.periods}: {st}", flush=True)


def test_memory_budget_limits_admission(ode):
    from paper_1810_03931_amd.serve import Server, request_bytes
    reqs = _small_mix(10, seed=5)
    budget = max(request_bytes(r.problem) for r in reqs)
    res = Server(precision="fp64", slots=4, memory_budget=budget).run(reqs)
    # at every admission, the requests in flight fit the budget
    for r in res:
        inflight = sum(request_bytes(q.problem) for q, x in zip(reqs, res)
                       if x.admitted <= r.admitted < x.done)
        assert inflight <= budget
    with pytest.raises(ValueError):
        Server(precision="fp64", memory_budget=budget // 4).run(reqs)


def test_resident_results_same_alone_and_in_mix(ode):
    """Requests admitted into running served launches (one per kernel class,
    each on a share of the device) give bit-identical results to the same
    request solved alone, under Poisson arrivals and when all arrive at once;
    with a pool smaller than the mix, admission waits for slots."""
    from paper_1810_03931_amd.serve import ResidentServer, Server
    for prec in ("fp64", "mixed"):
        reqs = _small_mix()
        alone = Server(precision=prec, slots=1, max_batch_systems=0)
        ref = [alone.run([r])[0] for r in reqs]
        srv = ResidentServer(precision=prec, capacity=4096, max_workgroups=64)
        arr = I.poisson_arrivals(len(reqs), 400.0, seed=1)
        mixed = srv.run(reqs, arr, stall_s=60)
        burst = srv.run(reqs, stall_s=60)            # all at once: slots run out
        for a, b, c in zip(ref, mixed, burst):
            for k in a.outputs:
                assert np.array_equal(a.outputs[k], b.outputs[k], equal_nan=True), (prec, a.rid, k)
                assert np.array_equal(a.outputs[k], c.outputs[k], equal_nan=True), (prec, a.rid, k)
        st = srv.stats()
        assert st["launches"] >= 3
        # every class launches and copies on its queue's own streams
        handles = [h for c in srv.classes.values() for h in (c.stream.cuda_stream, c.copy.cuda_stream)]
        assert len(set(handles)) == len(handles) == 2 * len(srv.classes)
        lat = np.array([r.latency for r in mixed])
        print(f"[serve] resident {prec}: {len(reqs)} requests identical alone, under Poisson "
              f"arrivals and in a burst; {st}; latency p50 {np.median(lat) * 1e3:.1f} ms",
              flush=True)
        srv.shutdown()


def test_work_published_beside_a_long_chain_starts_on_every_lane(ode):
    """A served launch keeps all its waves while any of its work is in flight,
    so a large request that arrives while one wave integrates a long
    single-system request starts on every idle lane and finishes first.  (Were
    the idle waves to leave, it would run on the 63 idle lanes of that one
    wave: about 4e6 attempts per lane, several times the long request.)"""
    from paper_1810_03931_amd.serve import ResidentServer
    km = I.CONFIGS["keller_miksis"]()
    # about 1.1e6 attempts in one serial chain, against at most 2e5 for any bulk system
    long = I.Request(0, km.subset([141]).with_horizon(32.0, t_record=0.0), 32)
    bulk_pb = km.subset(I.stratified_sample(km.n, 16384, seed=5)).with_horizon(8.0, t_record=0.0)
    bulk = I.Request(1, bulk_pb, 8)
    srv = ResidentServer(precision="fp64", capacity=1 << 15, max_workgroups=64)
    try:
        a, b = srv.run([long, bulk], np.array([0.0, 0.3]), stall_s=120)
    finally:
        srv.shutdown()
    print(f"[serve] long chain done at {a.done:.2f} s; bulk request of {bulk_pb.n} systems "
          f"(arrived at 0.3 s) done at {b.done:.2f} s", flush=True)
    assert b.done < a.done
