"""Autotuner (ode_ensemble_tune): it only reads the caller's arrays, picks a
configuration among its candidates, and a tuned handle gives bit-identical
results (each system's arithmetic does not depend on the launch shape)."""
import numpy as np
import pytest

from _parity import run_gpu
from paper_1810_03931_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["duffing_rkck45", "relief_valve"])
def test_tune_reads_only_and_keeps_results(ode, name):
    import torch
    from paper_1810_03931_amd import ensemble as E
    pb = I.short_horizon(I.CONFIGS[name]())
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(pb.time_domain, device=dev).clone()
    y = torch.as_tensor(pb.state, device=dev).clone()
    p = torch.as_tensor(pb.params, device=dev).clone()
    ens = E.Ensemble(pb.model, pb.method)
    r = ens.tune(td, y, p, probe_fraction=0.5, **pb.options)
    torch.cuda.synchronize()
    print(f"[tune] {name}: {r}", flush=True)
    assert torch.equal(td.cpu(), torch.as_tensor(pb.time_domain))
    assert torch.equal(y.cpu(), torch.as_tensor(pb.state))
    assert r["block_size"] in (64, 128, 256) and r["candidates"] >= 5
    assert 0 < r["best_ms"] <= r["default_ms"]
    info = ens.info()
    assert info["block_size"] == r["block_size"]
    tuned = run_gpu(pb, ens=ens)
    plain = run_gpu(pb)
    for k in ("status", "counts", "y", "t", "acc", "event_counts", "event_records"):
        assert np.array_equal(tuned[k], plain[k], equal_nan=True), k


def test_tune_with_gather_list_reads_only(ode):
    import torch
    from paper_1810_03931_amd import ensemble as E
    pb = I.short_horizon(I.duffing_rkck45_sweep())
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(pb.time_domain, device=dev).clone()
    y = torch.as_tensor(pb.state, device=dev).clone()
    p = torch.as_tensor(pb.params, device=dev).clone()
    idx = torch.arange(0, pb.n, 5, dtype=torch.int64, device=dev)
    ens = E.Ensemble(pb.model, pb.method)
    r = ens.tune(td, y, p, probe_fraction=0.25, system_index=idx, **pb.options)
    torch.cuda.synchronize()
    assert torch.equal(td.cpu(), torch.as_tensor(pb.time_domain))
    assert torch.equal(y.cpu(), torch.as_tensor(pb.state))
    assert r["candidates"] >= 5 and r["best_ms"] <= r["default_ms"]
