"""Planned queue order on the GPU: the probe-based plan changes which lane
runs each system, never its result."""
import numpy as np
import pytest
import torch

from paper_1810_03931_amd import ensemble as E
from paper_1810_03931_amd import inputs as I

pytestmark = pytest.mark.gpu


def _solve(ens, pb, index=None):
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(pb.time_domain, device=dev).clone()
    y = torch.as_tensor(pb.state, device=dev).clone()
    p = torch.as_tensor(pb.params, device=dev)
    out = ens.solve(td, y, p, system_index=index, **pb.options)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    r["t"], r["y"] = td[0].cpu().numpy(), y.cpu().numpy()
    return r


def _plan(ens, pb, frac):
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(pb.time_domain, device=dev)
    y = torch.as_tensor(pb.state, device=dev)
    p = torch.as_tensor(pb.params, device=dev)
    before = (td.clone(), y.clone())
    index = ens.plan(td, y, p, probe_fraction=frac, **pb.options)
    torch.cuda.synchronize()
    assert torch.equal(td, before[0]) and torch.equal(y, before[1])   # inputs only read
    return index


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("n", [131072, 100000])
def test_resident_plan_is_bitwise_neutral(n):
    pb = I.duffing_rkck45_sweep().subset(np.arange(n)).with_horizon(24 * I.TWO_PI, t_record=16 * I.TWO_PI)
    ens = E.Ensemble(pb.model, pb.method)
    plain = _solve(ens, pb)
    info = ens.info()
    index = _plan(ens, pb, 0.1)
    idx = index.cpu().numpy()
    bs = info["block_size"]
    assert n <= info["resident_systems"]
    assert idx.size == 64 * (-(-n // bs)) * (bs // 64)
    assert np.array_equal(np.sort(idx[idx >= 0]), np.arange(n))
    print(f"[plan] n={n} positions={idx.size} holes={np.sum(idx < 0)}", flush=True)
    _same(plain, _solve(ens, pb, index))


def test_queue_plan_with_caller_index_is_bitwise_neutral():
    # more systems than lanes (one workgroup per CU): longest chunks first
    pb = I.relief_valve_sweep().with_horizon(2.0, t_record=1.0)
    ens = E.Ensemble(pb.model, pb.method, blocks_per_cu=1)
    rng = np.random.default_rng(5)
    sub = rng.permutation(pb.n)[:pb.n - 3000]
    dev = torch.device("cuda", 0)
    caller = torch.as_tensor(sub.astype(np.int64), device=dev)
    td = torch.as_tensor(pb.time_domain, device=dev)
    y = torch.as_tensor(pb.state, device=dev)
    p = torch.as_tensor(pb.params, device=dev)
    index = ens.plan(td, y, p, probe_fraction=0.2, system_index=caller, **pb.options)
    idx = index.cpu().numpy()
    assert idx.size == sub.size and np.array_equal(np.sort(idx), np.sort(sub))
    a = _solve(ens, pb, caller)
    b = _solve(ens, pb, index)
    for k in a:
        assert np.array_equal(a[k][..., sub], b[k][..., sub], equal_nan=True), k


def test_plan_rejects_bad_probe_arguments():
    pb = I.duffing_rkck45_sweep().subset(np.arange(4096)).with_horizon(2 * I.TWO_PI, t_record=0.0)
    ens = E.Ensemble(pb.model, pb.method)
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(pb.time_domain, device=dev)
    y = torch.as_tensor(pb.state, device=dev)
    p = torch.as_tensor(pb.params, device=dev)
    for kw in (dict(probe_fraction=0.0), dict(probe_fraction=1.5),
               dict(probe_tolerance_scale=0.5), dict(probe_tolerance_scale=float("inf"))):
        with pytest.raises(E.OdeError):
            ens.plan(td, y, p, **kw, **pb.options)
