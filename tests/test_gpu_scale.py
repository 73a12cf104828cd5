"""Large launches: many more systems than resident lanes (every lane refills
from the work queue many times), and a large leading dimension addressed
through a sparse gather list.  Checked on a stratified sample against the
oracle, and against the same systems solved alone on the GPU (bitwise)."""
import numpy as np
import pytest

from _parity import compare, reference, run_gpu, take
from paper_1810_03931_amd import inputs as I

pytestmark = pytest.mark.gpu


def _tiled_duffing(n):
    """The Duffing sweep's 2^17 systems repeated to n systems, short horizon,
    few event records."""
    base = I.short_horizon(I.duffing_rkck45_sweep())
    idx = np.arange(n) % base.n
    pb = base.subset(idx)
    pb.options["record_cap"] = 4
    return pb


def test_many_more_systems_than_resident_lanes(ode, oracle):
    pb = _tiled_duffing(1 << 21)                   # 16x the resident lanes
    g = run_gpu(pb)
    assert np.all(g["status"] == 0)
    # a system's results do not depend on when or where it ran: copies of
    # one system agree bit for bit across the 16 tiles
    base_n = 1 << 17
    for k in (1, 7, 15):
        sl = slice(k * base_n, (k + 1) * base_n)
        for key in ("y", "t", "counts", "event_counts", "event_records"):
            a, b = g[key][..., :base_n], g[key][..., sl]
            assert np.array_equal(a, b, equal_nan=True), (k, key)
    sample = I.stratified_sample(pb.n, 1536, seed=31)
    st = compare(take(g, sample), reference(pb.subset(sample)), label="2^21 systems")
    print(f"[scale] 2^21 systems: {st}", flush=True)


def test_large_leading_dimension_sparse_gather(ode, oracle):
    import torch
    from paper_1810_03931_amd import ensemble as E
    ld = 1 << 22
    rng = np.random.default_rng(33)
    chosen = np.sort(rng.choice(ld, 50000, replace=False))
    base = I.short_horizon(I.relief_valve_sweep())
    src = rng.integers(0, base.n, ld)               # every column holds some valve system
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(base.time_domain[:, src], device=dev).contiguous()
    y = torch.as_tensor(base.state[:, src], device=dev).contiguous()
    p = torch.as_tensor(base.params[:, src], device=dev).contiguous()
    y_before = y.clone()
    ens = E.Ensemble(base.model, base.method)
    out = ens.solve(td, y, p, system_index=torch.as_tensor(chosen, device=dev), **base.options)
    torch.cuda.synchronize()
    status = out["status"].cpu().numpy()
    assert np.all(status[chosen] == 0)
    untouched = np.ones(ld, dtype=bool)
    untouched[chosen] = False
    assert np.all(status[untouched] == -1)
    assert torch.equal(y[:, torch.as_tensor(untouched, device=dev)],
                       y_before[:, torch.as_tensor(untouched, device=dev)])
    pick = chosen[I.stratified_sample(len(chosen), 1024, seed=34)]
    sub = base.subset(src[pick])
    ref = reference(sub)
    g = {"y": y[:, torch.as_tensor(pick, device=dev)].cpu().numpy(),
         "t": td[0, torch.as_tensor(pick, device=dev)].cpu().numpy(),
         "status": status[pick], "counts": out["counts"].cpu().numpy()[:, pick],
         "acc": out["acc"].cpu().numpy()[:, pick],
         "event_counts": out["event_counts"].cpu().numpy()[:, pick],
         "event_records": np.zeros((0, 2, len(pick)))}
    st = compare(g, ref, label="ld 2^22 gather")
    print(f"[scale] ld=2^22, 50000 gathered systems: {st}", flush=True)
