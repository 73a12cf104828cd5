"""Repeated horizons recorded as one HIP graph (ode_ensemble_solve_segments).

The paper's Sec. 7 workflow advances a sweep one excitation period per solve
call, each end point starting the next call, and keeps the points of the last
calls (Poincare sections, per-period maxima).  The graph must give exactly
what the host loop of solve calls gives; and the host loop must match the
oracle doing the same loop on the CPU.
"""
import numpy as np
import pytest

from _parity import short_twins

from paper_1810_03931_amd import inputs as I

pytestmark = pytest.mark.gpu

T = I.TWO_PI


def _duffing1(n):
    """Double-well Duffing, B = 0.3, k uniform in [0.2, 0.3], RK4 with the
    paper's fixed step 1e-2, max of y1 per period (paper Sec. 7.1)."""
    i = np.arange(n, dtype=np.float64)
    k = 0.2 + 0.1 * i / max(n - 1, 1)
    params = np.stack([k, np.full(n, 0.3), np.ones(n), np.full(n, -1.0), np.ones(n)])
    g = np.random.default_rng(7)
    state = g.uniform(-1e-3, 1e-3, size=(2, n))
    td = np.stack([np.zeros(n), np.full(n, T)])
    opts = dict(h0=1e-2, accessories=[("max", 0)], max_steps=10**6)
    return I.Problem("duffing1", "duffing", "rk4", td, state, params, opts)


def _device(pb):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.as_tensor(pb.time_domain, device=dev).clone(),
            torch.as_tensor(pb.state, device=dev).clone(),
            torch.as_tensor(pb.params, device=dev).clone())


def _eager(ens, pb, n_seg, first):
    import torch
    td, y, p = _device(pb)
    snaps = []
    for k in range(n_seg):
        td[1] = td[0] + T
        out = ens.solve(td, y, p, **pb.options)
        if k >= first:
            snaps.append(torch.cat([y, out["acc"]]).clone())
    torch.cuda.synchronize()
    return td.cpu(), y.cpu(), torch.stack(snaps).cpu(), out


@pytest.mark.parametrize("method", ["rk4", "rkck45"])
def test_graph_equals_host_loop_and_replays(ode, method):
    import torch
    from paper_1810_03931_amd import ensemble as E
    pb = _duffing1(3000)
    if method == "rkck45":
        pb.method = "rkck45"
        pb.options.update(h0=1e-3, rtol=1e-9, atol=1e-9)
    n_seg, first = 24, 16
    ens = E.Ensemble(pb.model, pb.method)
    td_e, y_e, snap_e, _ = _eager(ens, pb, n_seg, first)

    ens_g = E.Ensemble(pb.model, pb.method)
    td, y, p = _device(pb)
    out = ens_g.outputs(pb.n, n_accessories=1)
    snaps = torch.full((n_seg - first, 4, pb.n), float("nan"), dtype=torch.float64, device="cuda")
    td0, y0 = td.clone(), y.clone()
    for rep in range(3):
        td.copy_(td0)
        y.copy_(y0)
        snaps.fill_(float("nan"))
        ens_g.solve_segments(td, y, p, n_seg, T, first_snapshot=first, snapshots=snaps, out=out,
                             **pb.options)
        torch.cuda.synchronize()
        assert torch.equal(td.cpu(), td_e), f"replay {rep}: time domain"
        assert torch.equal(y.cpu(), y_e), f"replay {rep}: state"
        assert torch.equal(snaps.cpu(), snap_e), f"replay {rep}: snapshots"
        # eager work of the program between replays, including a plain solve
        # on the same handle and a reduction over many blocks
        _ = (snaps.sum() + y.abs().max()).item()
        tdx, yx, px = _device(pb)
        ens_g.solve(tdx, yx, px, **pb.options)
        torch.cuda.synchronize()
    print(f"[segments] {method}: graph == host loop over {n_seg} segments, 3 replays", flush=True)


def _oracle_loop(pb, y0, n_seg, first):
    from oracle import oracle as O
    td, y = pb.time_domain.copy(), y0.copy()
    snaps = []
    for k in range(n_seg):
        td[1] = td[0] + T
        ro = O.solve(pb.model, pb.method, td, y, pb.params, **pb.options)
        if k >= first:
            snaps.append(np.concatenate([y, ro["acc"]]))
    return td, np.stack(snaps)


def test_host_loop_matches_oracle_loop(ode, oracle):
    """The graph's segments against the oracle doing the same loop, with the
    conditioning-aware bar of the sweeps' parity tests: the oracle's own
    rounding-level twins (initial state moved by 1e-15, parameters by one ulp)
    give each snapshot row's sensitivity (the double-well transient is
    chaotic)."""
    from paper_1810_03931_amd import ensemble as E
    pb = _duffing1(777)
    n_seg, first = 6, 3
    ens = E.Ensemble(pb.model, pb.method)
    td, y, p = _device(pb)
    out = ens.outputs(pb.n, n_accessories=1)
    r = ens.solve_segments(td, y, p, n_seg, T, first_snapshot=first, out=out, **pb.options)
    snaps = r["snapshots"].cpu().numpy()
    tdo, exp = _oracle_loop(pb, pb.state, n_seg, first)
    scale = np.maximum(np.abs(exp), 1.0)
    floor = np.zeros(exp.shape[1:])                 # [snapshot row, system]
    for tw_pb in short_twins(pb):
        _, tw = _oracle_loop(tw_pb, tw_pb.state, n_seg, first)
        floor = np.maximum(floor, np.max(np.abs(tw - exp) / scale, axis=0))
    bar = np.maximum(1e-11, 100.0 * floor)
    err = np.max(np.abs(snaps - exp) / scale, axis=0)
    print(f"[segments] oracle loop: max err {err.max():.3e}, rows held at 1e-11: "
          f"{np.sum(bar == 1e-11)} of {bar.size}, systems with a floor > 1e-13: "
          f"{np.sum(np.any(floor > 1e-13, axis=0))} of {pb.n}", flush=True)
    assert np.all(err <= bar)
    assert np.array_equal(td.cpu().numpy()[0], tdo[0])


def test_segments_arguments_are_validated(ode):
    import torch
    from paper_1810_03931_amd import ensemble as E
    pb = _duffing1(64)
    ens = E.Ensemble(pb.model, pb.method)
    td, y, p = _device(pb)
    snaps = torch.zeros((2, 4, pb.n), dtype=torch.float64, device="cuda")
    for n_seg, seg, first in ((0, T, 0), (2, 0.0, 0), (2, float("nan"), 0), (2, T, 3),
                              (2, T, -1)):
        with pytest.raises(E.OdeError) as ei:
            ens.solve_segments(td, y, p, n_seg, seg, first_snapshot=first, snapshots=snaps,
                               **pb.options)
        assert ei.value.code == E.EINVAL
    torch.cuda.synchronize()
    assert torch.equal(td.cpu(), torch.as_tensor(pb.time_domain))


def test_segments_with_gather_list_and_window_starts(ode):
    """The graph honours a gather list (only the listed systems move) and
    per-system window starts, exactly as the host loop does."""
    import torch
    from paper_1810_03931_amd import ensemble as E
    pb = _duffing1(2000)
    dev = torch.device("cuda", 0)
    idx = torch.arange(3, 2000, 3, dtype=torch.int64, device=dev)
    starts = torch.as_tensor(np.linspace(-1.0, 3 * T, pb.n), device=dev)
    n_seg, first = 5, 2
    ens = E.Ensemble(pb.model, pb.method)
    td_e, y_e, p = _device(pb)
    snaps_e = []
    for k in range(n_seg):
        td_e[1, idx] = td_e[0, idx] + T
        out = ens.solve(td_e, y_e, p, system_index=idx, record_start=starts, **pb.options)
        if k >= first:
            snaps_e.append(torch.cat([y_e, out["acc"]])[:, idx].clone())
    td, y, p = _device(pb)
    out = ens.outputs(pb.n, n_accessories=1)
    r = ens.solve_segments(td, y, p, n_seg, T, first_snapshot=first, system_index=idx,
                           record_start=starts, out=out, **pb.options)
    torch.cuda.synchronize()
    assert torch.equal(td, td_e) and torch.equal(y, y_e)
    assert torch.equal(r["snapshots"][:, :, idx], torch.stack(snaps_e))
    untouched = torch.ones(pb.n, dtype=torch.bool, device=dev)
    untouched[idx] = False
    assert torch.equal(y[:, untouched].cpu(), torch.as_tensor(pb.state)[:, untouched.cpu()])
