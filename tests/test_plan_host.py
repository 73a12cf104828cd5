"""Queue planner (ode_plan_order): host logic, no GPU.  The planner only
reorders queue positions; these tests check that every position survives
exactly once, chunks of 64 stay whole and in order, and the dealing puts a
long and a short chunk on each pair of SIMD partner waves."""
import numpy as np
import pytest

from paper_1810_03931_amd import ensemble as E


def _chunks(n):
    return [np.arange(k, min(n, k + 64)) for k in range(0, n, 64)]


@pytest.mark.parametrize("n", [64 * 2048, 64 * 2048 - 100, 64 * 1500 + 7])
def test_resident_deal_pairs_long_with_short(n):
    rng = np.random.default_rng(n)
    cost = rng.integers(1000, 500000, size=n)
    waves, rw = 2048, 1024
    out = E.plan_order(cost, waves, rw)
    assert out.size == waves * 64
    filled = out[out >= 0]
    assert np.array_equal(np.sort(filled), np.arange(n))          # every position once
    assert np.sum(out < 0) == waves * 64 - n
    per_wave = out.reshape(waves, 64)
    cc = {}
    for w in range(waves):                                         # whole chunks, in order
        v = per_wave[w][per_wave[w] >= 0]
        if v.size:
            assert v[0] % 64 == 0 and np.array_equal(v, np.arange(v[0], v[0] + v.size))
            cc[w] = cost[v].max()
        else:
            cc[w] = 0
    # partners: wave w of the first dispatch round shares a SIMD with wave w of the second
    pair = np.array([cc[w] + cc[w + rw] for w in range(rw)])
    chunk_cost = np.array([cost[c].max() for c in _chunks(n)])
    srt = np.sort(chunk_cost)[::-1]
    srt = np.concatenate([srt, np.zeros(2 * rw - srt.size, dtype=srt.dtype)])
    best = (srt[:rw] + srt[rw:][::-1]).max()                      # longest with shortest
    assert pair.max() == best
    ident = np.array([chunk_cost[w] + (chunk_cost[w + rw] if w + rw < chunk_cost.size else 0)
                      for w in range(rw)])
    assert pair.max() <= ident.max()


def test_not_resident_is_longest_first_and_complete():
    rng = np.random.default_rng(3)
    n = 64 * 40 + 5
    cost = rng.integers(0, 1000, size=n)
    queue = rng.permutation(10 * n)[:n]                           # caller's own system index
    out = E.plan_order(cost, waves=4, round_waves=8, queue=queue)
    assert out.size == n
    assert np.array_equal(np.sort(out), np.sort(queue))
    pos = {int(s): q for q, s in enumerate(queue)}
    src = np.array([pos[int(s)] for s in out])                    # original positions
    starts = [i for i in range(n) if i == 0 or src[i] != src[i - 1] + 1]
    costs = [cost[src[a:b]].max() for a, b in zip(starts, starts[1:] + [n])]
    assert all(x >= y for x, y in zip(costs, costs[1:]))          # chunks, most expensive first
    assert all(src[a] % 64 == 0 for a in starts)


def test_ties_keep_order_and_rounds_alternate():
    n, waves, rw = 64 * 8, 8, 4
    out = E.plan_order(np.ones(n, dtype=np.int64), waves, rw)
    first = out.reshape(waves, 64)[:, 0] // 64
    # equal costs: chunk ranks 0..3 forward in the first dispatch round, 4..7 backward in the second
    assert list(first) == [0, 1, 2, 3, 7, 6, 5, 4]


def test_degenerate_and_errors():
    assert E.plan_order(np.zeros(0, dtype=np.int64), 4, 4).size == 0
    one = E.plan_order(np.array([5]), 1, 1)
    assert one[0] == 0 and np.all(one[1:] == -1) and one.size == 64
    with pytest.raises(E.OdeError):
        E.plan_order(np.ones(10, dtype=np.int64), 0, 1)
    with pytest.raises(E.OdeError):
        E.plan_order(np.ones(10, dtype=np.int64), 1, 0)
    with pytest.raises(ValueError):
        E.plan_order(np.ones(10, dtype=np.int64), 1, 1, queue=np.arange(3))
