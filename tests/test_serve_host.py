"""Host logic of the served queues (no GPU): the slot allocator of a class
pool and the position ring's wrap-around."""
import numpy as np

from paper_1810_03931_amd.serve import _Resident


def _pool(cap):
    r = object.__new__(_Resident)
    r.cap = cap
    r.free = [(0, cap)]
    return r


def test_first_fit_and_merge():
    r = _pool(100)
    a = r._alloc(30)
    b = r._alloc(50)
    c = r._alloc(20)
    assert (a, b, c) == (0, 30, 80) and r.free == []
    assert r._alloc(1) is None
    r._release(b, 50)
    assert r._alloc(60) is None
    r._release(a, 30)
    assert r.free == [(0, 80)]            # neighbours merge
    r._release(c, 20)
    assert r.free == [(0, 100)]
    assert r._alloc(100) == 0


def test_ring_positions_never_collide_with_untaken_ones():
    """Queue position q holds slot ring[q % C].  With at most C systems in
    slots, the positions of a new request and those still untaken are distinct
    modulo C (the argument the kernel's ring relies on)."""
    rng = np.random.default_rng(5)
    C = 64
    r = _pool(C)
    published, taken = 0, 0
    live = []                                   # (start, m, first position)
    for _ in range(2000):
        if live and rng.random() < 0.5:
            # the oldest request finishes (its positions were taken first)
            a, m, q0 = live.pop(0)
            taken = max(taken, q0 + m)
            r._release(a, m)
        m = int(rng.integers(1, 20))
        a = r._alloc(m)
        if a is None:
            continue
        untaken = set(p % C for p in range(taken, published))
        new = set(p % C for p in range(published, published + m))
        assert not (untaken & new)
        live.append((a, m, published))
        published += m
