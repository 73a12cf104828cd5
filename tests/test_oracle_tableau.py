"""Pins for the oracle's Cash-Karp tableau: the Runge-Kutta order conditions.

The paper names the Cash-Karp 4(5) pair (Sec. 3) without printing it.  Instead
of re-reading the coefficients, these tests check what makes them a 4(5) pair:
the rooted-tree order conditions, generated here from the tree definitions,
in exact rational arithmetic.
"""
import math
from fractions import Fraction

import numpy as np


def _as_rational(x):
    """The short rational a tableau double was rounded from."""
    f = Fraction(x).limit_denominator(10**7)
    assert float(f) == x, (x, f)
    return f


def _trees(order):
    """All rooted trees with ``order`` vertices, as sorted tuples of subtrees."""
    if order == 1:
        return [()]
    out = set()

    def partitions(n, maxpart):
        if n == 0:
            yield []
            return
        for p in range(min(n, maxpart), 0, -1):
            for rest in partitions(n - p, p):
                yield [p] + rest

    for parts in partitions(order - 1, order - 1):
        def combos(i):
            if i == len(parts):
                yield []
                return
            for t in _trees(parts[i]):
                for rest in combos(i + 1):
                    yield [t] + rest
        for kids in combos(0):
            out.add(tuple(sorted(kids)))
    return sorted(out)


def _gamma(t):
    n = 1 + sum(_size(k) for k in t)
    g = n
    for k in t:
        g *= _gamma(k)
    return g


def _size(t):
    return 1 + sum(_size(k) for k in t)


def _phi(t, A, s):
    """Elementary weight vector Phi_i(t) for stages i."""
    v = [Fraction(1)] * s
    for k in t:
        pk = _phi(k, A, s)
        inner = [sum(A[i][j] * pk[j] for j in range(s)) for i in range(s)]
        v = [v[i] * inner[i] for i in range(s)]
    return v


def _conditions(b, A, max_order):
    res = {}
    for p in range(1, max_order + 1):
        for t in _trees(p):
            lhs = sum(b[i] * _phi(t, A, len(b))[i] for i in range(len(b)))
            res[(p, t)] = lhs == Fraction(1, _gamma(t))
    return res


def test_tree_counts():
    # 1, 1, 2, 4, 9 rooted trees of order 1..5: 17 conditions up to order 5.
    assert [len(_trees(p)) for p in range(1, 6)] == [1, 1, 2, 4, 9]


def test_cash_karp_order_conditions(oracle):
    c, a, b, bs, e = oracle.tableau()
    A = [[_as_rational(a[i, j]) for j in range(6)] for i in range(6)]
    C = [_as_rational(x) for x in c]
    B = [_as_rational(x) for x in b]
    BS = [_as_rational(x) for x in bs]
    # explicit: strictly lower triangular; row sums equal the nodes
    for i in range(6):
        assert all(A[i][j] == 0 for j in range(i, 6))
        assert sum(A[i]) == C[i]
    fifth = _conditions(B, A, 5)
    assert len(fifth) == 17 and all(fifth.values()), "propagated weights must be order 5"
    fourth = _conditions(BS, A, 5)
    assert all(v for (p, _), v in fourth.items() if p <= 4), "embedded weights must be order 4"
    assert not any(v for (p, _), v in fourth.items() if p == 5), "embedded weights are not order 5"


def test_error_weights_are_difference(oracle):
    c, a, b, bs, e = oracle.tableau()
    for i in range(6):
        assert _as_rational(e[i]) == _as_rational(b[i]) - _as_rational(bs[i])
    assert abs(sum(_as_rational(x) for x in e)) == 0


def test_rk4_is_classical(oracle):
    """One RK4 step on the undamped linear oscillator x'' = -x: the classical
    RK4 amplification of a rotation by h is the degree-4 Taylor polynomial of
    exp(-i h) acting on x + i v."""
    h = 0.3
    y0 = np.array([1.0, 0.0])
    p = np.array([0.0, 0.0, 1.0, 1.0, 0.0])     # k = 0, B = 0, lin = 1, cub = 0
    y1, _ = oracle.step("duffing", "rk4", 0.0, y0, p, h)
    z = sum((1j * h) ** m / math.factorial(m) for m in range(5))
    # x = Re, v = -Im for x'' = -x starting at (1, 0): (x, v) -> (Re z, -Im z)
    assert abs(y1[0] - z.real) < 1e-15 and abs(y1[1] + z.imag) < 1e-15
