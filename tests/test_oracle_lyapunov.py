"""Pins of the oracle's Lyapunov workload: the Duffing system with its
linearisation in polar coordinates (paper Sec. 2.1, Eqs. (3)-(6)), Poincare
sections t_n = n*T as forced step boundaries, and the log-and-reset
accumulator of the largest Lyapunov exponent.

Pinned against:
  * the matrix exponential (scipy) of the constant-coefficient variational
    system of the linear oscillator (cub = 0), whose tangent vector is
    w(t) = expm(A t) w(0) exactly: the accumulated sum of logarithms, the
    final angle, and the limits -k/2 (under-damped) and the slow eigenvalue
    (over-damped);
  * central finite differences of the plain Duffing model (a second oracle
    model) for the nonlinear tangent dynamics, which fixes g1 = dF2/dy1 and
    g2 = dF2/dy2;
  * the same quantity without resets (linear growth of r), for the reset logic;
  * exact counts of the sections that fall inside the window.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import oracle as O

T = 2.0 * math.pi
TOL = dict(rtol=1e-11, atol=1e-11, h0=1e-3, h_min=1e-14, h_max=1e6, grow=5.0, shrink=0.1)


def _params(k, B, w, lin, cub):
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    n = k.size
    return np.stack([k, np.broadcast_to(B, n), np.broadcast_to(w, n), np.broadcast_to(lin, n),
                     np.broadcast_to(cub, n)]).astype(np.float64).copy()


def _run(p, y0, t0, t1, **kw):
    n = p.shape[1]
    td = np.stack([np.full(n, t0), np.full(n, t1)]).astype(np.float64)
    y = np.ascontiguousarray(np.array(y0, dtype=np.float64).reshape(4, -1) * np.ones((1, n)))
    opts = dict(TOL)
    opts.update(kw)
    method = opts.pop("method", "rkck45")
    r = O.solve("duffing_lyapunov", method, td, y, p, **opts)
    return td, y, r


def test_rhs_is_polar_form_of_tangent_dynamics():
    """r' and phi' follow from u' = v, v' = g1 u + g2 v with (u, v) = r(cos, sin)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        k, B, w, lin, cub = rng.uniform(0.05, 1.0), rng.uniform(0, 2), rng.uniform(0.5, 2), \
            rng.uniform(-1.5, 1.5), rng.uniform(0, 2)
        y1, y2, r, phi = rng.normal(), rng.normal(), rng.uniform(0.5, 3.0), rng.uniform(-7, 7)
        t = rng.uniform(0, 50)
        p = np.array([k, B, w, lin, cub])
        f = O.rhs("duffing_lyapunov", t, [y1, y2, r, phi], p)
        # The first two components are the plain Duffing model.
        np.testing.assert_array_equal(f[:2], O.rhs("duffing", t, [y1, y2], p))
        # Tangent dynamics by finite differences of the plain model's right-hand side.
        eps = 1e-6
        J = np.zeros((2, 2))
        for j in range(2):
            d = np.zeros(2)
            d[j] = eps
            J[:, j] = (O.rhs("duffing", t, np.array([y1, y2]) + d, p)
                       - O.rhs("duffing", t, np.array([y1, y2]) - d, p)) / (2 * eps)
        u, v = r * math.cos(phi), r * math.sin(phi)
        du, dv = J @ np.array([u, v])
        r_dot = (u * du + v * dv) / r
        phi_dot = (u * dv - v * du) / r**2
        assert abs(f[2] - r_dot) <= 1e-7 * max(1.0, abs(r_dot))
        assert abs(f[3] - phi_dot) <= 1e-7 * max(1.0, abs(phi_dot))


@pytest.mark.parametrize("k,lin", [(0.1, 1.0), (0.5, 1.0), (3.0, 2.0), (0.3, 4.0)])
def test_linear_oscillator_matches_matrix_exponential(k, lin):
    """cub = 0: constant tangent matrix A = [[0, 1], [-lin, -k]]; the sum of
    ln r over the window's sections is ln|expm(A t1) w0| - ln|expm(A t_rec) w0|."""
    phi0 = 0.3
    p = _params(k, 0.3, 1.0, lin, 0.0)
    t_rec, t1 = 5 * T, 15 * T
    td, y, r = _run(p, [0.0, 0.0, 1.0, phi0], 0.0, t1, t_record=t_rec, section_period=T,
                    accessories=[("log_reset", 2)])
    assert r["status"][0] == O.DONE and td[0, 0] == t1
    A = np.array([[0.0, 1.0], [-lin, -k]])
    w0 = np.array([math.cos(phi0), math.sin(phi0)])
    w_rec, w_end = expm(A * t_rec) @ w0, expm(A * t1) @ w0
    expect = math.log(np.linalg.norm(w_end)) - math.log(np.linalg.norm(w_rec))
    assert r["acc"][1, 0] == 10.0                          # sections t_rec+T .. t1
    assert abs(r["acc"][0, 0] - expect) <= 1e-8 * max(1.0, abs(expect))
    assert y[2, 0] == 1.0                                  # reset at the final section t1
    ang = math.atan2(w_end[1], w_end[0])
    assert abs(math.remainder(y[3, 0] - ang, 2 * math.pi)) <= 1e-8


@pytest.mark.parametrize("k,lin,lam", [(0.1, 1.0, -0.05), (0.4, 2.0, -0.2),
                                       (3.0, 2.0, -1.0), (5.0, 4.0, -1.0)])
def test_linear_oscillator_exponent_limit(k, lin, lam):
    """lambda = (sum ln r) / (count * T) tends to the largest real part of the
    eigenvalues of A: -k/2 (under-damped) or (-k + sqrt(k^2 - 4 lin))/2."""
    p = _params(k, 0.3, 1.0, lin, 0.0)
    _, _, r = _run(p, [0.2, 0.0, 1.0, 1.0], 0.0, 150 * T, t_record=30 * T, section_period=T,
                   accessories=[("log_reset", 2)])
    est = r["acc"][0, 0] / (r["acc"][1, 0] * T)
    # Bounded oscillation of ln r about the exponential trend, spread over 120 periods.
    assert abs(est - lam) <= 2.0 / (120 * T)
    assert abs(est - lam) <= 3e-3


def test_nonlinear_tangent_matches_finite_differences():
    """Double-well Duffing (lin = -1, cub = 1): r(t)(cos phi, sin phi) equals the
    derivative of the flow along the initial tangent, computed by central
    differences of two plain-Duffing solves."""
    p = _params(0.25, 0.3, 1.0, -1.0, 1.0)
    y0 = np.array([0.8, -0.1])
    phi0 = 0.7
    t1 = 1.5 * T
    _, y, r = _run(p, [y0[0], y0[1], 1.0, phi0], 0.0, t1)
    assert r["status"][0] == O.DONE
    eps = 1e-5
    w0 = np.array([math.cos(phi0), math.sin(phi0)])
    ends = []
    for sgn in (1.0, -1.0):
        yy = np.ascontiguousarray((y0 + sgn * eps * w0).reshape(2, 1))
        td = np.array([[0.0], [t1]])
        O.solve("duffing", "rkck45", td, yy, p, **TOL)
        ends.append(yy[:, 0])
    tangent = (ends[0] - ends[1]) / (2 * eps)
    got = y[2, 0] * np.array([math.cos(y[3, 0]), math.sin(y[3, 0])])
    np.testing.assert_allclose(got, tangent, rtol=1e-5, atol=1e-5 * np.linalg.norm(tangent))


def test_resets_equal_unreset_growth_nonlinear():
    """The per-section reset only rescales r (r' is linear in r and phi' does
    not depend on r): the window's sum of ln r equals ln(r(t1)/r(t_rec)) of a
    solve without resets."""
    p = _params(0.4, 0.3, 1.0, 1.0, 1.0)    # hardening single well, periodic response
    t_rec, t1 = 10 * T, 40 * T
    _, _, ra = _run(p, [0.1, 0.0, 1.0, 0.0], 0.0, t1, t_record=t_rec, section_period=T,
                    accessories=[("log_reset", 2)])
    td, yb, rb = _run(p, [0.1, 0.0, 1.0, 0.0], 0.0, t_rec)
    r_rec = yb[2, 0]
    td[1, 0] = t1
    O.solve("duffing_lyapunov", "rkck45", td, yb, p, **TOL)
    expect = math.log(yb[2, 0]) - math.log(r_rec)
    assert ra["acc"][1, 0] == 30.0
    assert abs(ra["acc"][0, 0] - expect) <= 1e-7 * abs(expect)


def test_section_placement_and_counts():
    """Sections are absolute multiples of T; a window start between sections
    counts only later ones; t0 that is not a multiple is handled; the final
    time is t1 exactly; RK4 visits the same sections."""
    p = _params(0.3, 0.3, 1.0, 1.0, 0.0)
    for method, h0 in (("rkck45", 1e-3), ("rk4", T / 200)):
        t0, t_rec, t1 = 2.5 * T, 7.25 * T, 19.5 * T
        td, y, r = _run(p, [0.0, 0.0, 1.0, 0.0], t0, t1, t_record=t_rec, section_period=T,
                        accessories=[("log_reset", 2), ("max", 0)], method=method, h0=h0)
        assert r["status"][0] == O.DONE and td[0, 0] == t1
        assert r["acc"][1, 0] == 12.0                   # n = 8 .. 19
        assert y[2, 0] != 1.0                            # t1 is not a section: r grew since 19 T
        # Split at a section: the second half visits the same sections.
        tda, ya, ra = _run(p, [0.0, 0.0, 1.0, 0.0], t0, 11 * T, t_record=t_rec,
                           section_period=T, accessories=[("log_reset", 2)], method=method, h0=h0)
        assert ra["acc"][1, 0] == 4.0                   # n = 8 .. 11
        assert ya[2, 0] == 1.0


def test_lyapunov_rk4_linear_limit():
    p = _params(0.2, 0.3, 1.0, 1.0, 0.0)
    _, _, r = _run(p, [0.0, 0.0, 1.0, 0.5], 0.0, 100 * T, t_record=20 * T, section_period=T,
                   accessories=[("log_reset", 2)], method="rk4", h0=T / 200)
    est = r["acc"][0, 0] / (r["acc"][1, 0] * T)
    assert r["acc"][1, 0] == 80.0
    assert abs(est + 0.1) <= 2.0 / (80 * T)


def test_log_reset_requires_sections():
    p = _params(0.2, 0.3, 1.0, 1.0, 0.0)
    with pytest.raises(ValueError):
        _run(p, [0.0, 0.0, 1.0, 0.0], 0.0, T, accessories=[("log_reset", 2)])
    with pytest.raises(ValueError):
        _run(p, [0.0, 0.0, 1.0, 0.0], 0.0, T, section_period=-1.0)
