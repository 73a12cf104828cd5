"""Pins for the oracle's stepping and step control on closed-form solutions.

The linear driven damped oscillator x'' + k x' + x = B cos(w t) (the Duffing
model of paper Sec. 2.1 with no cubic term) has an exact solution.  It fixes:
  * RK4 global error of order 4 and Cash-Karp (fixed step, h_min = h_max) of
    order 5 -- measured slopes, paper Sec. 3;
  * the embedded solution's local error of order 5 (order 4 method) and the
    propagated one of order 6 (order 5 method);
  * the adaptive controller: error tracks the tolerance and the step count
    grows like tol^(-1/5).
"""
import math

import numpy as np
import pytest


def exact(t, x0, v0, k, B, w):
    """Closed form of x'' + k x' + x = B cos(w t), 0 < k < 2."""
    D = (1.0 - w * w) ** 2 + (k * w) ** 2
    A = B * (1.0 - w * w) / D
    Bs = B * k * w / D
    wd = math.sqrt(1.0 - k * k / 4.0)
    c1 = x0 - A
    c2 = (v0 - Bs * w + 0.5 * k * c1) / wd
    e = math.exp(-0.5 * k * t)
    x = e * (c1 * math.cos(wd * t) + c2 * math.sin(wd * t)) + A * math.cos(w * t) + Bs * math.sin(w * t)
    dx = (-0.5 * k * e * (c1 * math.cos(wd * t) + c2 * math.sin(wd * t))
          + e * wd * (-c1 * math.sin(wd * t) + c2 * math.cos(wd * t))
          - A * w * math.sin(w * t) + Bs * w * math.cos(w * t))
    return np.array([x, dx])


K, BAMP, W, X0, V0 = 0.3, 0.7, 1.3, 0.4, -0.2
PAR = np.array([[K], [BAMP], [W], [1.0], [0.0]])


def _run(oracle, method, T, h, **kw):
    td = np.array([[0.0], [T]])
    st = np.array([[X0], [V0]])
    r = oracle.solve("duffing", method, td, st, PAR.copy(), h0=h, **kw)
    assert r["status"][0] == 0
    assert td[0, 0] == T, "the final step must land exactly on t1"
    return st[:, 0], r


def _slope(hs, errs):
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


def test_exact_solution_is_consistent():
    # the closed form satisfies the ODE (finite difference) and the initial data
    t, d = 1.7, 1e-5
    x = lambda s: exact(s, X0, V0, K, BAMP, W)[0]
    xdd = (x(t + d) - 2 * x(t) + x(t - d)) / d**2
    xd = exact(t, X0, V0, K, BAMP, W)[1]
    assert abs(xdd + K * xd + x(t) - BAMP * math.cos(W * t)) < 1e-5
    assert np.allclose(exact(0.0, X0, V0, K, BAMP, W), [X0, V0], atol=1e-15)


def test_rk4_global_order_4(oracle):
    T = 5.0
    ref = exact(T, X0, V0, K, BAMP, W)
    hs = np.array([T / 40, T / 80, T / 160, T / 320])
    errs = [np.max(np.abs(_run(oracle, "rk4", T, h)[0] - ref)) for h in hs]
    assert 3.9 <= _slope(hs, errs) <= 4.1


def test_cash_karp_fixed_step_global_order_5(oracle):
    T = 5.0
    ref = exact(T, X0, V0, K, BAMP, W)
    hs = np.array([T / 10, T / 20, T / 40, T / 80])
    errs = []
    for h in hs:
        y, r = _run(oracle, "rkck45", T, h, h_min=h, h_max=h, rtol=1e-30, atol=1e-30)
        assert r["counts"][1, 0] == 0          # nothing rejected at h = h_min
        errs.append(np.max(np.abs(y - ref)))
    assert 4.9 <= _slope(hs, errs) <= 5.15


def test_local_error_orders(oracle):
    """One step from the exact solution: propagated (5th order) local error
    ~ h^6, embedded (4th order, y5 - err) local error ~ h^5."""
    t0 = 0.9
    y0 = exact(t0, X0, V0, K, BAMP, W)

    def local(h):
        y5, err = oracle.step("duffing", "rkck45", t0, y0, PAR[:, 0], h)
        ref = exact(t0 + h, X0, V0, K, BAMP, W)
        return np.max(np.abs(y5 - ref)), np.max(np.abs(y5 - err - ref))

    h5 = np.array([0.2, 0.1, 0.05, 0.025])
    assert 5.8 <= _slope(h5, [local(h)[0] for h in h5]) <= 6.2
    # the embedded solution reaches its asymptotic regime at smaller steps
    # (above the rounding floor, which 0.005 already reaches)
    h4 = np.array([0.04, 0.02, 0.01])
    assert 4.75 <= _slope(h4, [local(h)[1] for h in h4]) <= 5.2


@pytest.mark.parametrize("tol", [1e-6, 1e-8, 1e-10])
def test_adaptive_error_tracks_tolerance(oracle, tol):
    T = 20.0
    ref = exact(T, X0, V0, K, BAMP, W)
    y, r = _run(oracle, "rkck45", T, 1e-3, rtol=tol, atol=tol, h_min=1e-12, h_max=1e6)
    err = np.max(np.abs(y - ref))
    assert err <= 50 * tol
    assert r["counts"][2, 0] == 0


def test_adaptive_step_count_scaling(oracle):
    T = 20.0
    tols = np.array([1e-6, 1e-8, 1e-10, 1e-12])
    steps = [_run(oracle, "rkck45", T, 1e-3, rtol=t, atol=t)[1]["counts"][0, 0] for t in tols]
    s = _slope(tols, steps)
    assert -0.23 <= s <= -0.17, s     # accepted steps ~ tol^(-1/5)


def test_rk4_grid_and_window(oracle):
    """96 periods at dt = T/200 are exactly 19200 RK4 steps; the window opens
    at 64 periods and the accessory times fall inside it."""
    T = 2 * math.pi
    td = np.array([[0.0], [96 * T]])
    st = np.array([[1e-3], [0.0]])
    par = np.array([[0.2], [1.0], [1.0], [1.0], [1.0]])
    r = oracle.solve("duffing", "rk4", td, st, par, h0=T / 200, t_record=64 * T,
                     accessories=[("max", 0), ("min", 0)])
    assert r["counts"][0, 0] == 19200 and r["counts"][1, 0] == 0
    assert td[0, 0] == 96 * T
    acc = r["acc"][:, 0]
    assert 64 * T <= acc[1] <= 96 * T and 64 * T <= acc[3] <= 96 * T
    assert acc[0] > 0 > acc[2]


@pytest.mark.parametrize("method", ["rk4", "rkck45"])
def test_accessory_grid_max_brackets_amplitude(oracle, method):
    """On the steady state x = A cos wt + Bs sin wt the grid maximum lies at
    most the sampling bound R (w h)^2 / 8 below the exact amplitude
    R = sqrt(A^2 + Bs^2) and no more than the integration error above it."""
    k, B, w = 0.3, 0.7, 1.0
    D = (1 - w * w) ** 2 + (k * w) ** 2
    A, Bs = B * (1 - w * w) / D, B * k * w / D
    R = math.hypot(A, Bs)
    T = 2 * math.pi / w
    dt = T / 200
    td = np.array([[0.0], [3 * T]])
    st = np.array([[A], [Bs * w]])
    par = np.array([[k], [B], [w], [1.0], [0.0]])
    r = oracle.solve("duffing", method, td, st, par, h0=dt, t_record=0.0, rtol=1e-12,
                     atol=1e-12, h_max=dt, accessories=[("max", 0), ("min", 0)])
    amax, amin = r["acc"][0, 0], r["acc"][2, 0]
    integ = 1e-6 if method == "rk4" else 1e-10     # RK4 global error at T/200
    slack = R * (w * dt) ** 2 / 8
    assert R - slack - integ <= amax <= R + integ
    assert -R - integ <= amin <= -R + slack + integ
