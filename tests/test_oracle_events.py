"""Pins for the oracle's event handling (paper Sec. 4 and Sec. 6.6).

Free flight y'' = -g has exact impact times, and Cash-Karp integrates its
quadratic trajectory exactly (up to rounding), so the only error left is the
event location, bounded by the event tolerance.  A bouncing ball with the
restitution action y2 <- -r*y2 has the closed-form bounce sequence
t_{n+1} = t_n + 2 r^n v_1 / g.  The steady state of the linear driven
oscillator has its maxima at w t = atan2(Bs, A) + 2 pi n.
"""
import math

import numpy as np

from oracle import oracle as O


def ball(oracle, y0, v0, g, t1, method="rkck45", **kw):
    td = np.array([[0.0], [t1]])
    st = np.array([[y0], [v0]])
    par = np.array([[g], [0.8]])[:1]
    r = oracle.solve("ballistic", method, td, st, par, **kw)
    return td[0, 0], st[:, 0], r


IMPACT = dict(component=0, level=0.0, direction=-1)


def test_first_impact_time(oracle):
    y0, v0, g, tol = 1.0, 0.5, 9.81, 1e-10
    t, y, r = ball(oracle, y0, v0, g, 10.0, h0=1e-2, h_max=10.0,
                   events=[dict(IMPACT, tolerance=tol, stop_after=1)])
    t_star = (v0 + math.sqrt(v0 * v0 + 2 * g * y0)) / g
    v_star = math.sqrt(v0 * v0 + 2 * g * y0)
    assert r["status"][0] == O.STOP_EVENT
    assert abs(y[0]) <= tol
    assert abs(t - t_star) <= tol / v_star + 1e-13
    assert r["counts"][2, 0] > 0                       # located by the secant
    assert r["event_counts"][0, 0] == 1


def test_bounce_sequence_with_restitution(oracle):
    """Action y2 <- (-1 * p[0]) * y2 with the restitution read from the
    parameters, as in the paper's impact law (Sec. 2.3)."""
    g, r_c, tol = 2.0, 0.8, 1e-11
    td = np.array([[0.0], [100.0]])
    st = np.array([[1.0], [0.0]])
    # restitution as a literal coefficient; the parameter array stays (g,).
    # h_max stays well below a flight time: Cash-Karp is exact on a parabola,
    # so the error test never limits the step, and a step spanning a whole
    # flight would end below the seat without a sign change to detect.
    par = np.array([[g]])
    n_b = 6
    r = oracle.solve("ballistic", "rkck45", td, st, par, h0=1e-2, h_max=0.05, t_record=0.0,
                     events=[dict(IMPACT, tolerance=tol, stop_after=n_b, action_component=1,
                                  action_coef=-r_c, record_component=0)],
                     record_cap=8)
    v1 = math.sqrt(2 * g * 1.0)
    t_n = [math.sqrt(2 * 1.0 / g)]
    for m in range(1, n_b):
        t_n.append(t_n[-1] + 2 * r_c**m * v1 / g)
    rec_t = r["event_records"][:n_b, 0, 0]
    assert r["status"][0] == O.STOP_EVENT
    assert r["event_counts"][0, 0] == n_b
    assert np.all(np.abs(rec_t - np.array(t_n)) <= 1e-9)
    assert np.all(np.abs(r["event_records"][:n_b, 1, 0]) <= tol)
    assert abs(td[0, 0] - t_n[-1]) <= 1e-9
    # after the last impact the velocity was reversed and damped by r
    assert abs(st[1, 0] - r_c**n_b * v1) <= 1e-8


def test_action_coefficient_from_parameter(oracle):
    """y[c] <- action_coef * p[action_param] * y[c] equals the literal form."""
    outs = []
    for kw in (dict(action_coef=-0.8), dict(action_coef=-1.0, action_param=0)):
        td = np.array([[0.0], [5.0]])
        st = np.array([[1.0], [0.0]])
        par = np.array([[0.8]])                    # g = 0.8 doubles as the coefficient
        oracle.solve("ballistic", "rkck45", td, st, par, h0=1e-2, h_max=0.05,
                     events=[dict(IMPACT, tolerance=1e-10, stop_after=3, action_component=1,
                                  **kw)])
        outs.append((td.copy(), st.copy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_initial_point_in_zone_is_not_detected(oracle):
    """Starting on the seat (inside the zone) is not an event (paper Sec. 7.2)."""
    g, v0 = 1.0, 1.0
    t, y, r = ball(oracle, 0.0, v0, g, 10.0, h0=1e-2, h_max=0.1,
                   events=[dict(IMPACT, tolerance=1e-10, stop_after=1)])
    assert r["status"][0] == O.STOP_EVENT
    assert abs(t - 2 * v0 / g) <= 1e-9


def test_landing_in_zone_needs_no_location(oracle):
    """RK4 with dt = 0.25 on y = 1 - t^2 lands exactly on y = 0 at t = 1: the
    event is detected inside the zone and no secant step is taken."""
    t, y, r = ball(oracle, 1.0, 0.0, 2.0, 10.0, method="rk4", h0=0.25,
                   events=[dict(IMPACT, tolerance=1e-12, stop_after=1)])
    assert r["status"][0] == O.STOP_EVENT
    assert t == 1.0 and abs(y[0]) <= 1e-12
    assert r["counts"][2, 0] == 0 and r["counts"][0, 0] == 4


def test_largest_index_is_located(oracle):
    """Two zones crossed in one step: the one specified last is located
    precisely (paper Sec. 4); the other is counted at the same point."""
    events = [dict(component=0, level=0.5, direction=-1, tolerance=1e-10),
              dict(component=0, level=0.4, direction=-1, tolerance=1e-10, stop_after=1)]
    t, y, r = ball(oracle, 1.0, 0.0, 1.0, 10.0, h0=2.0, h_max=10.0, events=events)
    assert r["status"][0] == O.STOP_EVENT
    assert abs(t - math.sqrt(1.2)) <= 1e-9            # where y = 0.4, not 0.5
    assert r["event_counts"][0, 0] == 1 and r["event_counts"][1, 0] == 1
    # reversed order: the 0.5 level is now last, so it is the one located
    events_rev = [dict(events[1], stop_after=0), dict(events[0], stop_after=1)]
    t2, _, r2 = ball(oracle, 1.0, 0.0, 1.0, 10.0, h0=2.0, h_max=10.0, events=events_rev)
    assert abs(t2 - 1.0) <= 1e-9
    assert r2["event_counts"][1, 0] == 1 and r2["event_counts"][0, 0] == 0


def _steady(k=0.3, B=0.7, w=1.0):
    D = (1 - w * w) ** 2 + (k * w) ** 2
    A, Bs = B * (1 - w * w) / D, B * k * w / D
    return A, Bs, math.hypot(A, Bs), math.atan2(Bs, A)


def test_direction_convention_maxima_minima(oracle):
    """Event y2 = 0: direction -1 (y2 decreasing) finds the maxima of y1,
    +1 the minima, 0 both (paper Sec. 6.6, Duffing3 setup)."""
    k, B, w = 0.3, 0.7, 1.0
    A, Bs, R, phi = _steady(k, B, w)
    T = 2 * math.pi / w
    tol = 1e-9
    out = {}
    for d in (-1, 1, 0):
        td = np.array([[0.0], [4 * T]])
        st = np.array([[A], [Bs * w]])
        par = np.array([[k], [B], [w], [1.0], [0.0]])
        r = oracle.solve("duffing", "rkck45", td, st, par, h0=1e-3, rtol=1e-12, atol=1e-12,
                         t_record=0.0, record_cap=16,
                         events=[dict(component=1, level=0.0, direction=d, tolerance=tol,
                                      record_component=0)])
        c = r["event_counts"][0, 0]
        out[d] = (c, r["event_records"][:c, 0, 0], r["event_records"][:c, 1, 0])
    c, t, x = out[-1]
    assert c == 4
    assert np.all(np.abs(x - R) <= 1e-9)
    assert np.allclose(t, (phi + 2 * math.pi * np.arange(4)) / w, atol=1e-7, rtol=0)
    c, t, x = out[1]
    assert c == 4 and np.all(np.abs(x + R) <= 1e-9)
    c, t, x = out[0]
    assert c == 8 and np.all(np.abs(np.abs(x) - R) <= 1e-9)
    assert np.all(np.diff(t) > 0)


def test_record_overflow_is_counted_not_stored(oracle):
    k, B, w = 0.3, 0.7, 1.0
    A, Bs, R, phi = _steady(k, B, w)
    td = np.array([[0.0], [6 * 2 * math.pi]])
    st = np.array([[A], [Bs * w]])
    par = np.array([[k], [B], [w], [1.0], [0.0]])
    r = oracle.solve("duffing", "rkck45", td, st, par, h0=1e-3, t_record=0.0, record_cap=3,
                     events=[dict(component=1, direction=-1, tolerance=1e-8, record_component=0)])
    assert r["event_counts"][0, 0] == 6
    assert np.all(np.isfinite(r["event_records"][:3, :, 0]))


def test_window_counts_only_recorded_interval(oracle):
    k, B, w = 0.3, 0.7, 1.0
    A, Bs, R, phi = _steady(k, B, w)
    T = 2 * math.pi
    td = np.array([[0.0], [6 * T]])
    st = np.array([[A], [Bs * w]])
    par = np.array([[k], [B], [w], [1.0], [0.0]])
    r = oracle.solve("duffing", "rkck45", td, st, par, h0=1e-3, t_record=4 * T, record_cap=8,
                     events=[dict(component=1, direction=-1, tolerance=1e-8, record_component=0)])
    assert r["event_counts"][0, 0] == 2
    assert np.all(r["event_records"][:2, 0, 0] >= 4 * T)


def test_equilibrium_stop(oracle):
    """Relief valve above the Hopf point converges to its equilibrium inside
    the zone of the event y2 = 0 and stops after 50 steps there (paper Sec. 4,
    configuration d; Sec. 7.3)."""
    q, delta = 10.0, 10.0
    y1s = np.roots([1.0, delta, 0.0, -q * q])
    y1s = float(np.real(y1s[(np.abs(np.imag(y1s)) < 1e-12) & (np.real(y1s) > 0)][0]))
    td = np.array([[0.0], [1e4]])
    st = np.array([[0.0], [0.0], [delta]])
    par = np.array([[1.25], [delta], [20.0], [q], [0.8]])
    r = oracle.solve("relief_valve", "rkck45", td, st, par, h0=1e-3, max_equilibrium_steps=50,
                     events=[dict(component=1, direction=-1, tolerance=1e-6)])
    assert r["status"][0] == O.STOP_EQUILIBRIUM
    assert abs(st[0, 0] - y1s) < 1e-5 and abs(st[2, 0] - (y1s + delta)) < 1e-5
    assert td[0, 0] < 1e4


def test_nan_at_minimum_step_stops(oracle):
    """A negative chamber pressure makes sqrt(y3) NaN: the step is rejected and
    shrunk until the minimum step, then the system stops (paper Sec. 6.5)."""
    td = np.array([[0.0], [1.0]])
    st = np.array([[0.1], [0.0], [-1.0]])
    par = np.array([[1.25], [10.0], [20.0], [5.0], [0.8]])
    r = oracle.solve("relief_valve", "rkck45", td, st, par, h0=1e-2, h_min=1e-6)
    assert r["status"][0] == O.FAIL_NAN
    # 1e-2 -> 1e-3 -> ... -> 1e-6 (one more if 0.1*1e-5 rounds above 1e-6)
    assert 4 <= r["counts"][1, 0] <= 5 and r["counts"][0, 0] == 0


def test_minimum_step_continues_without_tolerance(oracle):
    """With h_min = h_max the error test is waived: nothing is rejected."""
    td = np.array([[0.0], [2.0]])
    st = np.array([[1.0], [0.0]])
    par = np.array([[0.1], [5.0], [1.0], [1.0], [1.0]])
    r = oracle.solve("duffing", "rkck45", td, st, par, h0=0.5, h_min=0.5, h_max=0.5,
                     rtol=1e-14, atol=1e-14)
    assert r["status"][0] == O.DONE and r["counts"][1, 0] == 0 and r["counts"][0, 0] == 4


def test_max_steps_budget(oracle):
    td = np.array([[0.0], [100.0]])
    st = np.array([[1.0], [0.0]])
    par = np.array([[0.1], [0.3], [1.0], [1.0], [1.0]])
    r = oracle.solve("duffing", "rkck45", td, st, par, h0=1e-3, max_steps=37)
    assert r["status"][0] == O.MAX_STEPS
    assert r["counts"][:, 0].sum() == 37
    assert 0.0 < td[0, 0] < 100.0


def test_per_system_record_start_equals_separate_solves():
    """A per-system window start gives, for every system, what a separate
    solve with that scalar t_record gives (bit for bit)."""
    from oracle import oracle as O
    import numpy as np
    n = 12
    T = 2 * np.pi
    k = np.linspace(0.1, 0.5, n)
    p = np.stack([k, np.full(n, 1.0), np.ones(n), np.ones(n), np.ones(n)])
    y0 = np.zeros((2, n))
    td0 = np.stack([np.zeros(n), np.full(n, 6 * T)])
    starts = np.linspace(-1.0, 7 * T, n)          # before t0, inside, and after t1
    opts = dict(h0=1e-3, rtol=1e-9, atol=1e-9, accessories=[("max", 0), ("min", 1)],
                events=[dict(component=1, direction=-1, record_component=0)], record_cap=8)
    td, y = td0.copy(), y0.copy()
    r = O.solve("duffing", "rkck45", td, y, p, record_start=starts, **opts)
    for s in range(n):
        tds, ys = td0[:, s:s + 1].copy(), y0[:, s:s + 1].copy()
        rs = O.solve("duffing", "rkck45", tds, ys, p[:, s:s + 1].copy(), t_record=starts[s], **opts)
        assert np.array_equal(ys[:, 0], y[:, s]) and tds[0, 0] == td[0, s]
        np.testing.assert_array_equal(rs["acc"][:, 0], r["acc"][:, s])
        np.testing.assert_array_equal(rs["event_counts"][:, 0], r["event_counts"][:, s])
        np.testing.assert_array_equal(rs["event_records"][:, :, 0], r["event_records"][:, :, s])
