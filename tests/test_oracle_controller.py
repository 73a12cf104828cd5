"""Pin of the oracle's adaptive step control (error norm, step factor,
accept/reject, clipping to the end of the interval) against an independent
formulation of the same method.

For a linear autonomous system y' = A y every Cash-Karp stage is a matrix
times y: k_i = A M_i y with M_i = I + h sum_j a_ij A M_j.  The propagated
solution is (I + h sum_i b_i A M_i) y and the error estimate h sum_i e_i A M_i y.
This test builds those matrices from the tableau (pinned on its own by the
order conditions), runs the step-size control of paper Sec. 6.5 as read in
the design notes on them, and requires the oracle's stage-by-stage
integration of the linear Duffing oscillator (cub = 0, B = 0) to take exactly
the same accepted and rejected steps to the same final state.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _replica(A, y0, t1, *, h0, rtol, atol, h_min, h_max, grow, shrink):
    c, a, b, bstar, e = O.tableau()
    I2 = np.eye(2)
    t, y, h = 0.0, y0.astype(float).copy(), h0
    n_acc = n_rej = 0
    while t < t1:
        h_try, clipped = (t1 - t, True) if h >= t1 - t else (h, False)
        M = []
        for i in range(6):
            M.append(I2 + h_try * sum(a[i, j] * (A @ M[j]) for j in range(i)))
        y5 = (I2 + h_try * sum(b[i] * (A @ M[i]) for i in range(6))) @ y
        err = (h_try * sum(e[i] * (A @ M[i]) for i in range(6))) @ y
        sc = atol + rtol * np.maximum(np.abs(y), np.abs(y5))
        E = float(np.max(np.abs(err) / sc))
        fac = grow if E == 0.0 else min(grow, max(shrink, 0.9 * E ** -0.2))
        h_next = min(h_max, max(h_min, fac * h_try))
        if E <= 1.0 or h_try <= h_min:
            t = t1 if clipped else t + h_try
            y = y5
            n_acc += 1
            h = max(h_next, h) if clipped else h_next
        else:
            h = h_next
            n_rej += 1
    return y, n_acc, n_rej, h


@pytest.mark.parametrize("k,lin,tol,h0", [(0.1, 1.0, 1e-8, 1e-3), (0.5, 4.0, 1e-10, 0.5),
                                          (2.0, 1.0, 1e-6, 2.0), (0.0, 9.0, 1e-9, 1e-4)])
def test_step_control_matches_matrix_replica(k, lin, tol, h0):
    A = np.array([[0.0, 1.0], [-lin, -k]])
    y0 = np.array([1.0, -0.3])
    t1 = 7.3
    opts = dict(h0=h0, rtol=tol, atol=tol, h_min=1e-12, h_max=1e6, grow=5.0, shrink=0.1)
    y_r, acc_r, rej_r, h_r = _replica(A, y0, t1, **opts)
    td = np.array([[0.0], [t1]])
    y = y0.reshape(2, 1).copy()
    p = np.array([[k], [0.0], [1.0], [lin], [0.0]])
    nh = np.zeros(1)
    r = O.solve("duffing", "rkck45", td, y, p, next_h=nh, **opts)
    assert r["status"][0] == O.DONE and td[0, 0] == t1
    assert r["counts"][0, 0] == acc_r and r["counts"][1, 0] == rej_r
    if h0 >= 0.5:
        assert rej_r >= 1                  # the large first steps are rejected
    # the same steps, rounded in a different order: agreement to rounding
    # accumulated over a few hundred steps
    np.testing.assert_allclose(y[:, 0], y_r, rtol=0, atol=1e-12 * np.max(np.abs(y_r)))
    # the error estimate is a small difference of stage sums: its rounding in the
    # two formulations differs at ~1e-10 relative, and h_next follows it
    assert abs(nh[0] - h_r) <= 1e-8 * h_r
