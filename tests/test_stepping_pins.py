"""Pins of the stepping oracle (Sec. 4.2 time-step criteria; kick then drift)
to closed forms and hand-worked cases."""
import numpy as np
import pytest

import oracle


def test_kick_drift_constant_acceleration_closed_form():
    """Kick-then-drift with a constant a: after n steps of length dt,
    v_n = v_0 + n a dt and x_n = x_0 + n v_0 dt + a dt^2 n (n + 1) / 2."""
    x0 = np.array([[0.25, -1.0, 3.0]])
    v0 = np.array([[0.5, 0.25, -2.0]], dtype=np.float32)
    a = np.array([[1.0, -0.5, 0.125]], dtype=np.float32)
    dt = 0.0625            # a power of two: every product below is exact
    x, v = x0.copy(), v0.copy()
    n = 7
    for _ in range(n):
        x, v = oracle.kick_drift(x, v, a, dt, dt)
    np.testing.assert_array_equal(v, v0 + n * a * dt)
    np.testing.assert_array_equal(x, x0 + n * v0 * dt + a * dt * dt * n * (n + 1) / 2)


def test_kick_drift_rounding_model():
    """The kick is evaluated in double and rounded once to float; the drift
    uses the kicked float velocity."""
    rng = np.random.default_rng(2)
    x = rng.normal(size=(50, 3))
    v = rng.normal(size=(50, 3)).astype(np.float32)
    a = rng.normal(size=(50, 3)).astype(np.float32)
    k, d = 0.0137, 0.0291
    xn, vn = oracle.kick_drift(x, v, a, k, d)
    assert vn.dtype == np.float32
    np.testing.assert_array_equal(vn, (v.astype(np.float64) + k * a.astype(np.float64)).astype(np.float32))
    np.testing.assert_array_equal(xn, x + d * vn.astype(np.float64))


def test_step_stats_hand_worked():
    K, L = 5, 1.0
    h = L / K
    pos = np.array([[0.5, 0.5, 0.5], [0.6, 0.5, 0.5], [2.5, 0.5, 0.5]]) * h   # two in cell 0, one in cell (2,0,0)
    vel = np.array([[1, 0, 0], [0, 3, 4], [2, 3, 6]], dtype=np.float32)
    acc = np.array([[3, 4, 0], [0, 0, 1], [1, 2, 2]], dtype=np.float32)
    amax, vrms, glob = oracle.step_stats(pos, K, L, acc, vel)
    c1 = (2 * K + 0) * K + 0
    assert amax[0] == 5.0 and vrms[0] == np.sqrt(13.0)
    assert amax[c1] == 3.0 and vrms[c1] == 7.0
    assert np.count_nonzero(amax) == 2 and np.count_nonzero(vrms) == 2
    np.testing.assert_allclose(glob, [5.0, np.sqrt((1 + 25 + 49) / 3), 7.0], rtol=1e-15)


def test_choose_step_takes_the_smallest_bound():
    amax = np.array([5.0, 0.0, 3.0])
    vrms = np.array([np.sqrt(13.0), 0.0, 7.0])
    glob = np.array([5.0, 5.0, 7.0])
    # cell ratios: 0.7211 and 2.333 -> min 0.7211; global 1.0 -> max(0.7211, 1.0) = 1.0
    dt = oracle.choose_step(amax, vrms, glob, dlna_max=0.03, hubble=0.01, eta=0.15, cell_width=0.2)
    assert dt == pytest.approx(min(3.0, 0.15 * 1.0, 0.8 * 0.2 / 7.0))
    # a cold cell does not force a tiny step: the global ratio bounds it from below
    vrms2 = vrms.copy()
    vrms2[0] = 1e-6
    dt2 = oracle.choose_step(amax, vrms2, glob, dlna_max=10.0, hubble=1.0, eta=0.3, cell_width=100.0)
    assert dt2 == pytest.approx(0.3 * 1.0)
    # fast particles: the drift bound
    dt3 = oracle.choose_step(amax, vrms, np.array([5.0, 5.0, 70.0]), dlna_max=10.0, hubble=1.0,
                             eta=10.0, cell_width=0.2)
    assert dt3 == pytest.approx(0.8 * 0.2 / 70.0)
