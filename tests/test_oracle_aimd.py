"""Pins of the oracle's AIMD occupation-matrix extrapolation (Sec. II.B)."""
import numpy as np

from oracle import aimd


def _traj(t, R0, v, acc):
    return R0 + v * t + 0.5 * acc * t * t


def test_quadratic_trajectory_gives_second_order_coefficients():
    rng = np.random.default_rng(1)
    R0, v, acc = rng.normal(size=(6, 3)), rng.normal(size=(6, 3)), rng.normal(size=(6, 3))
    hist = [_traj(t, R0, v, acc) for t in (3, 2, 1)]
    a, b = aimd.extrapolation_coefficients(_traj(4, R0, v, acc), hist)
    assert abs(a - 2.0) < 1e-10 and abs(b + 1.0) < 1e-10
    # an occupation matrix quadratic in time is then carried forward exactly
    D0, D1, D2 = rng.normal(size=(3, 5, 5))
    Dt = lambda t: D0 + D1 * t + D2 * t * t
    got = aimd.extrapolate_occupation([Dt(3), Dt(2), Dt(1)], a, b)
    np.testing.assert_allclose(got, Dt(4), atol=1e-10)


def test_linear_trajectory_minimum_norm_and_exact_for_linear_D():
    rng = np.random.default_rng(2)
    R0, v = rng.normal(size=(6, 3)), rng.normal(size=(6, 3))
    hist = [R0 + v * t for t in (3, 2, 1)]
    a, b = aimd.extrapolation_coefficients(R0 + 4 * v, hist)
    assert abs(a - 0.5) < 1e-10 and abs(b - 0.5) < 1e-10
    D0, D1 = rng.normal(size=(2, 5, 5))
    got = aimd.extrapolate_occupation([D0 + D1 * t for t in (3, 2, 1)], a, b)
    np.testing.assert_allclose(got, D0 + 4 * D1, atol=1e-10)


def test_lower_orders_and_atomic_part():
    rng = np.random.default_rng(3)
    R0, v = rng.normal(size=(4, 3)), rng.normal(size=(4, 3))
    # one recorded step: the last D is kept
    assert aimd.extrapolation_coefficients(R0 + v, [R0]) == (0.0, 0.0)
    D = rng.normal(size=(5, 5))
    np.testing.assert_allclose(aimd.extrapolate_occupation([D], 0.0, 0.0), D)
    # two recorded steps of constant velocity: first order with a = 1
    a, b = aimd.extrapolation_coefficients(R0 + 2 * v, [R0 + v, R0])
    assert abs(a - 1.0) < 1e-12 and b == 0.0
    D0, D1 = rng.normal(size=(2, 5, 5))
    np.testing.assert_allclose(aimd.extrapolate_occupation([D0 + D1, D0], a, b), D0 + 2 * D1, atol=1e-12)
    # the isolated-atom part does not depend on time: it cancels
    hist = [rng.normal(size=(5, 5)) for _ in range(3)]
    Dat = 0.2 * np.eye(5)
    np.testing.assert_allclose(aimd.extrapolate_occupation(hist, 0.7, -0.3, Dat),
                               aimd.extrapolate_occupation(hist, 0.7, -0.3), atol=1e-14)
