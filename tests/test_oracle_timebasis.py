"""Oracle time basis against the Legendre identities the paper prints."""
import json
import os

import numpy as np
import pytest

from oracle import timebasis as tb

GOLD = os.path.join(os.path.dirname(__file__), "golden", "legendre_time_matrices.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


@pytest.mark.parametrize("dt", [2.0, 0.05, 0.37])
def test_U_is_scaled_orthogonality(dt):
    g = _gold()
    U = tb.overlap_U(g["n_t"], dt)
    np.testing.assert_allclose(U, np.diag(g["U_reference_diag"]) * dt / 2, atol=1e-14 * dt)


@pytest.mark.parametrize("dt", [2.0, 0.05])
def test_Q_pattern(dt):
    g = _gold()
    np.testing.assert_allclose(tb.derivative_Q(g["n_t"], dt), np.array(g["Q"], float), atol=1e-13)


def test_Q_pattern_larger():
    n_t = 9
    Q = tb.derivative_Q(n_t, 0.1)
    ref = np.array([[2.0 if (n > m and (n - m) % 2 == 1) else 0.0 for m in range(n_t)] for n in range(n_t)])
    np.testing.assert_allclose(Q, ref, atol=1e-12)


def test_end_values_and_derivative():
    g = _gold()
    n_t = g["n_t"]
    np.testing.assert_allclose(tb.end_values(n_t), g["P_at_plus_one"], atol=1e-14)
    np.testing.assert_allclose(tb.start_values(n_t), g["P_at_minus_one"], atol=1e-14)
    dp = [tb.legendre_dp(n, 1.0) for n in range(n_t)]
    np.testing.assert_allclose(dp, g["dP_at_plus_one"], atol=1e-12)


def test_field_matrix_constant_field_is_scaled_overlap():
    W = tb.field_matrix(6, 0.3, 0.05, lambda t: 0.7 * np.ones_like(t))
    np.testing.assert_allclose(W, 0.7 * tb.overlap_U(6, 0.05), atol=1e-16)


def test_field_matrix_linear_field_closed_form():
    # E(t) = y (the reference coordinate): int P_n y P_m dy from the three-term
    # recurrence y P_m = ((m+1) P_{m+1} + m P_{m-1}) / (2m+1), times dt/2.
    n_t, t0, dt = 6, 1.0, 0.2
    W = tb.field_matrix(n_t, t0, dt, lambda t: 2.0 * (t - t0) / dt - 1.0)
    ref = np.zeros((n_t, n_t))
    for m in range(n_t):
        for n in range(n_t):
            if n == m + 1:
                ref[n, m] = (m + 1) / (2 * m + 1) * 2 / (2 * n + 1)
            if n == m - 1:
                ref[n, m] = m / (2 * m + 1) * 2 / (2 * n + 1)
    np.testing.assert_allclose(W, ref * dt / 2, atol=1e-15)


def test_pulses():
    f = tb.pulse_sin2_cos(0.05, 0.057, 10.0)
    np.testing.assert_allclose(f(np.array([5.0])), 0.05 * np.cos(0.057 * 5.0), rtol=1e-15)
    assert f(np.array([-1.0, 11.0])).tolist() == [0.0, 0.0]
    g = tb.pulse_fourier_sine([0.1, -0.2], 4.0)
    t = np.array([1.0])
    np.testing.assert_allclose(g(t), 0.1 * np.sin(np.pi / 4) - 0.2 * np.sin(np.pi / 2), rtol=1e-15)
