"""Closed forms of one least-action step for a static Hamiltonian (oracle).

With E(t) = 0 every spatial operator in the step system is the identity or
H = T + diag(V0), and the initial-condition rows are I (x) s^T.  In the
eigenbasis H v_k = E_k v_k the system therefore splits into one scalar
(N_t + 1)-system per eigenvalue,

    M(E) = [[ iQ^T - E U,  s ],      M(E) (a; mu) = (0; 1),
            [ s^T,          0 ]]

and one step maps psi0 to f(H) psi0 with f(E) = sum_n T_n(t0 + dt) a_n(E).
This follows from Eq. (stationaryphase) with the multiplier rows of
Sec. "Review of the Least Action Principle"; it is what the physics tests use
to pin the assembled system from outside (spectral closed form, free plane
waves, norm change, the hand-derived N_t = 2 amplitude).

Parity: pinned (tests/test_oracle_physics.py).
"""
import numpy as np

from . import timebasis as tb


def scalar_system(E, n_t, dt):
    U = tb.overlap_U(n_t, dt)
    Q = tb.derivative_Q(n_t, dt)
    s = tb.start_values(n_t)
    M = np.zeros((n_t + 1, n_t + 1), complex)
    M[:n_t, :n_t] = 1j * Q.T - E * U
    M[:n_t, n_t] = s
    M[n_t, :n_t] = s
    return M


def amplitudes(E, n_t, dt):
    """(a_0..a_{N_t-1}, mu) solving M(E)(a; mu) = (0; 1)."""
    rhs = np.zeros(n_t + 1, complex)
    rhs[n_t] = 1.0
    return np.linalg.solve(scalar_system(E, n_t, dt), rhs)


def amplification(E, n_t, dt):
    """f(E) = psi(t0 + dt) / psi(t0) for an eigenstate of energy E."""
    a = amplitudes(E, n_t, dt)[:n_t]
    return complex(tb.end_values(n_t) @ a)


def amplification_nt2_closed_form(E, dt):
    """Hand-derived N_t = 2 amplitude: (1 + z/3) / (1 - 2z/3), z = -i E dt.

    Rows m = 0, 1 of the scalar system read 2i a_1 - E dt a_0 + mu = 0 and
    -(E dt / 3) a_1 - mu = 0, the constraint a_0 - a_1 = 1; eliminating mu and
    a_0 gives a_1 = E dt / (2i - 4 E dt / 3) and psi = a_0 + a_1 = 1 + 2 a_1.
    """
    z = -1j * E * dt
    return (1.0 + z / 3.0) / (1.0 - 2.0 * z / 3.0)


def spectral_step(H_dense, psi0, n_t, dt):
    """psi(t0 + dt) = V f(Lambda) V^T psi0 for real symmetric H."""
    w, V = np.linalg.eigh(H_dense)
    f = np.array([amplification(E, n_t, dt) for E in w])
    return V @ (f * (V.T @ np.asarray(psi0, complex)))


def norm_change_prediction(H_dense, psi0, n_t, dt):
    """sum_k |<v_k|psi0>|^2 (|f(E_k)|^2 - 1): the exact change of sum |psi|^2."""
    w, V = np.linalg.eigh(H_dense)
    f = np.array([amplification(E, n_t, dt) for E in w])
    p = np.abs(V.T @ np.asarray(psi0, complex)) ** 2
    return float(np.sum(p * (np.abs(f) ** 2 - 1.0)))


def free_plane_wave_energy(k, h, mass=1.0):
    """Eigenvalue of -(1/2m) Lap_h on exp(i k.x): sum_a (1 - cos k_a h)/(m h^2)."""
    k = np.atleast_1d(k)
    return float(np.sum(1.0 - np.cos(k * h)) / (mass * h * h))
