"""Legendre time basis of one propagation step (oracle, FP64).

Sec. "Review of the Least Action Principle": the wavefunction over one step is
phi(x,t) = sum_{i,n} C_in chi_i(x) T_n(t), and the time matrices are
U_nm = int T_n T_m dt and Q_nm = int T_n' T_m dt over the step.
Sec. "Implementation with Legendre Polynomials": T_n is the Legendre
polynomial P_n mapped from [-1, 1] onto the step [t0, t0 + dt].

Everything here is computed from those definitions by Gauss-Legendre
quadrature (exact for the polynomial integrands), not from the closed forms;
the closed forms the paper prints (orthogonality, the pattern of Q, the end
values P_n(+-1)) are what the tests pin these functions against.

Parity: pinned (tests/test_oracle_timebasis.py).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def _unit(n):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return c


def legendre_p(n, y):
    """P_n(y) for the Legendre polynomial of degree n."""
    return npleg.legval(y, _unit(n))


def legendre_dp(n, y):
    """dP_n/dy."""
    return npleg.legval(y, npleg.legder(_unit(n)))


def _nodes(npts, t0, dt):
    y, w = npleg.leggauss(npts)
    t = t0 + 0.5 * dt * (y + 1.0)
    return y, t, 0.5 * dt * w


def time_functions(n_t, y):
    """Matrix [n, k] = T_n at reference coordinate y_k in [-1, 1]."""
    return np.array([legendre_p(n, y) for n in range(n_t)])


def time_derivatives(n_t, y, dt):
    """Matrix [n, k] = dT_n/dt at y_k (chain rule dy/dt = 2/dt)."""
    return np.array([legendre_dp(n, y) for n in range(n_t)]) * (2.0 / dt)


def overlap_U(n_t, dt):
    """U_nm = int_step T_n(t) T_m(t) dt, by quadrature."""
    y, _, w = _nodes(n_t + 2, 0.0, dt)
    T = time_functions(n_t, y)
    return (T * w) @ T.T


def derivative_Q(n_t, dt):
    """Q_nm = int_step T_n'(t) T_m(t) dt, by quadrature (n: differentiated)."""
    y, _, w = _nodes(n_t + 2, 0.0, dt)
    T = time_functions(n_t, y)
    dT = time_derivatives(n_t, y, dt)
    return (dT * w) @ T.T


def start_values(n_t):
    """s_n = T_n(t0) (the initial-condition row of each multiplier)."""
    return np.array([legendre_p(n, -1.0) for n in range(n_t)])


def end_values(n_t):
    """e_n = T_n(t0 + dt) (evaluation of the step's final wavefunction)."""
    return np.array([legendre_p(n, 1.0) for n in range(n_t)])


def field_matrix(n_t, t0, dt, field, npts=64):
    """W_nm = int_{t0}^{t0+dt} T_n(t) T_m(t) E(t) dt for a smooth E(t).

    This is the time factor of V_ijnm for the dipole term z*E(t)
    (Sec. "Review of the Least Action Principle", definition of V_ijnm).
    """
    y, t, w = _nodes(npts, t0, dt)
    T = time_functions(n_t, y)
    return (T * (w * field(t))) @ T.T


# ---------------------------------------------------------------------------
# Pulses.  The paper's own test uses a constant potential; these are the
# time-dependent dipole fields of the synthetic workloads.
# ---------------------------------------------------------------------------

def pulse_zero():
    return lambda t: np.zeros_like(np.asarray(t, dtype=float))


def pulse_sin2_cos(e0, omega, t_total):
    """E(t) = e0 sin^2(pi t / T) cos(omega t) on [0, T], zero outside."""
    def f(t):
        t = np.asarray(t, dtype=float)
        inside = (t >= 0.0) & (t <= t_total)
        return np.where(inside, e0 * np.sin(np.pi * t / t_total) ** 2 * np.cos(omega * t), 0.0)
    return f


def pulse_fourier_sine(coef, t_total):
    """E(t) = sum_{q=1..Q} a_q sin(q pi t / T) on [0, T], zero outside."""
    coef = np.asarray(coef, dtype=float)

    def f(t):
        t = np.asarray(t, dtype=float)
        inside = (t >= 0.0) & (t <= t_total)
        acc = np.zeros_like(t)
        for q, a in enumerate(coef, start=1):
            acc = acc + a * np.sin(q * np.pi * t / t_total)
        return np.where(inside, acc, 0.0)
    return f


def fourier_basis_function(q, t_total):
    """The q-th (1-based) sine basis function, dE/da_q for the Fourier pulse."""
    def f(t):
        t = np.asarray(t, dtype=float)
        inside = (t >= 0.0) & (t <= t_total)
        return np.where(inside, np.sin(q * np.pi * t / t_total), 0.0)
    return f
