"""Brute-force assembly of the step system from the action (tiny cases only).

The step system's entries are the coefficients of the sesquilinear action of
Sec. "Review of the Least Action Principle",

    S' = sum_j int dt phi_j(t)^* [ i d/dt - H0 - V(x_j, t) ] phi_j(t)
         + sum_j lambda_j f_j^*,   f_j = phi_j(t0) - psi0_j,

so entry (row (j, m), column (i, n)) of K is S evaluated with the trial
function chi_i T_n and the test function chi_j T_m, the multiplier column of
row (j, m) is T_m(t0)^*, and the constraint row j is phi_j(t0).

This module evaluates exactly that, term by term, with its own Legendre
recurrence (Bonnet), its own derivative recurrence, a high-order time
quadrature and a neighbour loop for the Laplacian; it never touches U, Q, s
or the Kronecker assembly, which is what it is compared against.

Parity: this *is* a pin for kkt.assemble (tests/test_oracle_kkt.py).
"""
import itertools

import numpy as np


def _legendre_all(n_t, y):
    """Bonnet recurrence: (n+1) P_{n+1} = (2n+1) y P_n - n P_{n-1}."""
    y = np.asarray(y, dtype=float)
    P = [np.ones_like(y), y.copy()]
    for n in range(1, n_t):
        P.append(((2 * n + 1) * y * P[n] - n * P[n - 1]) / (n + 1))
    return np.array(P[:n_t])


def _legendre_deriv_all(n_t, y):
    """P'_{n+1} = P'_{n-1} + (2n+1) P_n, P'_0 = 0, P'_1 = 1."""
    y = np.asarray(y, dtype=float)
    P = _legendre_all(n_t + 1, y)
    D = [np.zeros_like(y), np.ones_like(y)]
    for n in range(1, n_t):
        D.append(D[n - 1] + (2 * n + 1) * P[n])
    return np.array(D[:n_t])


def _apply_kinetic(u, shape, h, mass, periodic):
    """-(1/2m) sum_axes (u[+e] - 2u + u[-e]) / h^2 by explicit neighbour loops."""
    u = np.asarray(u).reshape(shape)
    out = np.zeros_like(u)
    d = len(shape)
    for idx in itertools.product(*[range(n) for n in shape]):
        acc = 0.0
        for a in range(d):
            for step in (-1, 1):
                nb = list(idx)
                nb[a] += step
                if periodic:
                    nb[a] %= shape[a]
                    acc += u[tuple(nb)]
                elif 0 <= nb[a] < shape[a]:
                    acc += u[tuple(nb)]
            acc -= 2.0 * u[idx]
        out[idx] = -0.5 / mass * acc / (h * h)
    return out.ravel()


def assemble_from_action(shape, h, v0, z, n_t, dt, t0, field, mass=1.0,
                         periodic=False, nquad=40):
    """Dense K built entry by entry from the action (see module docstring)."""
    shape = tuple(shape)
    P = int(np.prod(shape))
    v0 = np.asarray(v0, float).ravel()
    z = np.asarray(z, float).ravel()
    y, w = np.polynomial.legendre.leggauss(nquad)
    t = t0 + 0.5 * dt * (y + 1.0)
    wt = 0.5 * dt * w
    Tv = _legendre_all(n_t, y)                       # T_n(t_k)
    Td = _legendre_deriv_all(n_t, y) * (2.0 / dt)    # dT_n/dt at t_k
    T0 = _legendre_all(n_t, np.array([-1.0]))[:, 0]  # T_n(t0)
    E = np.zeros_like(t) if field is None else field(t)

    nunk = P * (n_t + 1)
    K = np.zeros((nunk, nunk), complex)
    for i in range(P):
        chi_i = np.zeros(P)
        chi_i[i] = 1.0
        Hchi = _apply_kinetic(chi_i, shape, h, mass, periodic)
        for n in range(n_t):
            col = i * n_t + n
            # L applied to the trial function chi_i T_n, sampled in time:
            # i chi_i T_n' - (T chi_i) T_n - V(x, t) chi_i T_n
            for j in range(P):
                Lu = (1j * (j == i) * Td[n]
                      - Hchi[j] * Tv[n]
                      - (j == i) * (v0[j] + z[j] * E) * Tv[n])
                if not np.any(Lu):
                    continue
                for m in range(n_t):
                    K[j * n_t + m, col] = np.sum(wt * np.conj(Tv[m]) * Lu)
    for j in range(P):
        for m in range(n_t):
            K[j * n_t + m, P * n_t + j] = np.conj(T0[m])
        for n in range(n_t):
            K[P * n_t + j, j * n_t + n] = T0[n]
    return K
