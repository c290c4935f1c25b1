"""Adjoint of the step system and loss gradients (oracle, direct solves).

For one step K x = b(psi_k), psi_{k+1} = E x with (E x)_j = sum_n T_n(t0+dt) c_jn.
For a real loss L and g_{k+1} = dL/dpsi_{k+1}^* (Wirtinger convention, so that
dL = 2 Re <g, dpsi>):

* the adjoint solve is K^H mu = E^H g_{k+1};
* dL/dpsi_k^* = mu on the constraint rows (b depends on psi_k only there);
* for a real parameter theta of K, dL/dtheta = -2 Re( mu^H (dK/dtheta) x ).

The entries of K that depend on V0_i are -U_mn on rows (i, m), columns (i, n);
the dipole entries are -z_j W_mn with W linear in E(t), so a pulse
E(t) = sum_q a_q f_q(t) gives dK/da_q = -Z (x) W^(q), W^(q) = int T_n T_m f_q.

The loss of the workloads is the population of a reference state g after the
last step, L = |<g|psi_K>|^2 with <g|psi> = w sum_j g_j^* psi_j and the grid
quadrature weight w = h^d.

Parity: pinned by the dot-product identity and by central finite differences
of the oracle's own forward propagation (tests/test_oracle_adjoint.py).
"""
import numpy as np

from . import kkt
from . import timebasis as tb


def overlap(grid, g, psi):
    return grid.h ** grid.dim * np.vdot(np.asarray(g).ravel(), np.asarray(psi).ravel())


def population_loss(grid, g, psi):
    return float(abs(overlap(grid, g, psi)) ** 2)


def population_loss_grad(grid, g, psi):
    """dL/dpsi^* for L = |<g|psi>|^2."""
    return grid.h ** grid.dim * np.asarray(g, complex).ravel() * overlap(grid, g, psi)


def adjoint_rhs(system, g_out):
    """E^H g: g_j on every stationarity row (j, n) weighted by T_n(t0+dt)."""
    P, n_t = system.npts, system.n_t
    top = np.outer(np.asarray(g_out, complex).ravel(), system.e).ravel()
    return np.concatenate([top, np.zeros(P, complex)])


def adjoint_solve(system, rhs_vec):
    return kkt.solve_direct(system.K.conj().T.tocsr(), rhs_vec)


def step_gradients(system, x, mu, pulse_basis=()):
    """(dL/dpsi_k^*, dL/dV0, [dL/da_q]) from the forward x and adjoint mu."""
    P, n_t = system.npts, system.n_t
    c, _ = kkt.split(x, P, n_t)
    mu_c, mu_l = kkt.split(mu, P, n_t)
    dv0 = 2.0 * np.einsum("jm,mn,jn->j", mu_c.conj(), system.U, c).real
    z = system.grid.z()
    da = []
    for f in pulse_basis:
        Wq = tb.field_matrix(n_t, system.t0, system.dt, f)
        da.append(2.0 * np.real(np.einsum("j,jm,mn,jn->", z, mu_c.conj(), Wq, c)))
    return mu_l.copy(), dv0, np.array(da)


def loss_and_gradients(grid, v0, psi0, n_t, dt, n_steps, g, coef, t_total):
    """Forward direct steps with E(t) = sum a_q sin(q pi t/T), then backward.

    Returns (L, dL/dpsi0^*, dL/dV0, dL/da).
    """
    field = tb.pulse_fourier_sine(coef, t_total)
    basis = [tb.fourier_basis_function(q, t_total) for q in range(1, len(coef) + 1)]
    psis = [np.asarray(psi0, complex).ravel()]
    for k in range(n_steps):
        psi, _, _ = kkt.step(grid, v0, psis[-1], n_t, dt, k * dt, field)
        psis.append(psi)
    L = population_loss(grid, g, psis[-1])
    gk = population_loss_grad(grid, g, psis[-1])
    dv0 = np.zeros(grid.npts)
    da = np.zeros(len(coef))
    for k in reversed(range(n_steps)):
        sysm = kkt.StepSystem(grid, v0, n_t, dt, k * dt, field)
        x = kkt.solve_direct(sysm.K, kkt.rhs(sysm, psis[k]))
        mu = adjoint_solve(sysm, adjoint_rhs(sysm, gk))
        gk, dv, dq = step_gradients(sysm, x, mu, basis)
        dv0 += dv
        da += dq
    return L, gk, dv0, da


def forward_loss(grid, v0, psi0, n_t, dt, n_steps, g, coef, t_total):
    field = tb.pulse_fourier_sine(coef, t_total)
    psis = kkt.propagate(grid, v0, psi0, n_t, dt, n_steps, field)
    return population_loss(grid, g, psis[-1])
