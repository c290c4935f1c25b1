"""Oracle adjoint gradients against central finite differences of the forward."""
import numpy as np

from oracle import adjoint, kkt
from oracle import grid as G
from oracle import timebasis as tb


def _problem():
    g = G.Grid((12, 10), 0.4)
    X, Y = g.coords()
    v0 = (-1.0 / np.sqrt(X ** 2 + Y ** 2 + 1.0)).ravel()
    w, V = np.linalg.eigh(G.hamiltonian(g, v0).toarray())
    gs = V[:, 0] / np.sqrt(np.sum(V[:, 0] ** 2) * g.h ** 2)
    coef = np.array([0.3, -0.2, 0.15])
    return g, v0, gs, coef


def test_pulse_and_potential_gradients_match_central_differences():
    g, v0, gs, coef = _problem()
    n_t, dt, n_steps = 4, 0.1, 4
    T = n_steps * dt
    L, gpsi, dv0, da = adjoint.loss_and_gradients(g, v0, gs, n_t, dt, n_steps, gs, coef, T)
    eps = 1e-5
    for q in range(len(coef)):
        cp, cm = coef.copy(), coef.copy()
        cp[q] += eps
        cm[q] -= eps
        fd = (adjoint.forward_loss(g, v0, gs, n_t, dt, n_steps, gs, cp, T)
              - adjoint.forward_loss(g, v0, gs, n_t, dt, n_steps, gs, cm, T)) / (2 * eps)
        assert abs(fd - da[q]) < 1e-8, (q, fd, da[q])
    for i in [0, 37, 65]:
        vp, vm = v0.copy(), v0.copy()
        vp[i] += eps
        vm[i] -= eps
        fd = (adjoint.forward_loss(g, vp, gs, n_t, dt, n_steps, gs, coef, T)
              - adjoint.forward_loss(g, vm, gs, n_t, dt, n_steps, gs, coef, T)) / (2 * eps)
        assert abs(fd - dv0[i]) < 1e-8, (i, fd, dv0[i])


def test_initial_state_gradient_matches_central_differences():
    g, v0, gs, coef = _problem()
    rng = np.random.default_rng(0)
    psi0 = gs * np.exp(1j * rng.uniform(0, 0.3, g.npts))
    n_t, dt, n_steps = 3, 0.1, 2
    L, gpsi, _, _ = adjoint.loss_and_gradients(g, v0, psi0, n_t, dt, n_steps, gs, coef, 0.2)
    eps = 1e-6
    for i in [3, 50]:
        for direction in [1.0, 1j]:
            pp, pm = psi0.copy(), psi0.copy()
            pp[i] += eps * direction
            pm[i] -= eps * direction
            fd = (adjoint.forward_loss(g, v0, pp, n_t, dt, n_steps, gs, coef, 0.2)
                  - adjoint.forward_loss(g, v0, pm, n_t, dt, n_steps, gs, coef, 0.2)) / (2 * eps)
            # dL = 2 Re(conj(g) dpsi) with g = dL/dpsi^*
            assert abs(fd - 2 * np.real(np.conj(gpsi[i]) * direction)) < 1e-8


def test_adjoint_identity_on_step_system():
    g = G.Grid((6, 4), 0.3)
    rng = np.random.default_rng(2)
    sysm = kkt.StepSystem(g, rng.normal(size=24), 4, 0.05, 0.2, tb.pulse_sin2_cos(0.2, 1.0, 1.0))
    gout = rng.normal(size=24) + 1j * rng.normal(size=24)
    psi0 = rng.normal(size=24) + 1j * rng.normal(size=24)
    x = kkt.solve_direct(sysm.K, kkt.rhs(sysm, psi0))
    mu = adjoint.adjoint_solve(sysm, adjoint.adjoint_rhs(sysm, gout))
    # <g, E x> = <E^H g, x> = <K^H mu, x> = <mu, K x> = <mu, b> = <mu_lambda, psi0>
    lhs = np.vdot(gout, kkt.end_state(sysm, x))
    _, mu_l = kkt.split(mu, 24, 4)
    assert abs(lhs - np.vdot(mu_l, psi0)) < 1e-12 * abs(lhs)
