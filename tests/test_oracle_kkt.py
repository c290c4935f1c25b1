"""Oracle step system: Kronecker assembly pinned by brute force from the action."""
import numpy as np
import pytest

from oracle import bruteforce, kkt
from oracle import grid as G
from oracle import timebasis as tb


CASES = [
    # shape, h, n_t, dt, t0, field, mass, periodic
    ((5,), 0.7, 3, 0.2, 0.0, None, 1.0, False),
    ((3, 2), 0.5, 3, 0.1, 0.4, tb.pulse_sin2_cos(0.3, 1.1, 2.0), 1.0, False),
    ((2, 2, 2), 0.9, 2, 0.3, 0.1, tb.pulse_fourier_sine([0.2, -0.4], 1.0), 1.7, False),
    ((4,), 0.6, 3, 0.15, 0.0, lambda t: 0.5 + t, 1.0, True),
]


@pytest.mark.parametrize("case", CASES)
def test_assembly_matches_action_brute_force(case):
    shape, h, n_t, dt, t0, field, mass, periodic = case
    g = G.Grid(shape, h, periodic=periodic, mass=mass)
    rng = np.random.default_rng(7)
    v0 = rng.normal(size=g.npts)
    sysm = kkt.StepSystem(g, v0, n_t, dt, t0, field)
    Kb = bruteforce.assemble_from_action(shape, h, v0, g.z(), n_t, dt, t0, field, mass, periodic)
    np.testing.assert_allclose(sysm.K.toarray(), Kb, atol=1e-12)


def test_unknown_count():
    g = G.Grid((6, 4), 0.3)
    sysm = kkt.StepSystem(g, np.zeros(g.npts), 5, 0.1)
    assert sysm.K.shape == (g.npts * 6, g.npts * 6)  # N_x (N_t + 1)


def test_initial_guess_meets_initial_condition_rows():
    g = G.Grid((8,), 0.3)
    rng = np.random.default_rng(3)
    psi0 = rng.normal(size=8) + 1j * rng.normal(size=8)
    sysm = kkt.StepSystem(g, rng.normal(size=8), 4, 0.05)
    r = kkt.residual(sysm.K, kkt.rhs(sysm, psi0), kkt.initial_guess(sysm, psi0))
    _, sigma = kkt.split(r, 8, 4)
    assert np.abs(sigma).max() == 0.0


@pytest.mark.parametrize("shape,periodic", [((8,), False), ((6, 5), False), ((4, 4), True), ((3, 4, 2), False)])
def test_initial_guess_norm_closed_form(shape, periodic):
    """Without a field, the initial guess c_j0 = psi_j (other coefficients and
    lambda zero) leaves a residual only on the rows (j, 0), U_00 (H psi)_j: the
    constraint rows vanish and the time couplings see zero coefficients, so
    N0 = U_00^3 |H psi|^2 with H = T + V0 (the closed form the GPU library
    uses for the next step's N0)."""
    g = G.Grid(shape, 0.3, periodic=periodic)
    rng = np.random.default_rng(11)
    v0 = rng.normal(size=g.npts)
    psi0 = rng.normal(size=g.npts) + 1j * rng.normal(size=g.npts)
    n_t, dt = 5, 0.07
    sysm = kkt.StepSystem(g, v0, n_t, dt)
    r = kkt.residual(sysm.K, kkt.rhs(sysm, psi0), kkt.initial_guess(sysm, psi0))
    rho, sigma = kkt.split(r, g.npts, n_t)
    hpsi = G.hamiltonian(g, v0) @ psi0
    assert np.abs(sigma).max() == 0.0
    assert np.abs(rho[:, 1:]).max() <= 1e-12 * np.abs(hpsi).max()
    np.testing.assert_allclose(rho[:, 0], dt * hpsi, rtol=0, atol=1e-12 * np.abs(hpsi).max())
    n0 = kkt.residual_norm(sysm, r)
    assert abs(n0 - dt ** 3 * np.sum(np.abs(hpsi) ** 2)) <= 1e-12 * n0


def test_residual_norm_weights():
    g = G.Grid((2,), 1.0)
    sysm = kkt.StepSystem(g, np.zeros(2), 2, 0.3)
    r = kkt.join(np.array([[1.0, 2.0], [0.0, 1j]]), np.array([3.0, 0.5]))
    # U = diag(0.3, 0.1): 0.3*1 + 0.1*4 + 0.1*1 + 9 + 0.25
    assert abs(kkt.residual_norm(sysm, r) - (0.3 + 0.4 + 0.1 + 9.25)) < 1e-14


def test_direct_solution_solves_system_sparse_and_dense():
    for shape in [(16,), (48, 48)]:
        g = G.Grid(shape, 0.2)
        rng = np.random.default_rng(1)
        v0 = rng.normal(size=g.npts)
        psi0 = rng.normal(size=g.npts) + 1j * rng.normal(size=g.npts)
        sysm = kkt.StepSystem(g, v0, 4, 0.05)
        b = kkt.rhs(sysm, psi0)
        x = kkt.solve_direct(sysm.K, b)
        assert np.abs(sysm.K @ x - b).max() < 1e-12
