"""Oracle step against closed forms and physics the method fixes.

Each test checks the step's definition from outside: identities derived by
hand from the stationarity and constraint rows, the spectral decomposition of
a static Hamiltonian, free plane waves, the exact propagator exp(-iH dt) as
N_t grows, and the field term against an equivalent static potential.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import kkt, spectral
from oracle import grid as G
from oracle import timebasis as tb


def _gauss_1d(g, x0=-5.0, k0=1.0, sigma=1.0):
    x = g.coords()[0].ravel()
    psi = np.exp(-(x - x0) ** 2 / (2 * sigma ** 2) + 1j * k0 * x)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * g.h)


def test_single_time_function_keeps_psi_and_sets_lambda():
    # N_t = 1: constraint c_j0 = psi0_j; row m=0: -dt (H c)_j + lambda_j = 0.
    g = G.Grid((20,), 0.3)
    rng = np.random.default_rng(2)
    v0 = rng.normal(size=20)
    psi0 = rng.normal(size=20) + 1j * rng.normal(size=20)
    psi1, x, sysm = kkt.step(g, v0, psi0, 1, 0.07)
    np.testing.assert_allclose(psi1, psi0, atol=1e-14)
    _, lam = kkt.split(x, 20, 1)
    np.testing.assert_allclose(lam, 0.07 * (G.hamiltonian(g, v0) @ psi0), atol=1e-13)


def test_two_time_functions_hand_derived_amplitude_on_eigenstates():
    g = G.Grid((30,), 0.4)
    x = g.coords()[0].ravel()
    v0 = 0.5 * x ** 2
    H = G.hamiltonian(g, v0).toarray()
    w, V = np.linalg.eigh(H)
    for k in [0, 5, 29]:
        psi1, _, _ = kkt.step(g, v0, V[:, k], 2, 0.05)
        np.testing.assert_allclose(psi1, spectral.amplification_nt2_closed_form(w[k], 0.05) * V[:, k],
                                   atol=1e-13)


def test_scalar_system_zero_energy_mode():
    for n_t in [1, 3, 8]:
        a = spectral.amplitudes(0.0, n_t, 0.05)
        ref = np.zeros(n_t + 1)
        ref[0] = 1.0
        np.testing.assert_allclose(a, ref, atol=1e-13)


@pytest.mark.parametrize("shape,h,n_t", [((40,), 0.5, 8), ((8, 6), 0.3, 6)])
def test_spectral_closed_form(shape, h, n_t):
    g = G.Grid(shape, h)
    r2 = sum(c ** 2 for c in g.coords()).ravel()
    v0 = -1.0 / np.sqrt(r2 + 1.0)
    rng = np.random.default_rng(5)
    psi0 = rng.normal(size=g.npts) + 1j * rng.normal(size=g.npts)
    psi1, _, _ = kkt.step(g, v0, psi0, n_t, 0.05)
    ref = spectral.spectral_step(G.hamiltonian(g, v0).toarray(), psi0, n_t, 0.05)
    np.testing.assert_allclose(psi1, ref, atol=1e-13 * np.abs(psi0).max())


def test_last_stationarity_row_fixes_lambda_without_field():
    g = G.Grid((24,), 0.3)
    rng = np.random.default_rng(9)
    v0 = rng.normal(size=24)
    psi0 = rng.normal(size=24) + 1j * rng.normal(size=24)
    n_t, dt = 5, 0.05
    _, x, sysm = kkt.step(g, v0, psi0, n_t, dt)
    c, lam = kkt.split(x, 24, n_t)
    m = n_t - 1
    Hc = G.hamiltonian(g, v0) @ c[:, m]
    np.testing.assert_allclose(lam, (dt / (2 * m + 1)) * Hc / (-1) ** m, atol=1e-13)


def test_converges_to_exact_propagator_as_time_basis_grows():
    g = G.Grid((256,), 40.0 / 256)
    x = g.coords()[0].ravel()
    v0 = 0.5 * x ** 2
    psi0 = _gauss_1d(g)
    H = G.hamiltonian(g, v0).toarray()
    exact = sla.expm(-1j * 0.05 * H) @ psi0
    errs = []
    for n_t in [2, 4, 6, 8]:
        psi1, _, _ = kkt.step(g, v0, psi0, n_t, 0.05)
        errs.append(np.abs(psi1 - exact).max())
    assert all(b < a / 10 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-8


def test_periodic_free_plane_wave():
    g = G.Grid((32,), 0.25, periodic=True)
    x = g.coords()[0].ravel()
    for mode in [1, 5, 11]:
        k = 2 * np.pi * mode / (32 * 0.25)
        psi0 = np.exp(1j * k * x)
        Ek = spectral.free_plane_wave_energy(k, 0.25)
        psi1, _, _ = kkt.step(g, np.zeros(32), psi0, 2, 0.05)
        np.testing.assert_allclose(psi1, spectral.amplification_nt2_closed_form(Ek, 0.05) * psi0, atol=1e-13)
        psi8, _, _ = kkt.step(g, np.zeros(32), psi0, 8, 0.05)
        np.testing.assert_allclose(psi8, np.exp(-1j * Ek * 0.05) * psi0, atol=1e-9)


def test_norm_change_matches_spectral_prediction():
    g = G.Grid((40,), 0.2)
    x = g.coords()[0].ravel()
    v0 = -1.0 / np.sqrt(x ** 2 + 1.0)
    rng = np.random.default_rng(11)
    psi0 = rng.normal(size=40) + 1j * rng.normal(size=40)
    H = G.hamiltonian(g, v0).toarray()
    for n_t in [2, 8]:
        psi1, _, _ = kkt.step(g, v0, psi0, n_t, 0.05)
        drift = np.sum(np.abs(psi1) ** 2) - np.sum(np.abs(psi0) ** 2)
        pred = spectral.norm_change_prediction(H, psi0, n_t, 0.05)
        assert abs(drift - pred) < 1e-12 * np.sum(np.abs(psi0) ** 2)


def test_constant_field_equals_shifted_static_potential():
    g = G.Grid((6, 8), 0.35)
    rng = np.random.default_rng(4)
    v0 = rng.normal(size=g.npts)
    psi0 = rng.normal(size=g.npts) + 1j * rng.normal(size=g.npts)
    E0 = 0.37
    with_field, _, _ = kkt.step(g, v0, psi0, 6, 0.05, 0.3, lambda t: E0 * np.ones_like(t))
    shifted, _, _ = kkt.step(g, v0 + E0 * g.z(), psi0, 6, 0.05)
    np.testing.assert_allclose(with_field, shifted, atol=1e-13)
