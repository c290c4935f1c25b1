"""Degenerate and failure cases on the GPU (all kernels exit normally)."""
import numpy as np
import pytest

from gpu_util import Case, n, note, t_c
from oracle import grid as G
from oracle import kkt

pytestmark = pytest.mark.gpu


def test_single_time_function_keeps_psi():
    case = Case(shape=(16, 16), h=0.25, n_t=1, block=(4, 4), levels=2)
    note(f"n_t=1 {case}")
    prop = case.prop(tol=1e-13, max_cycles=40)
    psi_out, st = prop.solve_step(0.0, t_c(case.psi0))
    np.testing.assert_allclose(n(psi_out), case.psi0, atol=1e-14)
    _, lam_ = prop.get_state()
    Hpsi = G.hamiltonian(case.grid, case.v0) @ case.psi0
    assert np.abs(n(lam_) - case.dt * Hpsi).max() <= 1e-11 * np.abs(case.dt * Hpsi).max()
    prop.close()


def test_whole_grid_block_is_direct_solve_in_one_sweep():
    case = Case(shape=(8, 8), h=0.3, n_t=6, block=(8, 8), levels=1)
    note(f"one block {case}")
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt)
    x_ref = kkt.solve_direct(sysm.K, kkt.rhs(sysm, case.psi0))
    prop = case.prop()
    c0 = np.zeros((case.npts, case.n_t), complex)
    c0[:, 0] = case.psi0
    prop.set_state(0.0, t_c(case.psi0), t_c(c0), t_c(np.zeros(case.npts)))
    prop.relax_sweep(0)
    cg, lg = prop.get_state()
    x = np.concatenate([n(cg), n(lg)])
    assert np.abs(x - x_ref).max() <= 1e-12 * np.abs(x_ref).max()
    prop.close()


def test_single_point_blocks():
    case = Case(shape=(8, 6), h=0.3, n_t=4, block=(1, 1), levels=1)
    note(f"1-point blocks {case}")
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt)
    x_ref = kkt.solve_direct(sysm.K, kkt.rhs(sysm, case.psi0))
    prop = case.prop(tol=1e-12, max_cycles=200, nu_coarse=1)
    prop.solve_step(0.0, t_c(case.psi0))
    cg, _ = prop.get_state()
    c_ref, _ = kkt.split(x_ref, case.npts, case.n_t)
    assert np.abs(n(cg).reshape(-1, case.n_t) - c_ref).max() <= 1e-10 * np.abs(c_ref).max()
    prop.close()


def test_zero_wavefunction_returns_zero_without_cycles():
    case = Case(shape=(16,), h=0.25, n_t=4, block=(4,), levels=2)
    prop = case.prop()
    psi_out, st = prop.solve_step(0.0, t_c(np.zeros(16)))
    assert st["cycles"] == 0 and np.all(n(psi_out) == 0)
    prop.close()


def test_nan_input_reports_divergence():
    from paper_1111_4363_amd import lam
    case = Case(shape=(16, 16), h=0.25, n_t=4, block=(4, 4), levels=2)
    psi = case.psi0.copy()
    psi[17] = np.nan
    prop = case.prop()
    with pytest.raises(lam.LamError) as e:
        prop.solve_step(0.0, t_c(psi))
    assert e.value.code == lam.LAM_EDIVERGED
    prop.close()


def test_cycle_cap_reports_no_convergence_but_writes_output():
    from paper_1111_4363_amd import lam
    case = Case(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2)
    prop = case.prop(tol=1e-14, max_cycles=1)
    with pytest.raises(lam.NotConverged):
        prop.solve_step(0.0, t_c(case.psi0))
    psi_out, st = prop.solve_step(0.0, t_c(case.psi0), allow_noconv=True)
    assert st["cycles"] == 1 and np.isfinite(n(psi_out)).all()
    prop.close()


def test_out_of_regime_step_is_flagged():
    """kappa = dt/(2h^2) ~ 10 (1D, dt = 0.5): the paper's caveat that relaxation
    need not converge; the watchdog reports divergence or non-convergence."""
    from paper_1111_4363_amd import lam
    case = Case(shape=(256,), h=40 / 256, n_t=8, dt=0.5, block=(8,), levels=1, potential="harmonic")
    prop = case.prop(tol=1e-10, max_cycles=30, nu_coarse=2)
    with pytest.raises(lam.LamError) as e:
        prop.solve_step(0.0, t_c(case.psi0))
    assert e.value.code in (lam.LAM_EDIVERGED, lam.LAM_ENOCONV)
    prop.close()
