"""Time-step splitting through the C ABI against the oracle's direct sub-steps.

Sec. "Implementation with Legendre Polynomials" (after Eq.
(leastaction_dimensionless)): a step can be done as two steps of half the
length, which halves kappa = p_max^2 dt / 2 and nu = V dt.  With max_split > 0
the library abandons a solve whose residual grows and redoes the step as
halves.  The expected values are the oracle's direct solves of the sub-steps
(dt / 2^d each, 2^d of them per step); the depth d the library chose is
checked against the regime: the oracle's V-cycles diverge at dt = 0.5 and 0.25
and converge at 0.125 for the 1D case (pinned in test_oracle_relax.py).
"""
import numpy as np
import pytest

from gpu_util import Case, n, note, t_c, t_r
from oracle import adjoint as A
from oracle import kkt

pytestmark = pytest.mark.gpu

H1 = 40.0 / 256
PULSE = dict(kind="fourier", t_total=2.0, coef=[0.02, -0.01, 0.015])


def case_1d(pulse=None, n_pts=256):
    # kappa = dt / (2 h^2) = 10.2 at dt = 0.5: relaxation diverges; 2.56 after two halvings
    return Case(shape=(n_pts,), h=H1, n_t=8, dt=0.5, block=(8,), levels=3, potential="harmonic", pulse=pulse,
                field_axis=0 if pulse else -1)


def prop_of(case, precision, max_split, tol=None):
    # FP64 solves to 1e-12, the mixed path to 1e-10 as in its other parity tests (a
    # tolerance below what its refinement reaches would count as not converging)
    if tol is None:
        tol = 1e-12 if precision == "fp64" else 1e-10
    return case.prop(precision=precision, tol=tol, max_cycles=60, nu_coarse=4, coarse_reduction=1e-3,
                     max_split=max_split)


def bound(precision, substeps, n_t, scale):
    # each sub-step's coefficients to 1e-10 (FP64) / 1e-8 (mixed) of their size, as in
    # the single-step parity; psi sums n_t of them, and the errors add over sub-steps
    return substeps * n_t * (1e-10 if precision == "fp64" else 1e-8) * scale


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_step_matches_the_oracle_sub_steps(precision):
    case = case_1d()
    note(f"split step {precision} {case} dt={case.dt}")
    prop = prop_of(case, precision, max_split=3)
    psi, st = prop.solve_step(0.0, t_c(case.psi0))
    note(f"depth={st['split_depth']} substeps={st['substeps']} cycles={st['cycles']}")
    assert st["split_depth"] == 2 and st["substeps"] == 4
    psis = kkt.propagate(case.grid, case.v0, case.psi0, case.n_t, case.dt / 4, 4)
    ref = psis[-1]
    err = np.abs(n(psi) - ref).max()
    note(f"max |psi - psi_oracle| = {err:.2e}")
    assert err <= bound(precision, 4, case.n_t, np.abs(ref).max())
    # the state left in the context is the last sub-step's, at its own step length
    c, _ = prop.get_state()
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt / 4, 0.75 * case.dt, None)
    x = kkt.solve_direct(sysm.K, kkt.rhs(sysm, psis[-2]))
    c_ref, _ = kkt.split(x, case.npts, case.n_t)
    assert np.abs(n(c).reshape(-1, case.n_t) - c_ref).max() <= bound(precision, 4, 1, np.abs(c_ref).max())
    prop.close()


def test_too_few_halvings_still_fail():
    """One halving leaves kappa = 5.1, still divergent: the step is reported, not
    silently accepted; without splitting the behaviour is that of the plain solve."""
    from paper_1111_4363_amd import lam
    case = case_1d()
    for ms in (0, 1):
        note(f"max_split={ms}")
        prop = prop_of(case, "fp64", max_split=ms, tol=1e-10)
        with pytest.raises(lam.LamError) as e:
            prop.solve_step(0.0, t_c(case.psi0))
        assert e.value.code in (lam.LAM_EDIVERGED, lam.LAM_ENOCONV)
        prop.close()


def test_in_regime_step_is_not_split():
    case = Case(shape=(256,), h=H1, n_t=8, dt=0.1, block=(8,), levels=3, potential="harmonic")
    note("in-regime step, max_split=3")
    prop = prop_of(case, "fp64", max_split=3)
    psi, st = prop.solve_step(0.0, t_c(case.psi0))
    assert st["split_depth"] == 0 and st["substeps"] == 1
    ref = kkt.propagate(case.grid, case.v0, case.psi0, case.n_t, case.dt, 1)[-1]
    assert np.abs(n(psi) - ref).max() <= bound("fp64", 1, case.n_t, np.abs(ref).max())
    prop.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_propagation_with_a_field_matches_the_oracle(precision):
    """Three steps through lam_propagate (the step-ahead pipeline; each step's
    failed solve is redone as halves from its initial state), with a Fourier
    pulse along x: against twelve direct sub-steps of dt / 4."""
    case = case_1d(PULSE)
    note(f"split propagate {precision} {case}")
    prop = prop_of(case, precision, max_split=3)
    psi, st = prop.propagate(t_c(case.psi0), 3)
    st = st[0]
    note(f"depth={st['split_depth']} substeps={st['substeps']} cycles={st['cycles']}")
    assert st["split_depth"] == 2 and st["substeps"] == 12
    ref = kkt.propagate(case.grid, case.v0, case.psi0, case.n_t, case.dt / 4, 12, case.field)[-1]
    err = np.abs(n(psi) - ref).max()
    note(f"max |psi - psi_oracle| = {err:.2e}")
    assert err <= bound(precision, 12, case.n_t, np.abs(ref).max())
    prop.close()


def test_split_2d_step_takes_three_halvings():
    """2D, 64^2, h = 0.2, N_t = 6, 8 x 8 subvolumes, two levels, dt = 0.8 (kappa = 10):
    the V-cycles grow at dt = 0.4 and 0.2 and converge at 0.1, so the step becomes
    eight sub-steps; mixed precision against the oracle's eight direct sub-steps."""
    case = Case(shape=(64, 64), h=0.2, n_t=6, dt=0.8, block=(8, 8), levels=2)
    note(f"split 2D step {case}")
    prop = prop_of(case, "mixed", max_split=4)
    psi, st = prop.solve_step(0.0, t_c(case.psi0))
    note(f"depth={st['split_depth']} substeps={st['substeps']} cycles={st['cycles']}")
    assert st["split_depth"] == 3 and st["substeps"] == 8
    ref = kkt.propagate(case.grid, case.v0, case.psi0, case.n_t, case.dt / 8, 8)[-1]
    assert np.abs(n(psi) - ref).max() <= bound("mixed", 8, case.n_t, np.abs(ref).max())
    prop.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_adjoint_matches_the_oracle(precision):
    """Two split steps through the autograd function (forward lam_propagate,
    backward lam_adjoint_step, whose forward recomputation splits the same way):
    the loss, dL/dpsi0^*, dL/dV0 and dL/da against the oracle's direct forward and
    adjoint solves of eight sub-steps of dt / 4, relative to each gradient's largest
    entry."""
    import torch
    from paper_1111_4363_amd import lam
    case = case_1d(PULSE, n_pts=128)
    note(f"split adjoint {precision} {case}")
    g = case.psi0 / np.sqrt(np.sum(np.abs(case.psi0) ** 2) * case.h)
    coef = np.array(PULSE["coef"])
    L_ref, g0_ref, dv_ref, da_ref = A.loss_and_gradients(case.grid, case.v0, case.psi0, case.n_t, case.dt / 4, 8, g,
                                                         list(coef), PULSE["t_total"])
    prop = prop_of(case, precision, max_split=3)
    g_t = t_c(g)
    psi0 = t_c(case.psi0).requires_grad_(True)
    v0_t = t_r(case.v0).requires_grad_(True)
    cf = torch.tensor(coef, dtype=torch.float64, requires_grad=True)
    psiK = lam.propagate_differentiable(prop, psi0, v0_t, cf, 2)
    ov = case.h * torch.sum(torch.conj(g_t) * psiK)
    L = (ov * torch.conj(ov)).real
    L.backward()
    tol = 1e-9 if precision == "fp64" else 1e-7
    note(f"L={float(L):.12f} oracle {L_ref:.12f}")
    assert abs(float(L) - L_ref) <= tol
    g0 = 0.5 * n(psi0.grad)
    assert np.abs(g0 - g0_ref).max() <= tol * np.abs(g0_ref).max()
    assert np.abs(n(v0_t.grad) - dv_ref).max() <= tol * np.abs(dv_ref).max()
    assert np.abs(cf.grad.numpy() - da_ref).max() <= tol * np.abs(da_ref).max()
    prop.close()
