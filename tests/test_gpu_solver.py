"""GPU V-cycles, step solves and adjoint steps against the oracle.

V-cycle: one cycle from a random state against the oracle's reference
V-cycle with the same sweep counts, transfers and coarse operators; agreement
to 1e-10 of the state (dozens of local solves, each good to ~1e-13).
Step solve: coefficients against the oracle's direct solve, relative error
<= 1e-10 (FP64 path) and <= 1e-8 (mixed path), the target accuracies.
Adjoint step: the adjoint solution and the gradients against the oracle's
direct K^H solve.
"""
import numpy as np
import pytest

from gpu_util import EXACT_INNER_TOL, Case, n, note, t_c, t_r
from oracle import adjoint as A
from oracle import kkt, relax

pytestmark = pytest.mark.gpu

PULSE_SIN2 = dict(kind="sin2", e0=0.05, omega=0.057, t_total=1.0)
PULSE_FOURIER = dict(kind="fourier", t_total=0.4, coef=[0.03, -0.02, 0.05])


@pytest.mark.parametrize("cfg", [
    dict(shape=(32, 32), n_t=4, block=(4, 4), levels=3, h=0.2),
    dict(shape=(32, 16), n_t=6, block=(4, 4), levels=2, h=0.2, pulse=PULSE_SIN2, interp="constant"),
    dict(shape=(64,), n_t=8, block=(8,), levels=3, h=0.3, potential="harmonic"),
    dict(shape=(8, 8, 16), n_t=3, block=(2, 2, 2), levels=2, h=0.3),
    # ragged tiles of the fused residual-restriction (32 fine points: 2 x 16 in 2D,
    # 2 x 2 x 8 in 3D, 32 in 1D), with a field and the constant interpolation
    dict(shape=(16, 24), n_t=4, block=(4, 4), levels=2, h=0.2, pulse=PULSE_FOURIER),
    dict(shape=(8, 8, 12), n_t=3, block=(2, 2, 2), levels=2, h=0.3, interp="constant"),
    dict(shape=(40,), n_t=5, block=(4,), levels=2, h=0.3, potential="random"),
    # the residual-restriction that marches along x, periodic, with a field
    dict(shape=(8, 16, 16), n_t=8, block=(2, 2, 2), levels=2, h=0.3, periodic=True, pulse=PULSE_FOURIER),
], ids=lambda c: f"{c['shape']}-L{c['levels']}")
@pytest.mark.parametrize("adjoint", [False, True])
def test_vcycle_parity(cfg, adjoint):
    case = Case(**cfg)
    note(f"vcycle adjoint={adjoint} {case}")
    t0 = 0.1
    H = relax.build_hierarchy(case.grid, case.v0, case.n_t, case.dt, case.block, case.levels, t0=t0,
                              field=case.field, interp=case.interp)
    sysm = H[0].system
    c, lam = case.random_state(0.1)
    x = kkt.join(c, lam)
    prop = case.prop(nu_pre=1, nu_post=1, nu_coarse=2, n_inner=(8 if case.field else -1))
    if adjoint:
        b = A.adjoint_rhs(sysm, case.psi0)
        prop.set_adjoint_state(t0, t_c(case.psi0), t_c(c), t_c(lam))
    else:
        b = kkt.rhs(sysm, case.psi0)
        prop.set_state(t0, t_c(case.psi0), t_c(c), t_c(lam))
    x_ref = relax.reference_vcycle(H, 0, x, b, 1, 1, 2, adjoint=adjoint)
    N = prop.vcycle()
    cg, lg = prop.get_state()
    x_gpu = np.concatenate([n(cg), n(lg)])
    err = np.abs(x_gpu - x_ref).max()
    assert err <= 1e-10 * np.abs(x_ref).max(), err
    K = sysm.K.conj().T if adjoint else sysm.K
    N_ref = kkt.residual_norm(sysm, b - K @ x_ref)
    assert abs(N - N_ref) <= 1e-6 * N_ref + 1e-26
    prop.close()


@pytest.mark.parametrize("cfg", [
    dict(shape=(32, 32), n_t=4, block=(4, 4), levels=3, h=0.2),
    dict(shape=(8, 8, 16), n_t=6, block=(2, 2, 2), levels=2, h=0.3, pulse=PULSE_SIN2),
    dict(shape=(64,), n_t=8, block=(8,), levels=1, h=0.3, potential="harmonic"),
], ids=lambda c: f"{c['shape']}-L{c['levels']}")
@pytest.mark.parametrize("adjoint", [False, True])
def test_vcycle_parity_iterated_coarsest_solve(cfg, adjoint):
    """The coarsest solve iterated on the device until its residual fell by 1e3
    (at most 6 sweeps) against the oracle's V-cycle with the same rule; on one
    level the 'coarsest' level is the fine grid itself."""
    case = Case(**cfg)
    note(f"vcycle iterated coarsest adjoint={adjoint} {case}")
    t0 = 0.1
    H = relax.build_hierarchy(case.grid, case.v0, case.n_t, case.dt, case.block, case.levels, t0=t0,
                              field=case.field, interp=case.interp)
    sysm = H[0].system
    c, lam = case.random_state(0.1)
    x = kkt.join(c, lam)
    prop = case.prop(nu_pre=1, nu_post=1, nu_coarse=6, coarse_reduction=1e-3, n_inner=(8 if case.field else -1))
    if adjoint:
        b = A.adjoint_rhs(sysm, case.psi0)
        prop.set_adjoint_state(t0, t_c(case.psi0), t_c(c), t_c(lam))
    else:
        b = kkt.rhs(sysm, case.psi0)
        prop.set_state(t0, t_c(case.psi0), t_c(c), t_c(lam))
    counts = []
    x_ref = relax.reference_vcycle(H, 0, x, b, 1, 1, 6, adjoint=adjoint, coarse_reduction=1e-3, counts=counts)
    prop.vcycle()
    cg, lg = prop.get_state()
    x_gpu = np.concatenate([n(cg), n(lg)])
    assert np.abs(x_gpu - x_ref).max() <= 1e-10 * np.abs(x_ref).max()
    assert 1 <= counts[0] <= 6
    prop.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_with_iterated_coarsest_counts_its_sweeps(precision):
    """A step of the 2D workload reduced to 64^2 (3 levels) with the iterated
    coarsest solve: coefficients against the oracle's direct solve, every coarsest
    solve reached its reduction, and the coarsest sweeps the library reports equal
    the oracle's count for the same V-cycles (FP64 decisions on both sides)."""
    case = Case(shape=(64, 64), h=0.2, n_t=8, block=(8, 8), levels=3)
    note(f"solve with iterated coarsest {precision} {case}")
    t0 = 0.0
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t0, case.field)
    b = kkt.rhs(sysm, case.psi0)
    x_ref = kkt.solve_direct(sysm.K, b)
    prop = case.prop(precision=precision, tol=1e-10, max_cycles=40, nu_coarse=4, coarse_reduction=1e-3)
    _, st = prop.solve_step(t0, t_c(case.psi0))
    cg, _ = prop.get_state()
    c_ref, _ = kkt.split(x_ref, case.npts, case.n_t)
    target = 1e-10 if precision == "fp64" else 1e-8
    assert np.abs(n(cg).reshape(-1, case.n_t) - c_ref).max() <= target * np.abs(c_ref).max()
    assert st["coarse_unmet"] == 0 and st["coarse_sweeps"] >= st["cycles"]
    if precision == "fp64":
        H = relax.build_hierarchy(case.grid, case.v0, case.n_t, case.dt, case.block, case.levels, t0=t0)
        x = kkt.initial_guess(sysm, case.psi0)
        counts = []
        for _ in range(st["cycles"]):
            x = relax.reference_vcycle(H, 0, x, b, 1, 1, 4, coarse_reduction=1e-3, counts=counts)
        assert st["coarse_sweeps"] == sum(counts), (st["coarse_sweeps"], counts)
    prop.close()


SOLVE_CASES = [
    # the 1D workload at its full size
    dict(shape=(256,), h=40 / 256, n_t=8, block=(8,), levels=1, potential="harmonic", nu_coarse=2),
    dict(shape=(256,), h=40 / 256, n_t=8, block=(8,), levels=5, potential="harmonic", nu_coarse=2),
    # the 2D soft-Coulomb workload reduced to 64^2 (same h, dt, n_t, blocks)
    dict(shape=(64, 64), h=0.2, n_t=8, block=(8, 8), levels=3, nu_coarse=2),
    # the 3D laser workload reduced to 16^3
    dict(shape=(16, 16, 16), h=0.3, n_t=6, block=(4, 4, 4), levels=2, pulse=PULSE_SIN2, nu_coarse=2),
    # the 2D adjoint workload reduced to 32^2 with its Fourier pulse
    dict(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2, pulse=PULSE_FOURIER, nu_coarse=2),
]


@pytest.mark.parametrize("cfg", SOLVE_CASES, ids=lambda c: f"{c['shape']}-L{c['levels']}")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_step_parity(cfg, precision):
    cfg = dict(cfg)
    nu_coarse = cfg.pop("nu_coarse")
    case = Case(**cfg)
    note(f"solve {precision} {case}")
    t0 = 0.15
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t0, case.field)
    b = kkt.rhs(sysm, case.psi0)
    x_ref = kkt.solve_direct(sysm.K, b)
    prop = case.prop(precision=precision, tol=1e-10, max_cycles=40, nu_coarse=nu_coarse)
    psi_out, st = prop.solve_step(t0, t_c(case.psi0))
    cg, lg = prop.get_state()
    c_ref, _ = kkt.split(x_ref, case.npts, case.n_t)
    rel = np.abs(n(cg).reshape(-1, case.n_t) - c_ref).max() / np.abs(c_ref).max()
    target = 1e-10 if precision == "fp64" else 1e-8
    note(f"cycles={st['cycles']} resid ratio={st['resid'] / st['resid0']:.2e} coef rel err={rel:.2e}")
    assert rel <= target
    # psi_out = sum of the N_t coefficients of a point: its error is at most N_t times theirs
    psi_ref = kkt.end_state(sysm, x_ref)
    assert np.abs(n(psi_out) - psi_ref).max() <= case.n_t * target * np.abs(c_ref).max()
    prop.close()


@pytest.mark.parametrize("cfg", [SOLVE_CASES[3], SOLVE_CASES[4]], ids=lambda c: f"{c['shape']}-L{c['levels']}")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_defect_tolerance_leaves_the_step_unchanged(cfg, precision):
    """Subvolume solves with the default field-defect tolerance (1e-2) and exact
    ones (inner_tol 1e-13 in FP64, 1e-5 in FP32): the same V-cycle count, both
    within the precision's bound of the oracle's direct step, and the exact
    setting does take correction passes in a V-cycle's sweeps (so the two runs
    differ inside)."""
    cfg = dict(cfg)
    nu_coarse = cfg.pop("nu_coarse")
    case = Case(**cfg)
    note(f"defect tolerance {precision} {case}")
    t0 = 0.15
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t0, case.field)
    x_ref = kkt.solve_direct(sysm.K, kkt.rhs(sysm, case.psi0))
    c_ref, _ = kkt.split(x_ref, case.npts, case.n_t)
    runs = []
    for tol in (0.0, EXACT_INNER_TOL[precision]):
        prop = case.prop(precision=precision, tol=1e-10, max_cycles=40, nu_coarse=nu_coarse, inner_tol=tol)
        c0 = np.concatenate([case.psi0[:, None], np.zeros((case.npts, case.n_t - 1), complex)], 1)
        prop.set_state(t0, t_c(case.psi0), t_c(c0.ravel()), t_c(np.zeros(case.npts, complex)))
        prop.vcycle()
        hist, _ = prop.pass_stats(0)
        passes = sum(k * c for k, c in enumerate(hist))
        _, st = prop.solve_step(t0, t_c(case.psi0))
        cg, _ = prop.get_state()
        runs.append((st["cycles"], n(cg).reshape(-1, case.n_t), passes))
        prop.close()
    note(f"cycles {runs[0][0]} / {runs[1][0]}, passes in a V-cycle's last sweep {runs[0][2]} / {runs[1][2]}")
    assert runs[0][0] == runs[1][0]
    target = 1e-10 if precision == "fp64" else 1e-8
    for cycles, cg, _ in runs:
        assert np.abs(cg - c_ref).max() <= target * np.abs(c_ref).max()
    assert runs[1][2] > 0


def test_multi_step_propagation_matches_direct_steps():
    case = Case(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2, pulse=PULSE_FOURIER)
    note(f"propagate 8 steps {case}")
    psis = kkt.propagate(case.grid, case.v0, case.psi0, case.n_t, case.dt, 8, case.field)
    prop = case.prop(tol=1e-12, max_cycles=60)
    psi, _ = prop.propagate(t_c(case.psi0), 8)
    assert np.abs(n(psi) - psis[-1]).max() <= 1e-10 * np.abs(psis[-1]).max()
    prop.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_step_parity(precision):
    case = Case(shape=(16, 16), h=0.25, n_t=6, block=(4, 4), levels=2, pulse=PULSE_FOURIER)
    note(f"adjoint step {precision} {case}")
    t0 = 0.1
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t0, case.field)
    x = kkt.solve_direct(sysm.K, kkt.rhs(sysm, case.psi0))
    g_out = case.rng.normal(size=case.npts) + 1j * case.rng.normal(size=case.npts)
    mu = A.adjoint_solve(sysm, A.adjoint_rhs(sysm, g_out))
    from oracle import timebasis as tb
    basis = [tb.fourier_basis_function(q, PULSE_FOURIER["t_total"]) for q in (1, 2, 3)]
    g_in_ref, dv0_ref, da_ref = A.step_gradients(sysm, x, mu, basis)
    prop = case.prop(precision=precision, tol=1e-12, max_cycles=60)
    import torch
    dv0 = torch.zeros(case.npts, dtype=torch.float64, device="cuda")
    dcoef = [0.0, 0.0, 0.0]
    g_in, st = prop.adjoint_step(t0, t_c(case.psi0), t_c(g_out), dv0, dcoef)
    tol = 1e-10 if precision == "fp64" else 1e-8
    assert np.abs(n(g_in) - g_in_ref).max() <= tol * np.abs(g_in_ref).max()
    assert np.abs(n(dv0) - dv0_ref).max() <= tol * np.abs(dv0_ref).max()
    assert np.abs(np.array(dcoef) - da_ref).max() <= tol * np.abs(da_ref).max()
    prop.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_step_from_the_stored_forward_solution(precision):
    """lam_adjoint_step_stored with the forward step's converged coefficients:
    the oracle's adjoint state and gradients to the precision's bound (as the
    recomputing adjoint step), and agreement with lam_adjoint_step."""
    import torch
    case = Case(shape=(16, 16), h=0.25, n_t=6, block=(4, 4), levels=2, pulse=PULSE_FOURIER)
    note(f"stored adjoint step {precision} {case}")
    t0 = 0.1
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t0, case.field)
    x = kkt.solve_direct(sysm.K, kkt.rhs(sysm, case.psi0))
    g_out = case.rng.normal(size=case.npts) + 1j * case.rng.normal(size=case.npts)
    mu = A.adjoint_solve(sysm, A.adjoint_rhs(sysm, g_out))
    from oracle import timebasis as tb
    basis = [tb.fourier_basis_function(q, PULSE_FOURIER["t_total"]) for q in (1, 2, 3)]
    g_in_ref, dv0_ref, da_ref = A.step_gradients(sysm, x, mu, basis)
    prop = case.prop(precision=precision, tol=1e-12, max_cycles=60)
    prop.solve_step(t0, t_c(case.psi0))
    c_fwd, _ = prop.get_state()
    tol = 1e-10 if precision == "fp64" else 1e-8
    res = []
    for stored in (True, False):
        dv0 = torch.zeros(case.npts, dtype=torch.float64, device="cuda")
        dcoef = [0.0, 0.0, 0.0]
        if stored:
            g_in, st = prop.adjoint_step_stored(t0, c_fwd, t_c(g_out), dv0, dcoef)
            assert st["sweeps_fine"] == 2 * st["cycles"]   # no forward solve inside
        else:
            g_in, st = prop.adjoint_step(t0, t_c(case.psi0), t_c(g_out), dv0, dcoef)
        assert np.abs(n(g_in) - g_in_ref).max() <= tol * np.abs(g_in_ref).max()
        assert np.abs(n(dv0) - dv0_ref).max() <= tol * np.abs(dv0_ref).max()
        assert np.abs(np.array(dcoef) - da_ref).max() <= tol * np.abs(da_ref).max()
        res.append((n(g_in), n(dv0), np.array(dcoef)))
    for a_, b_ in zip(res[0], res[1]):
        assert np.abs(a_ - b_).max() <= tol * np.abs(b_).max()
    prop.close()


@pytest.mark.parametrize("cfg,precision", [
    (dict(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2), "fp64"),
    (dict(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2), "mixed"),
    (dict(shape=(8, 8, 16), h=0.3, n_t=8, block=(4, 4, 4), levels=2, field_axis=2), "mixed"),
], ids=["2d-fp64", "2d-mixed", "3d-mixed"])
def test_autograd_with_stored_forward_states_matches_the_recomputing_one(cfg, precision):
    """propagate_differentiable(store=True) keeps each step's forward
    coefficients and runs only the adjoint solves backward: the same
    gradients (psi0, V0, pulse amplitudes) as the recomputing form, 1e-10."""
    import torch
    from paper_1111_4363_amd import lam
    case = Case(pulse=None, **cfg)
    n_steps, T = 5, 5 * case.dt
    coef = np.array([0.3, -0.2, 0.25, 0.1])
    pulse = dict(kind="fourier", t_total=T, coef=list(coef))
    note(f"autograd stored vs recomputed {precision} {case}")
    prop = case.prop(pulse=pulse, tol=1e-13, max_cycles=80, precision=precision)
    g_t = t_c(case.psi0)
    grads = []
    for store in (False, True):
        psi0 = t_c(case.psi0).requires_grad_(True)
        v0 = t_r(case.v0).requires_grad_(True)
        cf = torch.tensor(coef, dtype=torch.float64, requires_grad=True)
        psiK = lam.propagate_differentiable(prop, psi0, v0, cf, n_steps, store=store)
        ov = torch.sum(torch.conj(g_t) * psiK)
        (ov * torch.conj(ov)).real.backward()
        grads.append((n(psi0.grad), n(v0.grad), cf.grad.numpy().copy()))
    for a_, b_ in zip(grads[0], grads[1]):
        assert np.abs(a_ - b_).max() <= 1e-10 * np.abs(a_).max()
    prop.close()


def test_autograd_gradients_match_finite_differences():
    """Loss = population of the grid ground state after K steps; gradients with
    respect to the pulse amplitudes and sampled V0 points against central
    differences of the GPU forward (eps = 1e-5), absolute 1e-6."""
    import torch
    from paper_1111_4363_amd import lam
    import workloads as W
    case = Case(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2, pulse=None)
    gs = W.ground_state(case.shape, case.h, case.v0)
    n_steps, T = 6, 6 * case.dt
    coef = np.array([0.3, -0.2, 0.25, 0.1])
    pulse = dict(kind="fourier", t_total=T, coef=list(coef))
    note(f"autograd vs FD {case}")
    prop = case.prop(pulse=pulse, tol=1e-13, max_cycles=80)
    g_t = t_c(gs)
    w = case.h ** 2

    def loss_of(psi):
        ov = w * torch.sum(torch.conj(g_t) * psi)
        return (ov * torch.conj(ov)).real

    psi0 = t_c(gs).requires_grad_(False)
    v0 = t_r(case.v0).requires_grad_(True)
    cf = torch.tensor(coef, dtype=torch.float64, requires_grad=True)
    psiK = lam.propagate_differentiable(prop, psi0, v0, cf, n_steps)
    L = loss_of(psiK)
    L.backward()

    def fwd(vv, cc):
        prop.set_potential(t_r(vv))
        prop.set_pulse(list(cc))
        psi, _ = prop.propagate(t_c(gs), n_steps)
        return float(loss_of(psi))

    eps = 1e-5
    for q in range(len(coef)):
        cp, cm = coef.copy(), coef.copy()
        cp[q] += eps
        cm[q] -= eps
        fd = (fwd(case.v0, cp) - fwd(case.v0, cm)) / (2 * eps)
        assert abs(fd - cf.grad[q].item()) < 1e-6, (q, fd, cf.grad[q].item())
    gv = n(v0.grad)
    for i in [0, 300, 528, 1000]:
        vp, vm = case.v0.copy(), case.v0.copy()
        vp[i] += eps
        vm[i] -= eps
        fd = (fwd(vp, coef) - fwd(vm, coef)) / (2 * eps)
        assert abs(fd - gv[i]) < 1e-6, (i, fd, gv[i])
    prop.close()


def test_native_propagate_matches_stepwise_and_edge_cases():
    """lam_propagate (steps back to back, batched convergence checks) against
    step-by-step lam_solve_step and against the oracle's direct steps; the
    in-place form (psi_in == psi_out) and n_steps = 0."""
    import torch
    case = Case(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2, pulse=PULSE_FOURIER)
    note(f"native propagate {case}")
    psis = kkt.propagate(case.grid, case.v0, case.psi0, case.n_t, case.dt, 5, case.field)
    prop = case.prop(tol=1e-12, max_cycles=60)
    psi_native, st = prop.propagate(t_c(case.psi0), 5)
    seq, _ = prop.propagate(t_c(case.psi0), 5, keep=True)
    ref = np.abs(psis[-1]).max()
    assert np.abs(n(psi_native) - psis[-1]).max() <= 1e-10 * ref
    assert np.abs(n(psi_native) - n(seq[-1])).max() <= 1e-10 * ref
    assert st[0]["cycles"] >= 5 and st[0]["resid"] <= 1e-12 * st[0]["resid0"] * 1.0001
    # in place
    from paper_1111_4363_amd import lam
    buf = t_c(case.psi0).clone()
    code = prop._lib.lam_propagate(prop._ctx, 0.0, 5, lam._ptr(buf, torch.complex128, case.npts),
                                   lam._ptr(buf, torch.complex128, case.npts), None)
    assert code == lam.LAM_OK
    assert np.abs(n(buf) - psis[-1]).max() <= 1e-10 * ref
    # zero steps: nothing written
    keep = t_c(case.psi0).clone()
    out = torch.full_like(keep, 7.0)
    assert prop._lib.lam_propagate(prop._ctx, 0.0, 0, lam._ptr(keep, torch.complex128, case.npts),
                                   lam._ptr(out, torch.complex128, case.npts), None) == lam.LAM_OK
    assert torch.all(out == 7.0)
    prop.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("pulse", [None, dict(kind="sin2", e0=0.05, omega=0.057, t_total=0.1)],
                         ids=["no-field", "field-ends-mid-run"])
def test_native_propagate_queued_next_step(pulse, precision):
    """Each step's successor has its start queued ahead of each wait (spare
    buffers swapped in when the step has converged).  Against the oracle's
    direct steps and the step-by-step path: a run with no field, and one whose
    pulse ends with the second step; the in-place form; the context state after the run is the last
    step's, and an adjoint step on the same context (its state buffers swapped
    by the runs) matches the oracle's direct adjoint; a tiny max_cycles stops
    the run at its first step with that step's result."""
    import torch
    from paper_1111_4363_amd import lam
    case = Case(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2, pulse=pulse)
    note(f"native propagate, next step queued ahead {precision} {case}")
    K = 7
    psis = kkt.propagate(case.grid, case.v0, case.psi0, case.n_t, case.dt, K, case.field)
    ref = np.abs(psis[-1]).max()
    tol = 1e-10 if precision == "fp64" else 1e-8
    prop = case.prop(tol=1e-12, max_cycles=60, precision=precision)
    psi_native, st = prop.propagate(t_c(case.psi0), K)
    assert np.abs(n(psi_native) - psis[-1]).max() <= tol * ref
    assert st[0]["resid"] <= 1e-12 * st[0]["resid0"] * 1.0001
    cg, _ = prop.get_state()
    assert np.abs(n(cg).reshape(-1, case.n_t).sum(axis=1) - n(psi_native)).max() <= 1e-14 * ref
    # the last step's N0 came from the queued-ahead pass (H applied to the end
    # state psi): the same as the residual of that step's initial guess
    psi_prev, _ = prop.propagate(t_c(case.psi0), K - 1)
    _, st1 = prop.solve_step((K - 1) * case.dt, psi_prev)
    assert abs(st[0]["resid0_last"] - st1["resid0"]) <= 1e-9 * st1["resid0"]
    seq, _ = prop.propagate(t_c(case.psi0), K, keep=True)
    assert np.abs(n(psi_native) - n(seq[-1])).max() <= tol * ref
    buf = t_c(case.psi0).clone()
    assert prop._lib.lam_propagate(prop._ctx, 0.0, K, lam._ptr(buf, torch.complex128, case.npts),
                                   lam._ptr(buf, torch.complex128, case.npts), None) == lam.LAM_OK
    assert np.abs(n(buf) - psis[-1]).max() <= tol * ref
    # adjoint step of the last step, on the context the runs above left behind
    t_last = (K - 1) * case.dt
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t_last, case.field)
    x = kkt.solve_direct(sysm.K, kkt.rhs(sysm, psis[-2]))
    g_out = case.rng.normal(size=case.npts) + 1j * case.rng.normal(size=case.npts)
    mu = A.adjoint_solve(sysm, A.adjoint_rhs(sysm, g_out))
    g_in_ref, dv0_ref, _ = A.step_gradients(sysm, x, mu)
    dv0 = torch.zeros(case.npts, dtype=torch.float64, device="cuda")
    g_in, _ = prop.adjoint_step(t_last, t_c(psis[-2]), t_c(g_out), dv0)
    assert np.abs(n(g_in) - g_in_ref).max() <= tol * np.abs(g_in_ref).max()
    assert np.abs(n(dv0) - dv0_ref).max() <= tol * np.abs(dv0_ref).max()
    prop.close()
    # two cycles cannot reach 1e-12: LAM_ENOCONV after the first step, psi_out = its end state
    short = case.prop(tol=1e-12, max_cycles=2)
    out = torch.zeros_like(t_c(case.psi0))
    code = short._lib.lam_propagate(short._ctx, 0.0, K, lam._ptr(t_c(case.psi0), torch.complex128, case.npts),
                                    lam._ptr(out, torch.complex128, case.npts), None)
    assert code == lam.LAM_ENOCONV
    short.close()
    one = case.prop(tol=1e-12, max_cycles=2)
    psi1, _ = one.solve_step(0.0, t_c(case.psi0), allow_noconv=True)
    assert torch.equal(out, psi1)
    one.close()


@pytest.mark.parametrize("cfg", [
    dict(shape=(64,), n_t=8, block=(8,), levels=2, h=0.3, potential="harmonic"),
    dict(shape=(16, 16), n_t=4, block=(4, 4), levels=2, h=0.3, periodic=True),
    dict(shape=(8, 8, 8), n_t=6, block=(4, 4, 4), levels=2, h=0.3),
], ids=lambda c: f"{c['shape']}-p{c.get('periodic', False)}")
def test_queued_step_across_grids(cfg):
    """The queued-ahead start of field-free steps on 1D, periodic 2D and 3D
    grids: the run matches the step-by-step path, and the last step's N0 (from
    the same pass as its initial state) the plain residual of that guess."""
    case = Case(**cfg)
    note(f"queued step {case}")
    K = 4
    prop = case.prop(tol=1e-12, max_cycles=60)
    psi_native, st = prop.propagate(t_c(case.psi0), K)
    seq, _ = prop.propagate(t_c(case.psi0), K, keep=True)
    ref = np.abs(n(seq[-1])).max()
    assert np.abs(n(psi_native) - n(seq[-1])).max() <= 1e-10 * ref
    _, st1 = prop.solve_step((K - 1) * case.dt, seq[-2])
    assert abs(st[0]["resid0_last"] - st1["resid0"]) <= 1e-9 * st1["resid0"]
    prop.close()


@pytest.mark.parametrize("cfg", [
    dict(shape=(16, 16), n_t=8, block=(4, 4), levels=2, h=0.3, field_axis=0),
    dict(shape=(8, 8, 8), n_t=6, block=(4, 4, 4), levels=2, h=0.3, field_axis=2, periodic=True),
], ids=lambda c: f"{c['shape']}-axis{c['field_axis']}")
def test_queued_field_step_has_the_initial_norm_of_its_guess(cfg):
    """Field steps also take the queued-ahead start: the N0 of the last step of
    a run inside the pulse (formed from the end state psi with that step's
    field) equals the plain residual norm of the same initial guess."""
    pulse = dict(kind="sin2", e0=0.2, omega=0.9, t_total=1.0)
    case = Case(pulse=pulse, **cfg)
    note(f"queued field step {case}")
    K = 4
    t_start = 0.3
    prop = case.prop(tol=1e-12, max_cycles=60)
    psi_native, st = prop.propagate(t_c(case.psi0), K, t_start)
    seq, _ = prop.propagate(t_c(case.psi0), K, t_start, keep=True)
    ref = np.abs(n(seq[-1])).max()
    assert np.abs(n(psi_native) - n(seq[-1])).max() <= 1e-10 * ref
    _, st1 = prop.solve_step(t_start + (K - 1) * case.dt, seq[-2])
    assert abs(st[0]["resid0_last"] - st1["resid0"]) <= 1e-9 * st1["resid0"]
    prop.close()
    # the field term matters here: without it the same guess has another N0
    plain = Case(**cfg).prop(tol=1e-12, max_cycles=60)
    _, st0 = plain.solve_step(t_start + (K - 1) * case.dt, seq[-2])
    assert abs(st0["resid0"] - st1["resid0"]) > 1e-6 * st1["resid0"]
    plain.close()


def test_sweep_profiling_samples_every_kth_launch():
    """lam_profile(k) records the 1st, (k+1)-th, ... finest-level sweep launch."""
    case = Case(shape=(32, 32), h=0.2, n_t=8, block=(8, 8), levels=2)
    note(f"profile sampling {case}")
    prop = case.prop(tol=1e-10, max_cycles=40)
    for k in (1, 3):
        prop.profile(k)
        _, st = prop.solve_step(0.0, t_c(case.psi0))
        launches, ms = prop.profile_read()
        prop.profile(0)
        total = 2 * st["sweeps_fine"]          # two colour launches per full sweep
        assert launches == (total + k - 1) // k, (k, launches, total)
        assert ms > 0.0
    prop.close()
