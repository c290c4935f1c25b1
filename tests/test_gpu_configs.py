"""The differentiation workloads at their own configurations, and mixed against FP64.

* 2d_adjoint (256^2, h = 0.2, N_t = 8, 8x8 subvolumes, 4 levels, 40 steps,
  16 Fourier amplitudes ~ N(0, 0.02^2) seed 0, loss = population of the grid
  ground state after the last step): autograd gradients with respect to every
  amplitude and sampled V0 points against central differences of the GPU
  forward, at the full size, in FP64 and mixed; the same pipeline at 32^2
  against the oracle's direct forward and adjoint solves.
* 3d_large (256^3, mixed, sin^2 pulse plus 32 Fourier amplitudes, 20 steps):
  forward and adjoint through the autograd function, gradients of a subset of
  the amplitudes against central differences.
* Mixed against FP64 element by element after the workloads' own number of
  steps, at full size.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import n, note, t_c, t_r
from oracle import adjoint as A
from oracle import grid as G

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def make_prop(cfg, v0, precision, tol, max_cycles=80):
    import torch
    from paper_1111_4363_amd import lam
    p = cfg["pulse"]
    pulse = None
    if p:
        pulse = dict(kind=p["kind"], e0=p.get("e0", 0.0), omega=p.get("omega", 0.0), t_total=cfg["t_total"],
                     coef=list(W.pulse_coefficients(cfg)))
    return lam.Propagator(cfg["shape"], cfg["h"], torch.as_tensor(v0, device="cuda"), cfg["n_t"], cfg["dt"],
                          (cfg["block"],) * cfg["dim"], levels=cfg["levels"], nu_coarse=cfg["nu_coarse"],
                          coarse_reduction=cfg["coarse_reduction"], pulse=pulse, precision=precision, tol=tol,
                          max_cycles=max_cycles)


def population(g_t, w):
    import torch

    def loss_of(psi):
        ov = w * torch.sum(torch.conj(g_t) * psi)
        return (ov * torch.conj(ov)).real
    return loss_of


def autograd_and_fd(cfg, precision, fd_coef, fd_points, ref_state=None):
    """Autograd gradients of L = |<g|psi_K>|^2 with respect to the Fourier
    amplitudes and V0, and central differences (eps = 1e-5) of the GPU forward
    for the amplitudes fd_coef and the points fd_points."""
    import torch
    from paper_1111_4363_amd import lam
    v0 = W.potential(cfg)
    psi0 = W.initial_state(cfg, v0)
    g = psi0 if ref_state is None else ref_state
    coef = W.pulse_coefficients(cfg)
    K = cfg["steps"]
    prop = make_prop(cfg, v0, precision, tol=1e-13)
    g_t = t_c(g)
    loss_of = population(g_t, cfg["h"] ** cfg["dim"])
    v0_t = t_r(v0).requires_grad_(True)
    cf = torch.tensor(coef, dtype=torch.float64, requires_grad=True)
    psiK = lam.propagate_differentiable(prop, t_c(psi0), v0_t, cf, K)
    L = loss_of(psiK)
    L.backward()
    ga, gv = cf.grad.numpy().copy(), n(v0_t.grad)

    def fwd(vv, cc):
        prop.hold(t_r(vv), list(cc))
        psi, _ = prop.propagate(t_c(psi0), K)
        return float(loss_of(psi))

    eps = 1e-5
    fd_a, fd_v = [], []
    for q in fd_coef:
        cp, cm = coef.copy(), coef.copy()
        cp[q] += eps
        cm[q] -= eps
        fd_a.append((fwd(v0, cp) - fwd(v0, cm)) / (2 * eps))
    for i in fd_points:
        vp, vm = v0.copy(), v0.copy()
        vp[i] += eps
        vm[i] -= eps
        fd_v.append((fwd(vp, coef) - fwd(vm, coef)) / (2 * eps))
    prop.close()
    return float(L), ga, gv, np.array(fd_a), np.array(fd_v)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_2d_adjoint_fullsize_autograd_against_finite_differences(precision):
    """The 2D adjoint workload as named: 256^2, 40 steps, 16 amplitudes, ground-state
    population; all 16 dL/da_q and dL/dV0 at points around the centre against
    central differences of the GPU forward, absolute 1e-6."""
    cfg = W.config("2d_adjoint")
    note(f"2d_adjoint full size autograd vs FD {precision} {cfg['shape']} steps={cfg['steps']}")
    N = cfg["n"]
    c = N // 2
    pts = [c * N + c, (c - 3) * N + c + 5, (c + 10) * N + c - 7]
    L, ga, gv, fd_a, fd_v = autograd_and_fd(cfg, precision, range(16), pts)
    note(f"L={L:.12f} max|dL/da|={np.abs(ga).max():.3e} max err a={np.abs(ga - fd_a).max():.2e} "
         f"v={np.abs(gv[pts] - fd_v).max():.2e}")
    assert np.abs(ga) .max() > 1e-5          # the gradient is not trivially zero
    assert np.abs(ga - fd_a).max() < 1e-6, (ga, fd_a)
    assert np.abs(gv[pts] - fd_v).max() < 1e-6, (gv[pts], fd_v)


@pytest.fixture(scope="module")
def oracle_2d_adjoint_reduced():
    cfg = W.config("2d_adjoint", n=32, levels=2)
    v0 = W.potential(cfg)
    g = W.initial_state(cfg, v0)
    coef = W.pulse_coefficients(cfg)
    grid = G.Grid(cfg["shape"], cfg["h"])
    L, g0, dv0, da = A.loss_and_gradients(grid, v0, g, cfg["n_t"], cfg["dt"], cfg["steps"], g, list(coef),
                                          cfg["t_total"])
    return cfg, L, g0, dv0, da


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_2d_adjoint_pipeline_against_oracle_direct_adjoint(precision, oracle_2d_adjoint_reduced):
    """The same 40-step pipeline (recipe, pulse, loss) at 32^2 against the oracle's
    direct forward and adjoint solves: L, dL/dpsi0^*, dL/dV0 and dL/da to 1e-10
    (FP64) / 1e-8 (mixed) relative to each gradient's largest entry."""
    import torch
    from paper_1111_4363_amd import lam
    cfg, L_ref, g0_ref, dv0_ref, da_ref = oracle_2d_adjoint_reduced
    note(f"2d_adjoint 32^2 40 steps vs oracle adjoint {precision}")
    v0 = W.potential(cfg)
    g = W.initial_state(cfg, v0)
    prop = make_prop(cfg, v0, precision, tol=1e-13)
    g_t = t_c(g)
    loss_of = population(g_t, cfg["h"] ** 2)
    psi0 = t_c(g).requires_grad_(True)
    v0_t = t_r(v0).requires_grad_(True)
    cf = torch.tensor(W.pulse_coefficients(cfg), dtype=torch.float64, requires_grad=True)
    L = loss_of(lam.propagate_differentiable(prop, psi0, v0_t, cf, cfg["steps"]))
    L.backward()
    tol = 1e-10 if precision == "fp64" else 1e-8
    assert abs(float(L) - L_ref) <= tol
    # torch's gradient of a real loss with respect to a complex input is 2 dL/dpsi^*
    g0 = 0.5 * n(psi0.grad)
    assert np.abs(g0 - g0_ref).max() <= tol * np.abs(g0_ref).max()
    assert np.abs(n(v0_t.grad) - dv0_ref).max() <= tol * np.abs(dv0_ref).max()
    assert np.abs(cf.grad.numpy() - da_ref).max() <= tol * np.abs(da_ref).max()
    prop.close()


def test_3d_large_fullsize_adjoint_against_finite_differences():
    """The 256^3 workload, mixed precision, 20 steps of the sin^2 + 32-amplitude
    pulse, loss = population of the initial state after the last step: forward and
    adjoint through the autograd function; dL/da_q of three amplitudes (low, middle
    and highest frequency) against central differences, absolute 1e-6."""
    cfg = W.config("3d_large")
    note(f"3d_large full size adjoint vs FD mixed {cfg['shape']} steps={cfg['steps']}")
    L, ga, gv, fd_a, _ = autograd_and_fd(cfg, "mixed", [0, 15, 31], [])
    note(f"L={L:.12f} dL/da[0,15,31]={ga[[0, 15, 31]]} FD={fd_a} max|dL/dV0|={np.abs(gv).max():.3e}")
    assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gv))
    assert np.abs(ga[[0, 15, 31]] - fd_a).max() < 1e-6, (ga[[0, 15, 31]], fd_a)


def test_autograd_restores_its_own_system_between_interleaved_forwards():
    """Two forwards on one Propagator with different potentials and pulses, then the
    two backwards in reverse order: each gradient is that of its own forward
    (against central differences), not of the system the Propagator last held."""
    import torch
    from paper_1111_4363_amd import lam
    cfg = W.config("2d_adjoint", n=32, levels=2, steps=4)
    v0a = W.potential(cfg)
    v0b = v0a + 0.05 * W.random_real(v0a.size, 3)
    g = W.initial_state(cfg, v0a)
    ca = W.pulse_coefficients(cfg) * 10.0
    cb = -0.5 * ca
    prop = make_prop(cfg, v0a, "fp64", tol=1e-13)
    loss_of = population(t_c(g), cfg["h"] ** 2)
    note("interleaved forwards on one Propagator")
    grads = []
    outs = []
    for vv, cc in ((v0a, ca), (v0b, cb)):
        v_t = t_r(vv).requires_grad_(True)
        c_t = torch.tensor(cc, dtype=torch.float64, requires_grad=True)
        outs.append((loss_of(lam.propagate_differentiable(prop, t_c(g), v_t, c_t, cfg["steps"])), v_t, c_t))
    for L, v_t, c_t in reversed(outs):
        L.backward()
        grads.append((n(v_t.grad), c_t.grad.numpy().copy()))
    grads = grads[::-1]

    def fwd(vv, cc):
        prop.hold(t_r(vv), list(cc))
        psi, _ = prop.propagate(t_c(g), cfg["steps"])
        return float(loss_of(psi))

    eps = 1e-5
    j = (cfg["n"] // 2) * cfg["n"] + cfg["n"] // 2
    for (vv, cc), (gv, ga) in zip(((v0a, ca), (v0b, cb)), grads):
        for q in (0, 5):
            cp, cm = cc.copy(), cc.copy()
            cp[q] += eps
            cm[q] -= eps
            assert abs((fwd(vv, cp) - fwd(vv, cm)) / (2 * eps) - ga[q]) < 1e-6
        vp, vm = vv.copy(), vv.copy()
        vp[j] += eps
        vm[j] -= eps
        assert abs((fwd(vp, cc) - fwd(vm, cc)) / (2 * eps) - gv[j]) < 1e-6
    prop.close()


@pytest.mark.parametrize("name", ["1d_harmonic", "2d_softcoulomb", "3d_laser", "2d_adjoint", "3d_large"])
def test_mixed_against_fp64_after_the_workload_steps(name):
    """Each workload's own number of steps at full size, solved to 1e-10 in FP64
    and on the mixed path: psi_K of the two agrees element by element to 1e-8 of
    its largest entry (the mixed path's target accuracy after refinement)."""
    cfg = W.config(name)
    v0 = W.potential(cfg)
    psi0 = W.initial_state(cfg, v0)
    out = {}
    for prec in ("fp64", "mixed"):
        prop = make_prop(cfg, v0, prec, tol=1e-10, max_cycles=60)
        psi, st = prop.propagate(t_c(psi0), cfg["steps"])
        out[prec] = n(psi)
        note(f"{name} {prec}: {cfg['steps']} steps, worst step ratio {st[0]['resid'] / st[0]['resid0']:.2e}")
        prop.close()
    ref = np.abs(out["fp64"]).max()
    err = np.abs(out["mixed"] - out["fp64"]).max() / ref
    note(f"{name}: max |psi_mixed - psi_fp64| / max |psi_fp64| = {err:.2e} after {cfg['steps']} steps")
    assert err <= 1e-8
