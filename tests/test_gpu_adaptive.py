"""The adaptive tree on the GPU (through the C ABI) against the oracle
(oracle/composite.py): the Galerkin hierarchy with piecewise-constant
interpolation, the Haar detail per subvolume, and solves with the finest level
refined on some subvolumes against the directly solved composite state
(Sec. "Multigrid Relaxation")."""
import numpy as np
import pytest

from gpu_util import Case, n, note, t_c
from oracle import composite as C
from oracle import kkt, relax

pytestmark = pytest.mark.gpu

PULSE = dict(kind="sin2", t_total=0.4, e0=0.2, omega=0.9)


def galerkin_case(**kw):
    return Case(interp="constant", **kw)


def gprop(case, **kw):
    args = dict(coarse_op="galerkin", nu_coarse=4, coarse_reduction=1e-3, max_cycles=80)
    args.update(kw)
    return case.prop(**args)


@pytest.mark.parametrize("cfg", [
    dict(shape=(32, 32), n_t=4, block=(4, 4), levels=3, h=0.2),
    dict(shape=(64,), n_t=8, block=(8,), levels=3, h=0.3, potential="harmonic"),
    dict(shape=(8, 8, 16), n_t=3, block=(2, 2, 2), levels=2, h=0.3, pulse=PULSE, field_axis=2),
], ids=lambda c: f"{c['shape']}-L{c['levels']}")
def test_galerkin_vcycle_parity(cfg):
    """One V-cycle of the Galerkin hierarchy (coarse kinetic coefficient halved per
    level) against the oracle's V-cycle over explicit R K I products."""
    case = galerkin_case(**cfg)
    note(f"galerkin vcycle {case}")
    t0 = 0.1
    H = C.galerkin_hierarchy(case.grid, case.v0, case.n_t, case.dt, case.block, case.levels, t0, case.field)
    sysm = H[0].system
    c, lam = case.random_state(0.1)
    x = kkt.join(c, lam)
    prop = gprop(case, nu_coarse=2, coarse_reduction=0.0, n_inner=(8 if case.field else -1))
    b = kkt.rhs(sysm, case.psi0)
    prop.set_state(t0, t_c(case.psi0), t_c(c), t_c(lam))
    x_ref = relax.reference_vcycle(H, 0, x, b, 1, 1, 2)
    prop.vcycle()
    cg, lg = prop.get_state()
    x_gpu = np.concatenate([n(cg), n(lg)])
    assert np.abs(x_gpu - x_ref).max() <= 1e-10 * np.abs(x_ref).max()
    prop.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_galerkin_solve_matches_the_direct_step(precision):
    case = galerkin_case(shape=(32, 32), n_t=6, block=(4, 4), levels=3, h=0.2)
    note(f"galerkin solve {precision} {case}")
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, 0.0, None)
    x_dir = kkt.solve_direct(sysm.K, kkt.rhs(sysm, case.psi0))
    prop = gprop(case, precision=precision, tol=1e-11)
    _, st = prop.solve_step(0.0, t_c(case.psi0))
    cg, _ = prop.get_state()
    c_ref, _ = kkt.split(x_dir, case.npts, case.n_t)
    note(f"cycles {st['cycles']}")
    assert np.abs(n(cg).reshape(-1, case.n_t) - c_ref).max() <= (1e-10 if precision == "fp64" else 1e-8) * \
        np.abs(c_ref).max()
    prop.close()


@pytest.mark.parametrize("shape,block", [((64,), (8,)), ((16, 24), (4, 4)), ((8, 8, 16), (4, 4, 4)),
                                         ((12, 12), (3, 3))])
def test_block_detail_matches_the_oracle(shape, block):
    """Haar detail energy per subvolume; the 3 x 3 blocks do not hold whole
    sibling cells, so siblings come from neighbouring subvolumes."""
    case = galerkin_case(shape=shape, n_t=2, block=block, levels=2, h=0.3)
    note(f"block detail {case}")
    prop = gprop(case)
    got = prop.block_detail(t_c(case.psi0))
    ref = C.haar_detail(case.grid, case.psi0, block)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    prop.close()


def _central_mask(case, radius):
    r2 = sum(x * x for x in case.grid.coords()).ravel()
    from oracle import grid as G
    return np.array([np.sqrt(r2[pts].mean()) < radius for _, pts in G.blocks(case.grid, case.block)])


@pytest.mark.parametrize("cfg", [
    dict(shape=(16, 16), n_t=4, block=(4, 4), levels=3, h=0.25),
    dict(shape=(64,), n_t=8, block=(8,), levels=3, h=0.2, potential="harmonic"),
    dict(shape=(8, 8, 8), n_t=3, block=(2, 2, 2), levels=2, h=0.3),
], ids=lambda c: f"{c['shape']}-L{c['levels']}")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_refined_solve_reaches_the_composite_state(cfg, precision):
    """The finest level refined on the central subvolumes only: the step's solve
    converges (composite norm to 1e-11 of its start) to the oracle's directly
    solved composite state, 1e-9 (FP64) / 1e-8 (mixed) of its largest entry."""
    case = galerkin_case(**cfg)
    act = _central_mask(case, 1.2)
    note(f"refined solve {precision} {case}: {act.sum()} of {act.size} subvolumes refined")
    assert 0 < act.sum() < act.size
    H = C.galerkin_hierarchy(case.grid, case.v0, case.n_t, case.dt, case.block, 2)
    sysm = H[0].system
    b = kkt.rhs(sysm, case.psi0)
    x_ref, eq = C.composite_solve(H, b, kkt.initial_guess(sysm, case.psi0), act)
    assert eq < 1e-10
    prop = gprop(case, precision=precision, tol=1e-11)
    prop.set_refinement(act)
    _, st = prop.solve_step(0.0, t_c(case.psi0))
    cg, lg = prop.get_state()
    x_gpu = np.concatenate([n(cg), n(lg)])
    err = np.abs(x_gpu - x_ref).max() / np.abs(x_ref).max()
    note(f"cycles {st['cycles']}, composite ratio {st['resid'] / st['resid0']:.1e}, error {err:.1e}")
    assert st["resid"] <= 1e-11 * st["resid0"]
    assert err <= (1e-9 if precision == "fp64" else 1e-8)
    prop.close()


def test_every_subvolume_refined_is_the_plain_step():
    case = galerkin_case(shape=(16, 16), n_t=4, block=(4, 4), levels=3, h=0.25)
    note(f"all refined {case}")
    prop = gprop(case, tol=1e-12)
    psi_plain, _ = prop.solve_step(0.0, t_c(case.psi0))
    prop.set_refinement(np.ones(16, np.uint8))
    psi_all, _ = prop.solve_step(0.0, t_c(case.psi0))
    prop.set_refinement(None)
    psi_again, _ = prop.solve_step(0.0, t_c(case.psi0))
    ref = np.abs(n(psi_plain)).max()
    # (each solve stops at its own tolerance, after as many V-cycles as it needed)
    assert np.abs(n(psi_all) - n(psi_plain)).max() <= 1e-10 * ref
    assert np.abs(n(psi_again) - n(psi_plain)).max() <= 1e-10 * ref
    prop.close()


def test_refinement_needs_the_galerkin_hierarchy_and_the_adjoint_runs_unrefined():
    import torch
    from paper_1111_4363_amd import lam
    case = Case(shape=(16, 16), n_t=4, block=(4, 4), levels=2, h=0.25)
    prop = case.prop()
    with pytest.raises(lam.LamError) as e:
        prop.set_refinement(np.ones(16, np.uint8))
    assert e.value.code == lam.LAM_EINVAL
    prop.close()
    gc = galerkin_case(shape=(16, 16), n_t=4, block=(4, 4), levels=2, h=0.25)
    prop = gprop(gc, tol=1e-12)
    g_out = t_c(gc.psi0)
    grads = []
    for mask in (None, _central_mask(gc, 1.2)):
        prop.set_refinement(mask)
        dv0 = torch.zeros(gc.npts, dtype=torch.float64, device="cuda")
        g_in, _ = prop.adjoint_step(0.0, t_c(gc.psi0), g_out, dv0)
        grads.append((n(g_in), n(dv0)))
    for k in (0, 1):
        assert np.abs(grads[1][k] - grads[0][k]).max() <= 1e-9 * np.abs(grads[0][k]).max()
    prop.close()
