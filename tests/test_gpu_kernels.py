"""GPU parity of the individual kernels against the oracle (through the C ABI).

Residual: elementwise within 1024 eps (|K||x| + |b|): the rounding of a row sum
of at most (2d + 2 n_t + 2) FP64 products on the HIP side plus the rounding the
oracle's quadrature-evaluated Q carries (gpu_util.rounding_bound).
Block factor: V orthogonal and V diag(e) V^T = T_U + diag(V0_U) within
1e-13 of ||A||_F (Jacobi converged to an off-diagonal Frobenius ratio 1e-15).
Transfers: averages and interpolation weights are exact binary fractions, so
1e-15 relative.
"""
import numpy as np
import pytest

from gpu_util import Case, EPS, EXACT_INNER_TOL, field_fn, n, note, rounding_bound, t_c
from oracle import adjoint as A
from oracle import grid as G
from oracle import kkt, relax

pytestmark = pytest.mark.gpu

PULSE_SIN2 = dict(kind="sin2", e0=0.05, omega=0.057, t_total=1.0)
PULSE_FOURIER = dict(kind="fourier", t_total=0.8, coef=[0.03, -0.02, 0.05])
PULSE_BOTH = dict(kind="sin2+fourier", e0=0.1, omega=0.3, t_total=1.0, coef=[0.02, 0.01])

RESIDUAL_CASES = [
    dict(shape=(24,), n_t=3, block=(8,)),
    dict(shape=(264,), n_t=8, block=(8,), potential="harmonic", h=40 / 256),
    dict(shape=(24, 40), n_t=8, block=(4, 4), pulse=PULSE_SIN2),
    dict(shape=(8, 12, 10), n_t=6, block=(2, 2, 2), pulse=PULSE_FOURIER),
    dict(shape=(16, 8), n_t=4, block=(4, 4), periodic=True, pulse=PULSE_BOTH),
    dict(shape=(20,), n_t=1, block=(4,), mass=1.7, potential="random"),
    dict(shape=(6, 10), n_t=5, block=(2, 2), field_axis=0, pulse=PULSE_SIN2),
    # 3D grids whose (y, z) plane tiles by 8 x 8 with an even x extent (the residual
    # that marches along x): ragged x ranges, periodic, each field axis, odd N_t
    dict(shape=(6, 8, 16), n_t=8, block=(2, 2, 2), pulse=PULSE_BOTH, field_axis=1),
    dict(shape=(8, 16, 8), n_t=3, block=(4, 4, 4), periodic=True, pulse=PULSE_FOURIER, field_axis=0),
    dict(shape=(34, 8, 8), n_t=5, block=(2, 2, 2), pulse=PULSE_SIN2),
]


@pytest.mark.parametrize("cfg", RESIDUAL_CASES, ids=lambda c: f"{c['shape']}-nt{c['n_t']}")
@pytest.mark.parametrize("adjoint", [False, True])
def test_residual_parity(cfg, adjoint):
    case = Case(**cfg)
    note(f"residual adjoint={adjoint} {case}")
    t0 = 0.35
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t0, case.field)
    c, lam = case.random_state()
    x = kkt.join(c, lam)
    prop = case.prop()
    if not adjoint:
        b = kkt.rhs(sysm, case.psi0)
        r_ref = b - sysm.K @ x
        rho, sig, N = prop.residual_action(t0, t_c(case.psi0), t_c(c), t_c(lam))
        K = sysm.K
    else:
        g = case.psi0 * 0.7 + 0.1j
        b = A.adjoint_rhs(sysm, g)
        K = sysm.K.conj().T.tocsr()
        r_ref = b - K @ x
        rho, sig, N = prop.residual_adjoint(t0, t_c(g), t_c(c), t_c(lam))
    r_gpu = np.concatenate([n(rho), n(sig)])
    bound = rounding_bound(K, x, b)
    err = np.abs(r_gpu - r_ref)
    assert np.all(err <= bound), (err.max(), bound[np.argmax(err - bound)])
    N_ref = kkt.residual_norm(sysm, r_ref)
    assert abs(N - N_ref) <= 1e-12 * N_ref
    prop.close()


@pytest.mark.parametrize("cfg", [dict(shape=(16, 16), block=(8, 8)), dict(shape=(8, 8, 8), block=(4, 4, 4)),
                                 dict(shape=(32,), block=(8,), potential="harmonic"),
                                 dict(shape=(12, 6), block=(3, 3), potential="random"),
                                 dict(shape=(8, 8), block=(8, 8), periodic=True)],
                         ids=lambda c: f"{c['shape']}-{c['block']}")
def test_block_factor_parity(cfg):
    case = Case(**cfg)
    note(f"block factor {case}")
    prop = case.prop()
    K = G.kinetic(case.grid)
    for blk, (_, pts) in enumerate(G.blocks(case.grid, case.block)):
        Ab = K[pts][:, pts].toarray() + np.diag(case.v0[pts])
        V, e = prop.block_factor(0, blk)
        nrm = np.linalg.norm(Ab)
        assert np.abs(V.T @ V - np.eye(len(pts))).max() < 1e-13
        assert np.abs(V @ np.diag(e) @ V.T - Ab).max() < 1e-13 * nrm
        np.testing.assert_allclose(np.sort(e), np.linalg.eigvalsh(Ab), atol=1e-13 * nrm)
    prop.close()


@pytest.mark.parametrize("cfg", [dict(shape=(16, 24), block=(4, 4), levels=2),
                                 dict(shape=(8, 8, 16), block=(2, 2, 2), levels=3),
                                 dict(shape=(32,), block=(4,), levels=2, periodic=True),
                                 dict(shape=(16, 8), block=(2, 2), levels=2, periodic=True),
                                 # coarse extents that the interpolation's 2 x 8 / 2 x 2 x 8 tiles
                                 # do not divide (partial tiles), Dirichlet and periodic
                                 dict(shape=(12, 20), block=(2, 2), levels=2),
                                 dict(shape=(4, 8, 24), block=(2, 2, 2), levels=2, periodic=True)],
                         ids=lambda c: f"{c['shape']}-L{c['levels']}-p{c.get('periodic', False)}")
@pytest.mark.parametrize("interp", ["linear", "constant"])
def test_transfer_parity(cfg, interp):
    case = Case(n_t=3, interp=interp, **cfg)
    note(f"transfers {interp} {case}")
    prop = case.prop()
    g = case.grid
    for level in range(case.levels - 1):
        gc = G.coarsen_grid(g)
        R = G.restriction(g)
        I = G.interpolation(g, interp)
        rho = case.rng.normal(size=(g.npts, 3)) + 1j * case.rng.normal(size=(g.npts, 3))
        sig = case.rng.normal(size=g.npts) + 1j * case.rng.normal(size=g.npts)
        rc, sc = prop.restrict(level, t_c(rho), t_c(sig))
        np.testing.assert_allclose(n(rc).reshape(-1, 3), R @ rho, rtol=0, atol=1e-15 * np.abs(rho).max())
        np.testing.assert_allclose(n(sc), R @ sig, rtol=0, atol=1e-15 * np.abs(sig).max())
        cc = case.rng.normal(size=(gc.npts, 3)) + 1j * case.rng.normal(size=(gc.npts, 3))
        lc = case.rng.normal(size=gc.npts) + 1j * case.rng.normal(size=gc.npts)
        cf = case.rng.normal(size=(g.npts, 3)) + 1j * case.rng.normal(size=(g.npts, 3))
        lf = case.rng.normal(size=g.npts) + 1j * case.rng.normal(size=g.npts)
        tcf, tlf = t_c(cf), t_c(lf)
        prop.prolong_add(level, t_c(cc), t_c(lc), tcf, tlf)
        np.testing.assert_allclose(n(tcf).reshape(-1, 3), cf + I @ cc, rtol=0, atol=1e-14 * np.abs(cf).max())
        np.testing.assert_allclose(n(tlf), lf + I @ lc, rtol=0, atol=1e-14 * np.abs(lf).max())
        g = gc
    prop.close()


SWEEP_CASES = [
    dict(shape=(256,), n_t=8, block=(8,), h=40 / 256, potential="harmonic", dt=0.05),
    dict(shape=(24, 16), n_t=8, block=(8, 8), h=0.2),
    dict(shape=(20, 12), n_t=5, block=(4, 4), h=0.2, pulse=PULSE_SIN2),
    dict(shape=(8, 8, 12), n_t=6, block=(4, 4, 4), h=0.3, pulse=PULSE_BOTH),
    dict(shape=(16, 8), n_t=4, block=(4, 4), h=0.3, periodic=True, pulse=PULSE_FOURIER),
    dict(shape=(12, 6), n_t=3, block=(3, 3), h=0.3, potential="random"),
    dict(shape=(16, 16), n_t=4, block=(4, 16), h=0.3, periodic=True),
    # 3D 4 x 4 x 4 blocks with N_t = 8 and N_t <= 4 (the mixed path's compile-time block
    # geometry), with a field, and periodic with one block spanning an axis
    dict(shape=(8, 12, 8), n_t=8, block=(4, 4, 4), h=0.3, pulse=PULSE_BOTH),
    dict(shape=(4, 8, 8), n_t=4, block=(4, 4, 4), h=0.3, periodic=True),
    # 2D 8 x 8 blocks (the other compile-time geometry), with a field, and periodic
    dict(shape=(32, 16), n_t=8, block=(8, 8), h=0.2, pulse=PULSE_SIN2, field_axis=0),
    dict(shape=(16, 32), n_t=4, block=(8, 8), h=0.25, periodic=True, pulse=PULSE_BOTH),
]


@pytest.mark.parametrize("cfg", SWEEP_CASES, ids=lambda c: f"{c['shape']}-{c['block']}-nt{c['n_t']}")
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("time_factor", ["shared", "stored"])
def test_sweep_parity(cfg, adjoint, precision, time_factor):
    """One colour, then the other, against the oracle's plain-loop local solves.

    FP64: the subvolume solve goes through an orthogonal eigenbasis and a
    pivoted (n_t+1)-system inverse, each backward stable, and the local KKT
    blocks have condition numbers below ~1e2, so the correction agrees to
    1e-11 of its size.  Mixed: the same in FP32, 1e-4 of its size.
    """
    case = Case(**cfg)
    note(f"sweep adjoint={adjoint} {precision} {time_factor} {case}")
    t0 = 0.2
    sysm = kkt.StepSystem(case.grid, case.v0, case.n_t, case.dt, t0, case.field)
    K = sysm.K.conj().T.tocsr() if adjoint else sysm.K
    c, lam = case.random_state()
    if adjoint:
        g = case.psi0
        b = A.adjoint_rhs(sysm, g)
    else:
        b = kkt.rhs(sysm, case.psi0)
    x = kkt.join(c, lam)
    # exact subvolume solves: FP32 corrections of the field defect to 1e-5
    prop = case.prop(precision=precision, n_inner=(6 if case.field is not None else -1), time_factor=time_factor,
                     inner_tol=EXACT_INNER_TOL[precision])
    if adjoint:
        prop.set_adjoint_state(t0, t_c(case.psi0), t_c(c), t_c(lam))
    else:
        prop.set_state(t0, t_c(case.psi0), t_c(c), t_c(lam))
    blocks = G.blocks(case.grid, case.block)
    rel = 1e-11 if precision == "fp64" else 1e-4
    for colour in (0, 1):
        x_ref = relax.reference_sweep_colour(K, b, x, blocks, colour, case.npts, case.n_t)
        prop.relax_sweep(colour)
        cg, lg = prop.get_state()
        x_gpu = np.concatenate([n(cg), n(lg)])
        delta = np.abs(x_ref - x).max()
        err = np.abs(x_gpu - x_ref)
        assert err.max() <= rel * delta + 64 * EPS * np.abs(x).max(), (colour, err.max(), delta)
        moved = np.zeros(x.size, bool)
        for col, pts in blocks:
            if col == colour:
                moved[relax.block_rows(pts, case.npts, case.n_t)] = True
        assert np.array_equal(x_gpu[~moved], x[~moved])
        x = x_gpu
    prop.close()
