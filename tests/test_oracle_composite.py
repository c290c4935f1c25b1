"""The adaptive tree's oracle (oracle/composite.py) pinned against closed forms,
identities and its own limits (Sec. "Multigrid Relaxation")."""
import numpy as np
import pytest

from oracle import composite as C
from oracle import grid as G
from oracle import kkt, relax
from oracle import timebasis as tb


def _setup(shape, h=0.3, periodic=False):
    g = G.Grid(shape, h, periodic, 1.0, 0)
    X = g.coords()
    r2 = sum(x * x for x in X).ravel()
    v0 = -1.0 / np.sqrt(r2 + 1.0)
    rng = np.random.default_rng(len(shape))
    psi0 = np.exp(-r2 / 2.0) * np.exp(1j * rng.uniform(0, 2 * np.pi, g.npts))
    return g, v0, psi0


@pytest.mark.parametrize("shape,periodic", [((16,), False), ((8, 12), False), ((8, 8), True), ((4, 8, 12), False)])
def test_galerkin_operator_is_the_coarse_step_operator_with_half_the_kinetic_coefficient(shape, periodic):
    """R K I with piecewise-constant I: the coarse step operator with the potential
    averaged over children, the field at the coarse cell centres and the kinetic
    term of spacing H / sqrt(2) (twice the rediscretised one at spacing H = 2h):
    per axis, the average over two children of the second difference of a
    piecewise-constant function is half the coarse second difference over h^2."""
    pulse = tb.pulse_sin2_cos(0.3, 0.7, 1.0)
    g, v0, _ = _setup(shape, periodic=periodic)
    n_t, dt, t0 = 4, 0.05, 0.2
    levels = C.galerkin_hierarchy(g, v0, n_t, dt, (2,) * len(shape), 2, t0, pulse)
    gc = G.coarsen_grid(g)
    coarse = levels[1].system
    z_c = gc.z()
    g_kin = G.Grid(gc.n, gc.h / np.sqrt(2.0), gc.periodic, gc.mass, gc.field_axis)
    ref = kkt.assemble(g_kin, levels[1].v0, coarse.U, coarse.Q, coarse.s, coarse.W, z=z_c)
    assert abs(coarse.K - ref).max() < 1e-13 * abs(ref).max()
    # and the potential is the children's average
    np.testing.assert_allclose(levels[1].v0, G.restriction(g) @ v0, atol=1e-15)


@pytest.mark.parametrize("shape", [(16,), (8, 12), (4, 4, 8)])
def test_haar_decomposition_is_orthogonal_and_local(shape):
    g, _, psi = _setup(shape)
    R = G.restriction(g)
    I = G.interpolation(g, "constant")
    block = (2,) * len(shape)
    det = C.haar_detail(g, psi, block)
    # ||psi||^2 = 2^d ||R psi||^2 + sum of details (orthogonal parts)
    lhs = np.sum(np.abs(psi) ** 2)
    rhs = 2 ** len(shape) * np.sum(np.abs(R @ psi) ** 2) + det.sum()
    assert abs(lhs - rhs) < 1e-12 * lhs
    # a piecewise-constant function has no detail; changing one subvolume's
    # points changes only that subvolume's detail
    assert np.abs(C.haar_detail(g, I @ (R @ psi), block)).max() < 1e-28 * lhs
    pts = G.blocks(g, block)[1][1]
    psi2 = psi.copy()
    psi2[pts] *= 1.7
    det2 = C.haar_detail(g, psi2, block)
    changed = np.flatnonzero(np.abs(det2 - det) > 1e-14 * lhs)
    assert list(changed) == [1]


def _levels(shape, block, nlev, active_frac=None, n_t=4, dt=0.05):
    g, v0, psi0 = _setup(shape, h=0.25)
    levels = C.galerkin_hierarchy(g, v0, n_t, dt, block, nlev)
    lev = levels[0]
    b = kkt.rhs(lev.system, psi0)
    x0 = kkt.initial_guess(lev.system, psi0)
    r2 = sum(x * x for x in g.coords()).ravel()
    act = np.array([np.sqrt(r2[pts].mean()) < active_frac for _, pts in lev.blocks]) if active_frac else None
    return levels, b, x0, act


def test_composite_state_limits():
    """Every subvolume refined: the direct solution of the step; none: x0 plus the
    interpolated Galerkin coarse solve of the projected residual."""
    levels, b, x0, _ = _levels((8, 8), (2, 2), 2)
    lev = levels[0]
    nb = len(lev.blocks)
    x_all, eq = C.composite_solve(levels, b, x0, np.ones(nb, bool))
    x_dir = kkt.solve_direct(lev.system.K, b)
    assert eq < 1e-12
    assert np.abs(x_all - x_dir).max() < 1e-10 * np.abs(x_dir).max()
    x_none, eq = C.composite_solve(levels, b, x0, np.zeros(nb, bool))
    r0 = b - lev.system.K @ x0
    yc = kkt.solve_direct(levels[1].system.K, relax.restrict(lev, r0))
    assert eq < 1e-12
    assert np.abs(x_none - (x0 + relax.prolong(lev, yc))).max() < 1e-10 * np.abs(x_none).max()


@pytest.mark.parametrize("shape,block,nlev", [((32,), (4,), 3), ((16, 16), (4, 4), 3)])
def test_masked_vcycles_converge_to_the_composite_state(shape, block, nlev):
    """V-cycles relaxing the finest level only on the refined subvolumes (the
    central ones), every coarser level in full and the coarsest directly, reach
    the composite state to 1e-9, and the composite norm falls by 1e-9."""
    levels, b, x0, act = _levels(shape, block, nlev, active_frac=1.6)
    assert 0 < act.sum() < act.size
    x_ref, eq = C.composite_solve(levels, b, x0, act)
    assert eq < 1e-11
    x = x0.copy()
    n0 = C.composite_norm(levels, b - levels[0].system.K @ x, act)
    for _ in range(20):
        x = relax.reference_vcycle(levels, 0, x, b, nu_coarse=0, coarse_direct=True, active=act)
    n = C.composite_norm(levels, b - levels[0].system.K @ x, act)
    assert np.sqrt(n / n0) < 1e-9
    assert np.abs(x - x_ref).max() < 1e-9 * np.abs(x_ref).max()


def test_galerkin_vcycles_converge_to_the_direct_solution():
    levels, b, x0, _ = _levels((16, 16), (4, 4), 3)
    x_dir = kkt.solve_direct(levels[0].system.K, b)
    x, hist = relax.solve_by_vcycles(levels, x0, b, tol=1e-11, max_cycles=20, nu_coarse=0, coarse_direct=True)
    assert hist[-1] <= 1e-11
    assert np.abs(x - x_dir).max() < 1e-9 * np.abs(x_dir).max()
