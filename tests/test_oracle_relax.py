"""Oracle relaxation and V-cycle semantics against properties the method fixes."""
import numpy as np
import pytest

from oracle import kkt, relax
from oracle import grid as G
from oracle import timebasis as tb


def _setup(shape=(32,), h=0.25, n_t=4, dt=0.05, seed=0, field=None, t0=0.0, periodic=False):
    g = G.Grid(shape, h, periodic=periodic)
    rng = np.random.default_rng(seed)
    r2 = sum(c ** 2 for c in g.coords()).ravel()
    v0 = -1.0 / np.sqrt(r2 + 1.0)
    psi0 = (np.exp(-r2 / 4) * np.exp(1j * rng.uniform(0, 2 * np.pi, g.npts)))
    sysm = kkt.StepSystem(g, v0, n_t, dt, t0, field)
    return g, v0, psi0, sysm


def test_whole_domain_block_is_direct_solve():
    g, v0, psi0, sysm = _setup((16,))
    b = kkt.rhs(sysm, psi0)
    x0 = kkt.initial_guess(sysm, psi0)
    bl = G.blocks(g, (16,))
    x1 = relax.reference_sweep_colour(sysm.K, b, x0, bl, 0, g.npts, 4)
    np.testing.assert_allclose(x1, kkt.solve_direct(sysm.K, b), atol=1e-13)


@pytest.mark.parametrize("shape,block", [((32,), (8,)), ((8, 8), (4, 4)), ((4, 4, 8), (2, 2, 4))])
def test_block_annihilation_and_untouched_exterior(shape, block):
    g, v0, psi0, sysm = _setup(shape, field=tb.pulse_sin2_cos(0.1, 0.5, 3.0), t0=0.7)
    b = kkt.rhs(sysm, psi0)
    x0 = kkt.initial_guess(sysm, psi0)
    bl = G.blocks(g, block)
    x1 = relax.reference_sweep_colour(sysm.K, b, x0, bl, 0, g.npts, 4)
    r1 = b - sysm.K @ x1
    moved = np.zeros(x0.size, bool)
    for col, pts in bl:
        if col == 0:
            rows = relax.block_rows(pts, g.npts, 4)
            assert np.abs(r1[rows]).max() < 1e-13
            moved[rows] = True
    assert np.all(x1[~moved] == x0[~moved])


def test_fixed_point():
    g, v0, psi0, sysm = _setup((8, 8))
    b = kkt.rhs(sysm, psi0)
    xd = kkt.solve_direct(sysm.K, b)
    xs = relax.reference_sweep(sysm.K, b, xd, G.blocks(g, (4, 4)), g.npts, 4)
    np.testing.assert_allclose(xs, xd, atol=1e-14)


def test_colour_order_invariance():
    g, v0, psi0, sysm = _setup((16, 8))
    b = kkt.rhs(sysm, psi0)
    x0 = kkt.initial_guess(sysm, psi0)
    bl = G.blocks(g, (4, 4))
    xa = relax.reference_sweep_colour(sysm.K, b, x0, bl, 1, g.npts, 4)
    n1 = sum(1 for c, _ in bl if c == 1)
    order = np.random.default_rng(1).permutation(n1)
    xb = relax.reference_sweep_colour_sequential(sysm.K, b, x0, bl, 1, g.npts, 4, order)
    np.testing.assert_allclose(xa, xb, atol=1e-15)


def test_residual_norm_non_increasing_per_sweep_in_regime():
    # 1D, h = 40/256, dt = 0.05: kappa = dt / (2 h^2) ~ 1.0, the configs' regime.
    g = G.Grid((256,), 40.0 / 256)
    x = g.coords()[0].ravel()
    sysm = kkt.StepSystem(g, 0.5 * x ** 2, 8, 0.05)
    psi0 = np.exp(-(x + 5) ** 2 / 2 + 1j * x)
    b = kkt.rhs(sysm, psi0)
    xk = kkt.initial_guess(sysm, psi0)
    bl = G.blocks(g, (8,))
    N0 = kkt.residual_norm(sysm, b - sysm.K @ xk)
    hist = [N0]
    for _ in range(8):
        xk = relax.reference_sweep(sysm.K, b, xk, bl, g.npts, 8)
        hist.append(kkt.residual_norm(sysm, b - sysm.K @ xk))
    for a, c in zip(hist, hist[1:]):
        assert c <= a + 1e-26 * N0
    assert hist[-1] < 1e-20 * N0


@pytest.mark.parametrize("levels,interp", [(2, "linear"), (3, "constant"), (3, "linear")])
def test_vcycles_converge_to_direct_solution(levels, interp):
    g, v0, psi0, sysm = _setup((32, 32), h=0.2, n_t=4, field=tb.pulse_sin2_cos(0.05, 0.057, 5.0), t0=1.0)
    H = relax.build_hierarchy(g, v0, 4, 0.05, (4, 4), levels, t0=1.0,
                              field=tb.pulse_sin2_cos(0.05, 0.057, 5.0), interp=interp)
    b = kkt.rhs(H[0].system, psi0)
    xs, hist = relax.solve_by_vcycles(H, kkt.initial_guess(H[0].system, psi0), b, tol=1e-12)
    xd = kkt.solve_direct(H[0].system.K, b)
    assert np.abs(xs - xd).max() <= 1e-10 * np.abs(xd).max()
    assert hist[-1] <= 1e-12


def test_adjoint_vcycles_converge_to_direct_adjoint():
    g, v0, psi0, sysm = _setup((16, 16), h=0.2, n_t=4)
    H = relax.build_hierarchy(g, v0, 4, 0.05, (4, 4), 2)
    rng = np.random.default_rng(3)
    b = rng.normal(size=H[0].system.size) + 1j * rng.normal(size=H[0].system.size)
    xs, hist = relax.solve_by_vcycles(H, np.zeros_like(b), b, tol=1e-12, adjoint=True)
    xd = kkt.solve_direct(H[0].system.K.conj().T.tocsr(), b)
    assert np.abs(xs - xd).max() <= 1e-10 * np.abs(xd).max()


def test_coarse_operator_is_rediscretisation():
    g, v0, psi0, sysm = _setup((8, 8), h=0.2, n_t=3)
    H = relax.build_hierarchy(g, v0, 3, 0.05, (2, 2), 2)
    gc = H[1].grid
    assert gc.n == (4, 4) and abs(gc.h - 0.4) < 1e-15
    np.testing.assert_allclose(H[1].v0, G.restriction(g) @ v0, atol=1e-15)


def test_coarsest_level_sweeps_reduce_residual_by_a_thousand():
    """On the 2D workload's coarsest level (512^2 coarsened four times: 32^2, h = 3.2,
    kappa = dt/(2h^2) ~ 0.0024) two colour sweeps reduce a random right-hand side's
    residual norm by at least 1e3, the reduction the iterated coarsest solve asks for:
    it needs at most two of its four sweeps there."""
    g = G.Grid((32, 32), 3.2)
    r2 = sum(c ** 2 for c in g.coords()).ravel()
    v0 = -1.0 / np.sqrt(r2 + 1.0)
    sysm = kkt.StepSystem(g, v0, 8, 0.05)
    rng = np.random.default_rng(2)
    b = rng.normal(size=sysm.size) + 1j * rng.normal(size=sysm.size)
    x = np.zeros_like(b)
    bl = G.blocks(g, (8, 8))
    N0 = kkt.residual_norm(sysm, b - sysm.K @ x)
    for _ in range(2):
        x = relax.reference_sweep(sysm.K, b, x, bl, g.npts, 8)
    assert kkt.residual_norm(sysm, b - sysm.K @ x) <= 1e-6 * N0


def _coarse_problem(n=16, h=3.2, n_t=8, block=(8, 8), seed=5):
    g = G.Grid((n, n), h)
    r2 = sum(c ** 2 for c in g.coords()).ravel()
    v0 = -1.0 / np.sqrt(r2 + 1.0)
    H = relax.build_hierarchy(g, v0, n_t, 0.05, block, 1)
    sysm = H[0].system
    rng = np.random.default_rng(seed)
    b = rng.normal(size=sysm.size) + 1j * rng.normal(size=sysm.size)
    return H[0], sysm, b


def test_iterated_coarsest_solve_converges_to_the_direct_coarse_solution():
    """Sweeps repeated to a tiny reduction reach the coarse system's direct
    solution, the coarse inverse of Eq. (correction_fine)."""
    lev, sysm, b = _coarse_problem(n=16, block=(4, 4))
    x, done = relax.coarsest_solve(lev, sysm.K, b, np.zeros_like(b), 60, coarse_reduction=1e-13)
    xd = kkt.solve_direct(sysm.K, b)
    assert np.abs(x - xd).max() <= 1e-11 * np.abs(xd).max()
    assert 1 < done < 60


def test_iterated_coarsest_solve_stops_at_the_first_sweep_that_meets_the_reduction():
    lev, sysm, b = _coarse_problem(n=16, block=(4, 4), seed=6)
    P, n_t = lev.grid.npts, sysm.n_t
    n0 = kkt.residual_norm(sysm, b)
    for red in (1e-2, 1e-5, 1e-8):
        x, done = relax.coarsest_solve(lev, sysm.K, b, np.zeros_like(b), 40, coarse_reduction=red)
        assert kkt.residual_norm(sysm, b - sysm.K @ x) <= red ** 2 * n0
        # the same number of plain sweeps, and one fewer: the count is the first that meets it
        xs = np.zeros_like(b)
        for k in range(done):
            prev = xs
            xs = relax.reference_sweep(sysm.K, b, xs, lev.blocks, P, n_t)
        np.testing.assert_array_equal(xs, x)
        assert done == 1 or kkt.residual_norm(sysm, b - sysm.K @ prev) > red ** 2 * n0
    # the cap: a reduction out of reach stops after nu_coarse sweeps
    _, done = relax.coarsest_solve(lev, sysm.K, b, np.zeros_like(b), 2, coarse_reduction=1e-30)
    assert done == 2


def test_vcycles_with_the_iterated_coarsest_solve_converge_like_a_direct_coarse_solve():
    """The reading of the coarsest solve: sweeps to a 1e-3 reduction in place of
    the direct coarse solve leave the V-cycle's convergence unchanged (2D
    soft-Coulomb, h = 0.2, N_t = 8, three levels, kappa = 0.625): every cycle's
    residual ratio within a factor 1.5 of the direct variant's."""
    g, v0, psi0, sysm = _setup((32, 32), h=0.2, n_t=8)
    H = relax.build_hierarchy(g, v0, 8, 0.05, (4, 4), 3)
    b = kkt.rhs(sysm, psi0)
    x0 = kkt.initial_guess(sysm, psi0)
    n0 = kkt.residual_norm(sysm, b - sysm.K @ x0)
    hist = {}
    for name, kw in (("direct", dict(coarse_direct=True)), ("iterated", dict(coarse_reduction=1e-3, nu_coarse=8))):
        x, h = x0, []
        for _ in range(4):
            x = relax.reference_vcycle(H, 0, x, b, 1, 1, **kw)
            h.append(np.sqrt(kkt.residual_norm(sysm, b - sysm.K @ x) / n0))
        hist[name] = np.array(h)
    assert hist["direct"][-1] < 1e-9
    assert np.all(hist["iterated"] <= 1.5 * hist["direct"]) and np.all(hist["direct"] <= 1.5 * hist["iterated"])


def _vcycle_history(dt, n=64, levels=3, cycles=8):
    """sqrt(N/N0) after each V-cycle of the 1D harmonic-oscillator step with
    h = 40/256 (kappa = dt / (2 h^2)), N_t = 8, subvolumes of 8 points."""
    h = 40.0 / 256
    grid = G.Grid((n,), h)
    x = (np.arange(n) - 0.5 * (n - 1)) * h
    v0 = 0.5 * x * x
    psi0 = np.exp(-0.5 * (x - 1.0) ** 2 + 0.5j * x)
    levs = relax.build_hierarchy(grid, v0, 8, dt, (8,), levels)
    sysm = levs[0].system
    _, hist = relax.solve_by_vcycles(levs, kkt.initial_guess(sysm, psi0), kkt.rhs(sysm, psi0), tol=1e-10,
                                     max_cycles=cycles, nu_coarse=2)
    return np.array(hist)


def test_halving_the_step_halves_both_dimensionless_parameters():
    """Without a field the step operator is affine in dt: the time coupling i Q
    does not depend on it, the kinetic and potential blocks (kappa, nu of Eq.
    (leastaction_dimensionless)) scale with it, so K(dt) - K(dt/2) = 2 (K(dt/2) - K(dt/4))
    and the dt-proportional part at dt/2 is half that at dt."""
    grid = G.Grid((12,), 0.3)
    v0 = np.linspace(-1.0, 2.0, 12)
    K = [kkt.StepSystem(grid, v0, 5, dt, 0.0, None).K.toarray() for dt in (0.4, 0.2, 0.1)]
    np.testing.assert_allclose(K[0] - K[1], 2.0 * (K[1] - K[2]), atol=1e-13)
    assert np.abs(K[0] - K[1]).max() > 0.01


def test_time_step_splitting_recovers_convergence():
    """The paper's remedy for a step outside the convergent regime: at kappa = 10.2
    and 5.1 (dt = 0.5, 0.25) the V-cycles' residual grows within a few cycles, at
    kappa = 2.56 (dt = 0.125, two halvings) it falls below 1e-6 in eight."""
    for dt in (0.5, 0.25):
        h = _vcycle_history(dt)
        assert h[-1] > 1.0 and np.any(np.diff(h[1:]) > 0)
    h = _vcycle_history(0.125)
    assert h[-1] < 1e-6 and np.all(np.diff(h) < 0)
