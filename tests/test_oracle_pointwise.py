"""Pins of the oracle's pointwise checkers against the assembled step system.

``kkt.residual_at_points`` and ``kkt.block_system`` are what the full-size GPU
tests compare with (grids too large to assemble).  Here they are compared, on
grids small enough to assemble, with the rows of b - K x and with the
sub-matrix K[rows][:, rows] of the Kronecker assembly, which is itself pinned
entry by entry to the action by brute force (tests/test_oracle_kkt.py).
A wrong neighbour wrap, dipole axis, sign, time-block orientation, box order
or multiplier placement in either checker fails here.
"""
import numpy as np
import pytest

from oracle import kkt
from oracle import grid as G
from oracle import relax
from oracle import timebasis as tb


FIELD = tb.pulse_sin2_cos(0.7, 2.3, 1.5)

RESID_CASES = [
    # shape, periodic, field, field_axis, mass, n_t
    ((11,), False, None, -1, 1.0, 4),
    ((12,), True, FIELD, -1, 1.0, 3),
    ((6, 5), False, FIELD, -1, 1.0, 5),
    ((6, 5), False, FIELD, 0, 1.3, 4),
    ((4, 6), True, FIELD, -1, 1.0, 3),
    ((3, 4, 5), False, FIELD, -1, 0.8, 3),
    ((4, 4, 4), True, FIELD, 1, 1.0, 2),
]


def _state(P, n_t, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(P, n_t)) + 1j * rng.normal(size=(P, n_t))
    lam = rng.normal(size=P) + 1j * rng.normal(size=P)
    psi0 = rng.normal(size=P) + 1j * rng.normal(size=P)
    g = rng.normal(size=P) + 1j * rng.normal(size=P)
    v0 = rng.normal(size=P)
    return c, lam, psi0, g, v0


@pytest.mark.parametrize("case", RESID_CASES)
def test_residual_at_points_equals_rows_of_assembled_residual(case):
    shape, periodic, field, fax, mass, n_t = case
    grid = G.Grid(shape, 0.35, periodic=periodic, mass=mass, field_axis=fax)
    P = grid.npts
    dt, t0 = 0.09, 0.4
    c, lam, psi0, _, v0 = _state(P, n_t, 5)
    sysm = kkt.StepSystem(grid, v0, n_t, dt, t0, field)
    r = kkt.residual(sysm.K, kkt.rhs(sysm, psi0), kkt.join(c, lam))
    rho_ref, sig_ref = kkt.split(r, P, n_t)
    pts = np.random.default_rng(1).permutation(P)
    rho, sig = kkt.residual_at_points(grid, v0, n_t, dt, t0, field, c, lam, psi0, pts)
    scale = np.abs(r).max()
    np.testing.assert_allclose(rho, rho_ref[pts], rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(sig, sig_ref[pts], rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("case", RESID_CASES)
def test_adjoint_residual_at_points_equals_rows_of_conjugate_transpose(case):
    """Adjoint: b - K^H mu with b = E^H g (g_j on every row (j, n), since every
    T_n is 1 at the end of the step) and zero constraint rows."""
    shape, periodic, field, fax, mass, n_t = case
    grid = G.Grid(shape, 0.35, periodic=periodic, mass=mass, field_axis=fax)
    P = grid.npts
    dt, t0 = 0.09, 0.4
    mu_c, mu_l, _, g, v0 = _state(P, n_t, 9)
    sysm = kkt.StepSystem(grid, v0, n_t, dt, t0, field)
    e_end = tb.end_values(n_t)
    b = kkt.join(np.outer(g, e_end), np.zeros(P))
    KH = sysm.K.conj().T.tocsr()
    r = b - KH @ kkt.join(mu_c, mu_l)
    rho_ref, sig_ref = kkt.split(r, P, n_t)
    pts = np.arange(P)[::-1]
    rho, sig = kkt.residual_at_points(grid, v0, n_t, dt, t0, field, mu_c, mu_l, np.zeros(P), pts,
                                      stat_rhs=g, adjoint=True)
    scale = np.abs(r).max()
    np.testing.assert_allclose(rho, rho_ref[pts], rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(sig, sig_ref[pts], rtol=0, atol=1e-13 * scale)


def test_residual_at_points_vanishes_at_direct_solution():
    grid = G.Grid((7, 6), 0.3)
    P, n_t = grid.npts, 4
    _, _, psi0, _, v0 = _state(P, n_t, 2)
    psi1, x, sysm = kkt.step(grid, v0, psi0, n_t, 0.05, 0.2, FIELD)
    c, lam = kkt.split(x, P, n_t)
    rho, sig = kkt.residual_at_points(grid, v0, n_t, 0.05, 0.2, FIELD, c, lam, psi0, range(P))
    assert np.abs(rho).max() < 1e-12 and np.abs(sig).max() < 1e-12


BOX_CASES = [
    # grid shape, box lower corner, box shape, field axis
    ((8, 8), (2, 3), (3, 2), -1),      # interior
    ((8, 8), (0, 4), (2, 4), -1),      # on an edge
    ((8, 8), (6, 0), (2, 2), 0),       # in a corner, field along axis 0
    ((9,), (3,), (4,), -1),            # 1D interior
    ((6, 5, 7), (1, 0, 3), (2, 3, 4), -1),   # 3D, touching one face
    ((6, 5, 7), (4, 2, 5), (2, 3, 2), 1),    # 3D corner region, field along axis 1
]


@pytest.mark.parametrize("case", BOX_CASES)
def test_block_system_is_submatrix_of_assembled_K(case):
    shape, lo, bshape, fax = case
    grid = G.Grid(shape, 0.3, field_axis=fax)
    n_t, dt, t0 = 3, 0.07, 0.25
    v0 = np.random.default_rng(4).normal(size=grid.npts)
    sysm = kkt.StepSystem(grid, v0, n_t, dt, t0, FIELD)
    idx = np.arange(grid.npts).reshape(shape)
    sl = tuple(slice(a, a + b) for a, b in zip(lo, bshape))
    pts = idx[sl].ravel()
    # an arbitrary order of the box's points: rows follow the order given
    pts = pts[np.random.default_rng(6).permutation(len(pts))]
    Kb = kkt.block_system(grid, v0, n_t, dt, t0, FIELD, pts)
    rows = relax.block_rows(pts, grid.npts, n_t)
    Kref = sysm.K[rows][:, rows].toarray()
    np.testing.assert_allclose(Kb, Kref, rtol=0, atol=1e-14 * np.abs(Kref).max())


def test_block_system_rejects_points_that_are_not_a_box():
    grid = G.Grid((6, 6), 0.3)
    with pytest.raises(ValueError):
        kkt.block_system(grid, np.zeros(36), 2, 0.05, 0.0, None, [0, 1, 7, 14])


# ---------------------------------------------------------------------------
# Boundary rows of the tensor-linear interpolation
# ---------------------------------------------------------------------------

def _ghost(gc, a, side):
    """Coordinate of the coarse ghost cell one spacing outside axis a."""
    x = gc.axis_coords(a)
    return x[0] - gc.h if side == 0 else x[-1] + gc.h


@pytest.mark.parametrize("shape", [(12,), (8, 6), (4, 6, 8)])
def test_linear_interpolation_boundary_rows_treat_ghosts_as_zero(shape):
    """With zero Dirichlet ghosts, the interpolation reproduces exactly every
    product of per-axis linear functions that vanish at the ghost cells the
    stencil reads: for each choice of (lower, upper) ghost per axis, the
    fine points on that side (and all interior ones) are exact.  Every fine
    point, boundary rows included, is covered by one choice."""
    g = G.Grid(shape, 0.25)
    gc = G.coarsen_grid(g)
    I = G.interpolation(g, "linear")
    X = g.coords()
    Xc = gc.coords()
    covered = np.zeros(g.n, bool)
    for sides in np.ndindex(*([2] * g.dim)):
        f = np.ones(g.n)
        fc = np.ones(gc.n)
        ok = np.ones(g.n, bool)
        for a, s in enumerate(sides):
            x0 = _ghost(gc, a, s)
            f = f * (X[a] - x0)
            fc = fc * (Xc[a] - x0)
            # the fine points next to the other side read the other ghost
            edge = [slice(None)] * g.dim
            edge[a] = g.n[a] - 1 if s == 0 else 0
            ok[tuple(edge)] = False
        fine = (I @ fc.ravel()).reshape(g.n)
        np.testing.assert_allclose(fine[ok], f[ok], rtol=0, atol=1e-12 * np.abs(f).max())
        covered |= ok
    assert covered.all()


def test_linear_interpolation_lower_boundary_row_weights():
    """The first fine point takes 3/4 of the first coarse cell and nothing else;
    the last takes 3/4 of the last (a linear function through zero at the ghost)."""
    g = G.Grid((10,), 0.5)
    I = G.interpolation(g, "linear").toarray()
    np.testing.assert_array_equal(I[0], np.eye(5)[0] * 0.75)
    np.testing.assert_array_equal(I[-1], np.eye(5)[-1] * 0.75)


@pytest.mark.parametrize("shape", [(12,), (8, 6)])
def test_periodic_linear_interpolation_commutes_with_shifts(shape):
    """Periodic wrap: shifting the coarse grid by one cell shifts the fine result
    by two points (so the wrap rows equal the interior ones up to translation),
    and constants are reproduced."""
    g = G.Grid(shape, 0.25, periodic=True)
    gc = G.coarsen_grid(g)
    I = G.interpolation(g, "linear")
    u = np.random.default_rng(0).normal(size=gc.n)
    base = (I @ u.ravel()).reshape(g.n)
    for a in range(g.dim):
        shifted = (I @ np.roll(u, 1, axis=a).ravel()).reshape(g.n)
        np.testing.assert_allclose(shifted, np.roll(base, 2, axis=a), rtol=0, atol=1e-14)
    np.testing.assert_allclose(I @ np.ones(gc.npts), np.ones(g.npts), rtol=0, atol=1e-15)
