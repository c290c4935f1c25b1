"""Oracle grid, transfers and subvolumes against closed forms and invariants."""
import numpy as np
import pytest

from oracle import grid as G


def test_coords_are_cell_centred():
    g = G.Grid((256,), 40.0 / 256)
    x = g.axis_coords(0)
    np.testing.assert_allclose([x[0], x[-1]], [-20 + g.h / 2, 20 - g.h / 2], atol=1e-13)


def test_laplacian_exact_on_quadratic_interior():
    g = G.Grid((12, 10), 0.3)
    X, Y = g.coords()
    u = (2 * X ** 2 - Y ** 2 + X * Y).ravel()
    Lu = (G.laplacian(g) @ u).reshape(g.n)
    np.testing.assert_allclose(Lu[1:-1, 1:-1], 2.0, atol=1e-11)


def test_kinetic_dirichlet_eigenvalues():
    n, h, m = 17, 0.4, 1.7
    w = np.linalg.eigvalsh(G.kinetic(G.Grid((n,), h, mass=m)).toarray())
    ref = np.sort((1 - np.cos(np.arange(1, n + 1) * np.pi / (n + 1))) / (m * h * h))
    np.testing.assert_allclose(w, ref, atol=1e-12)


def test_kinetic_periodic_plane_wave():
    g = G.Grid((16, 8), 0.5, periodic=True)
    X, Y = g.coords()
    kx, ky = 2 * np.pi * 3 / (16 * 0.5), 2 * np.pi * 1 / (8 * 0.5)
    u = np.exp(1j * (kx * X + ky * Y)).ravel()
    E = ((1 - np.cos(kx * 0.5)) + (1 - np.cos(ky * 0.5))) / 0.25
    np.testing.assert_allclose(G.kinetic(g) @ u, E * u, atol=1e-12)


@pytest.mark.parametrize("shape", [(8,), (4, 6), (4, 2, 6)])
def test_projection_times_constant_interpolation_is_identity(shape):
    g = G.Grid(shape, 0.2)
    R = G.restriction(g).toarray()
    I = G.interpolation(g, "constant").toarray()
    np.testing.assert_allclose(R @ I, np.eye(R.shape[0]), atol=1e-15)
    # I R is a projector with eigenvalues 1 (coarse-representable) and 0.
    IR = I @ R
    np.testing.assert_allclose(IR @ IR, IR, atol=1e-15)
    np.testing.assert_allclose(np.trace(IR), R.shape[0], atol=1e-12)


def test_linear_interpolation_reproduces_linear_functions_inside():
    g = G.Grid((16, 12), 0.25)
    gc = G.coarsen_grid(g)
    X, Y = g.coords()
    Xc, Yc = gc.coords()
    I = G.interpolation(g, "linear")
    fine = (I @ (1.5 * Xc - 0.5 * Yc + 2).ravel()).reshape(g.n)
    np.testing.assert_allclose(fine[1:-1, 1:-1], (1.5 * X - 0.5 * Y + 2)[1:-1, 1:-1], atol=1e-12)


def test_coarse_centres_average_children_and_restriction_preserves_linear():
    g = G.Grid((8, 4, 6), 0.3)
    gc = G.coarsen_grid(g)
    R = G.restriction(g)
    for a in range(3):
        np.testing.assert_allclose(R @ g.coords()[a].ravel(), gc.coords()[a].ravel(), atol=1e-14)
    np.testing.assert_allclose(gc.h, 0.6)


@pytest.mark.parametrize("shape,block,periodic", [((16,), (8,), False), ((16, 8), (4, 4), False),
                                                   ((8, 8, 8), (4, 2, 4), False), ((16, 8), (4, 4), True)])
def test_blocks_partition_and_same_colour_blocks_do_not_couple(shape, block, periodic):
    g = G.Grid(shape, 0.2, periodic=periodic)
    bl = G.blocks(g, block)
    allpts = np.sort(np.concatenate([p for _, p in bl]))
    np.testing.assert_array_equal(allpts, np.arange(g.npts))
    L = G.laplacian(g).tocsr()
    owner = np.empty(g.npts, int)
    colour = np.empty(g.npts, int)
    for k, (c, p) in enumerate(bl):
        owner[p] = k
        colour[p] = c
    rows, cols = L.nonzero()
    cross = owner[rows] != owner[cols]
    assert np.all(colour[rows[cross]] != colour[cols[cross]])


def test_periodic_needs_even_block_count():
    with pytest.raises(ValueError):
        G.blocks(G.Grid((12,), 0.1, periodic=True), (4,))
