"""Finite-difference spatial grid, level hierarchy and subvolumes (oracle).

Readings (the paper's own test uses Legendre finite elements):

* one spatial function per grid point, cell-centred coordinates
  x_a(i) = (i - (n_a - 1)/2) h along every axis a; the linear point index is
  C order over the axes (last axis fastest);
* H0 = T = -(1/2m) Lap_h with the (2d+1)-point Laplacian; the values one
  spacing outside the grid are zero (Dirichlet) or wrap around (periodic);
* the dipole coordinate z is the coordinate along ``field_axis``;
* level l+1 halves every axis and doubles h (Sec. "Multigrid Relaxation":
  each element of level l+1 is the union of 2^d elements of level l);
  the coarse potential is the average of its 2^d children;
* projection to the coarse level (P of Eq. (residual_rough)) is the average
  of the 2^d children; interpolation (I of Eq. (correction_fine)) is either
  piecewise constant, which makes P I the identity exactly as the paper asks,
  or the cell-centred tensor-linear stencil (3/4, 1/4 per axis);
* subvolumes are non-overlapping boxes of points, coloured by the parity of
  the sum of their box coordinates: two boxes of one colour never share a
  face, so a (2d+1)-point stencil never couples them (Sec. "Iterative
  relaxation to the least action solution": relaxations over non-overlapping
  volumes of a local Lagrangian are independent).

Parity: pinned (tests/test_oracle_grid.py; the Dirichlet and periodic boundary
rows of the interpolation in tests/test_oracle_pointwise.py).
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Grid:
    n: tuple            # points per axis, slowest axis first
    h: float
    periodic: bool = False
    mass: float = 1.0
    field_axis: int = -1

    @property
    def dim(self):
        return len(self.n)

    @property
    def npts(self):
        return int(np.prod(self.n))

    def axis_coords(self, a):
        na = self.n[a]
        return (np.arange(na) - 0.5 * (na - 1)) * self.h

    def coords(self):
        """List of d arrays of shape n: coordinate along each axis."""
        return np.meshgrid(*[self.axis_coords(a) for a in range(self.dim)], indexing="ij")

    def z(self):
        """Dipole coordinate of every point (flattened, C order)."""
        return self.coords()[self.field_axis % self.dim].ravel()


def _second_difference_1d(n, h, periodic):
    main = -2.0 * np.ones(n)
    off = np.ones(n - 1)
    D = sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="lil")
    if periodic and n > 2:
        D[0, n - 1] = 1.0
        D[n - 1, 0] = 1.0
    elif periodic and n == 2:
        D[0, 1] = 2.0
        D[1, 0] = 2.0
    return sp.csr_matrix(D) / (h * h)


def laplacian(grid):
    """Sparse (2d+1)-point Laplacian over the whole grid."""
    d = grid.dim
    L = sp.csr_matrix((grid.npts, grid.npts))
    for a in range(d):
        mats = [sp.identity(grid.n[b], format="csr") for b in range(d)]
        mats[a] = _second_difference_1d(grid.n[a], grid.h, grid.periodic)
        term = mats[0]
        for m in mats[1:]:
            term = sp.kron(term, m, format="csr")
        L = L + term
    return sp.csr_matrix(L)


def kinetic(grid):
    """T = -(1/2m) Lap_h."""
    return (-0.5 / grid.mass) * laplacian(grid)


def hamiltonian(grid, v0):
    """H = T + diag(V0) (the static part of the local Hamiltonian)."""
    return sp.csr_matrix(kinetic(grid) + sp.diags(np.asarray(v0, dtype=float).ravel()))


# ---------------------------------------------------------------------------
# Level hierarchy
# ---------------------------------------------------------------------------

def coarsen_grid(grid):
    for na in grid.n:
        if na % 2:
            raise ValueError("every axis must be even to coarsen")
    return Grid(tuple(na // 2 for na in grid.n), 2.0 * grid.h, grid.periodic,
                grid.mass, grid.field_axis)


def restriction(grid):
    """Coarse <- fine: average of the 2^d children (sparse, coarse x fine)."""
    mats = []
    for na in grid.n:
        nc = na // 2
        R = sp.lil_matrix((nc, na))
        for J in range(nc):
            R[J, 2 * J] = 0.5
            R[J, 2 * J + 1] = 0.5
        mats.append(sp.csr_matrix(R))
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return sp.csr_matrix(out)


def interpolation(grid, kind="linear"):
    """Fine <- coarse, sparse (fine x coarse).  ``grid`` is the fine grid.

    kind="constant": each child takes its parent's value.
    kind="linear":   cell-centred tensor-linear, per axis the child nearer a
                     coarse neighbour takes 3/4 of its parent and 1/4 of that
                     neighbour (zero outside a Dirichlet grid, wrapped when
                     periodic).
    """
    mats = []
    for na in grid.n:
        nc = na // 2
        I = sp.lil_matrix((na, nc))
        for J in range(nc):
            for child, nb in ((2 * J, J - 1), (2 * J + 1, J + 1)):
                if kind == "constant":
                    I[child, J] += 1.0
                elif kind == "linear":
                    I[child, J] += 0.75
                    if grid.periodic:
                        I[child, nb % nc] += 0.25
                    elif 0 <= nb < nc:
                        I[child, nb] += 0.25
                else:
                    raise ValueError(kind)
        mats.append(sp.csr_matrix(I))
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return sp.csr_matrix(out)


# ---------------------------------------------------------------------------
# Subvolumes
# ---------------------------------------------------------------------------

def blocks(grid, block):
    """List of (colour, point-index array) for the box partition ``block``."""
    block = tuple(block)
    if len(block) != grid.dim:
        raise ValueError("block rank must equal grid rank")
    for na, ba in zip(grid.n, block):
        if na % ba:
            raise ValueError("block must divide the grid")
    nb = [na // ba for na, ba in zip(grid.n, block)]
    if grid.periodic and any(k % 2 and k > 1 for k in nb):
        raise ValueError("a periodic grid needs an even number of blocks per axis")
    idx = np.arange(grid.npts).reshape(grid.n)
    out = []
    for bc in np.ndindex(*nb):
        sl = tuple(slice(c * b, (c + 1) * b) for c, b in zip(bc, block))
        out.append((int(sum(bc)) % 2, idx[sl].ravel().copy()))
    return out
