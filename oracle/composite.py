"""Non-uniform subdivision of the multigrid tree (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Multigrid Relaxation": the tree of elements need not subdivide every
volume equally; where the function has little detail a coarse element stands
for its children, a compressed representation related to a wavelet
decomposition.

Readings (the paper states the idea only):

* Hierarchy: the coarse spaces are those of piecewise-constant interpolation
  I (each child takes its parent's value) with the averaging restriction R
  (R I = identity), and each coarse step operator is the Galerkin product
  K_c = R K I of the finer one (Eq. (correction_fine): the coarse correction
  solves the projected problem).  With this pair the decomposition
  psi = I R psi + (psi - I R psi) is the Haar one: the two parts are
  orthogonal, and the detail psi - I R psi shows where the function has detail.
* Adaptive tree: the finest level is kept on a set A of its subvolumes (the
  refined ones); elsewhere the parent level is the leaf.  The state of a step
  is x = x0 + E_A y_A + I y_c (x0: the initial guess; E_A: the unknowns of the
  refined subvolumes; I y_c: a coarse correction, interpolated everywhere),
  and the step equations hold on the refined rows and in projection on the
  coarse level,

      E_A^T (b - K x) = 0,    R (b - K x) = 0.

  V-cycles that relax the finest level only on A (every coarser level in
  full) reach exactly this state: relaxation annihilates the residual on the
  volumes it relaxes, and the coarse correction vanishes once the projected
  residual does.  With A = every subvolume it is the step's own solution.

Parity: pinned by the closed form of the Galerkin operator (the step operator
of the coarse grid with half the kinetic coefficient per level), the Haar
identities, the two limits of the composite state (every subvolume refined:
the direct solution; none: the Galerkin coarse solve) and the convergence of
the masked V-cycles to the directly solved composite state
(tests/test_oracle_composite.py).
"""
import numpy as np
import scipy.sparse as sp

from . import grid as gmod
from . import kkt
from . import relax


def _kkt_transfer(M, n_t):
    """A point-space transfer (rows x cols) on the (c, lambda) layout of the step
    system: c is [point][n_t] (point-major), then lambda per point."""
    return sp.block_diag([sp.kron(M, sp.identity(n_t)), M], format="csr")


def galerkin_hierarchy(grid, v0, n_t, dt, block, levels, t0=0.0, field=None):
    """Levels whose coarse operators are R K I (piecewise-constant I).  Each Level
    is relax.Level with R and I set; its system is the rediscretised StepSystem
    of the coarse grid (time matrices, U weights) with K replaced by the
    Galerkin product."""
    out = []
    g, v = grid, np.asarray(v0, float).ravel()
    K = None
    for l in range(levels):
        sysm = kkt.StepSystem(g, v, n_t, dt, t0, field)
        if K is not None:
            sysm.K = K
        lev = relax.Level(g, v, sysm, gmod.blocks(g, block))
        if l + 1 < levels:
            lev.R = gmod.restriction(g)
            lev.I = gmod.interpolation(g, "constant")
            Rk = _kkt_transfer(lev.R, n_t)
            Ik = _kkt_transfer(lev.I, n_t)
            K = (Rk @ sysm.K @ Ik).tocsr()
            v = lev.R @ v
            g = gmod.coarsen_grid(g)
        out.append(lev)
    return out


def haar_detail(grid, psi, block):
    """Per subvolume of the partition `block` (in the order of grid.blocks), the
    detail energy sum_j |psi_j - (I R psi)_j|^2 over its points (I
    piecewise-constant, R the average of the 2^d children)."""
    R = gmod.restriction(grid)
    I = gmod.interpolation(grid, "constant")
    psi = np.asarray(psi, complex).ravel()
    d = np.abs(psi - I @ (R @ psi)) ** 2
    return np.array([d[pts].sum() for _, pts in gmod.blocks(grid, block)])


def _active_rows(lev, active):
    P, n_t = lev.grid.npts, lev.system.n_t
    rows = []
    for k, (_, pts) in enumerate(lev.blocks):
        if active[k]:
            rows.append(relax.block_rows(pts, P, n_t))
    return np.sort(np.concatenate(rows)) if rows else np.zeros(0, int)


def composite_solve(levels, b, x0, active):
    """The composite state of the two finest levels: x = x0 + E_A y_A + I y_c
    with E_A^T r = 0 and R r = 0 (r = b - K x), solved directly (dense least
    squares: the columns of E_A and I overlap where a coarse function lies
    inside the refined subvolumes, but x is unique).  Returns (x, the largest
    residual of the equations relative to |T r0|)."""
    lev = levels[0]
    K = lev.system.K.toarray()
    n_t = lev.system.n_t
    rows = _active_rows(lev, active)
    n = K.shape[0]
    E = np.zeros((n, rows.size))
    E[rows, np.arange(rows.size)] = 1.0
    Ik = _kkt_transfer(lev.I, n_t).toarray()
    Rk = _kkt_transfer(lev.R, n_t).toarray()
    S = np.hstack([E, Ik])
    T = np.vstack([E.T, Rk])
    r0 = b - K @ x0
    A = T @ K @ S
    y, *_ = np.linalg.lstsq(A, T @ r0, rcond=None)
    x = x0 + S @ y
    eq = T @ (b - K @ x)
    return x, np.abs(eq).max() / max(np.abs(T @ r0).max(), 1e-300)


def composite_norm(levels, r, active):
    """N of the composite equations: the U-weighted residual norm on the refined
    rows plus that of the projected residual on the coarse level."""
    lev = levels[0]
    rows = _active_rows(lev, active)
    mask = np.zeros(r.size, bool)
    mask[rows] = True
    fine = kkt.residual_norm(lev.system, np.where(mask, r, 0.0))
    return fine + kkt.residual_norm(levels[1].system, relax.restrict(lev, r))
