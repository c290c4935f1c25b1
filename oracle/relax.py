"""Reference semantics of subvolume relaxation and the V-cycle (oracle).

Sec. "Iterative relaxation to the least action solution": for a subvolume U
the relaxation finds the correction delta_phi_U with L_U delta_phi_U =
-L_U phi_bar, delta_phi(t0) = 0 and delta_phi = 0 on and outside the
subvolume boundary.  On the step system this is the local solve

    K_UU delta_U = (b - K x)_U,   x_U <- x_U + delta_U,

where U collects the rows and columns (j, m) and the multiplier rows j of the
subvolume's points; the initial-condition rows of the correction carry a
zero right-hand side once the trial state meets its own initial condition
(Eq. (ic_correction)), and in general the local right-hand side is the
residual of those rows.  Non-overlapping subvolumes of one colour do not
couple, so all of them are relaxed from the same state (one "colour").
A sweep is colour 0 followed by colour 1.

Sec. "Multigrid Relaxation", Eqs. (residual_rough) and (correction_fine): the
residual is projected to the coarse level, a correction is found there and
interpolated back.  The coarse operator is the step system rediscretised on
the coarse grid (same N_t, dt, field; potential averaged over children).
V-cycle with nu_pre / nu_post sweeps around the coarse correction.  The
coarsest-level solve (the coarse inverse of Eq. (correction_fine)) is either
nu_coarse sweeps, or sweeps repeated until the coarsest residual norm has
fallen by a given factor (at most nu_coarse of them), or the direct solve of
the coarsest system.

The adjoint variants use K^H at every level with the same transfers.

Parity: pinned by whole-domain block = direct solve, block annihilation,
fixed point, colour-order invariance and convergence of repeated V-cycles to
the direct solution (tests/test_oracle_relax.py).
"""
from dataclasses import dataclass

import numpy as np

from . import grid as gmod
from . import kkt


@dataclass
class Level:
    grid: gmod.Grid
    v0: np.ndarray
    system: kkt.StepSystem
    blocks: list
    R: object = None      # restriction to the next level (coarse x fine)
    I: object = None      # interpolation from the next level (fine x coarse)


def build_hierarchy(grid, v0, n_t, dt, block, levels, t0=0.0, field=None,
                    interp="linear"):
    out = []
    g, v = grid, np.asarray(v0, float).ravel()
    for l in range(levels):
        sysm = kkt.StepSystem(g, v, n_t, dt, t0, field)
        lev = Level(g, v, sysm, gmod.blocks(g, block))
        if l + 1 < levels:
            lev.R = gmod.restriction(g)
            lev.I = gmod.interpolation(g, interp)
            v = lev.R @ v
            g = gmod.coarsen_grid(g)
        out.append(lev)
    return out


def operator(level, adjoint=False):
    K = level.system.K
    return K.conj().T.tocsr() if adjoint else K


def block_rows(points, npts, n_t):
    pts = np.asarray(points)
    stat = (pts[:, None] * n_t + np.arange(n_t)[None, :]).ravel()
    return np.concatenate([stat, npts * n_t + pts])


def reference_sweep_colour(K, b, x, blocks, colour, npts, n_t):
    """Relax every block of one colour from the same state (plain loops)."""
    x = np.array(x, dtype=complex)
    r = b - K @ x
    for col, pts in blocks:
        if col != colour:
            continue
        rows = block_rows(pts, npts, n_t)
        Kbb = K[rows][:, rows].toarray()
        x[rows] += np.linalg.solve(Kbb, r[rows])
    return x


def reference_sweep_colour_sequential(K, b, x, blocks, colour, npts, n_t, order=None):
    """Same colour relaxed block after block, residual recomputed each time."""
    x = np.array(x, dtype=complex)
    sel = [pts for col, pts in blocks if col == colour]
    if order is not None:
        sel = [sel[i] for i in order]
    for pts in sel:
        rows = block_rows(pts, npts, n_t)
        r = b - K @ x
        Kbb = K[rows][:, rows].toarray()
        x[rows] += np.linalg.solve(Kbb, r[rows])
    return x


def reference_sweep(K, b, x, blocks, npts, n_t):
    x = reference_sweep_colour(K, b, x, blocks, 0, npts, n_t)
    return reference_sweep_colour(K, b, x, blocks, 1, npts, n_t)


def restrict(level, r):
    """Project a fine residual (rho, sigma) to the next level."""
    P, n_t = level.grid.npts, level.system.n_t
    rho, sig = kkt.split(r, P, n_t)
    return kkt.join(level.R @ rho, level.R @ sig)


def prolong(level, xc):
    """Interpolate a coarse correction (c, lambda) to this level."""
    Pc = level.R.shape[0]
    n_t = level.system.n_t
    cc, lc = kkt.split(xc, Pc, n_t)
    return kkt.join(level.I @ cc, level.I @ lc)


def coarsest_solve(lev, K, b, x, nu_coarse, coarse_reduction=None, direct=False):
    """The coarsest-level solve; returns (x, full sweeps done).

    direct: x = K^{-1} b.  coarse_reduction None: nu_coarse full sweeps.
    Otherwise full sweeps until sqrt(N / N0) <= coarse_reduction, N0 the norm
    at the start, checked after every sweep, at most nu_coarse sweeps.
    """
    P, n_t = lev.grid.npts, lev.system.n_t
    if direct:
        return kkt.solve_direct(K, b), 0
    if coarse_reduction is None:
        for _ in range(nu_coarse):
            x = reference_sweep(K, b, x, lev.blocks, P, n_t)
        return x, nu_coarse
    n0 = kkt.residual_norm(lev.system, b - K @ x)
    if n0 == 0.0:
        return x, 0
    done = 0
    for _ in range(nu_coarse):
        x = reference_sweep(K, b, x, lev.blocks, P, n_t)
        done += 1
        if kkt.residual_norm(lev.system, b - K @ x) <= coarse_reduction ** 2 * n0:
            break
    return x, done


def reference_vcycle(levels, l, x, b, nu_pre=1, nu_post=1, nu_coarse=2, adjoint=False, coarse_reduction=None,
                     coarse_direct=False, counts=None, active=None):
    """One V-cycle; counts (a list, optional) receives the coarsest sweeps done.
    active (optional, one flag per subvolume of the finest level): relax the
    finest level only on those subvolumes (an adaptive tree whose other volumes
    end on the next level; see composite.py)."""
    lev = levels[l]
    K = operator(lev, adjoint)
    P, n_t = lev.grid.npts, lev.system.n_t
    x = np.array(x, dtype=complex)
    if l == len(levels) - 1:
        x, done = coarsest_solve(lev, K, b, x, nu_coarse, coarse_reduction, coarse_direct)
        if counts is not None:
            counts.append(done)
        return x
    blocks = lev.blocks
    if l == 0 and active is not None:
        blocks = [bl for k, bl in enumerate(lev.blocks) if active[k]]
    for _ in range(nu_pre):
        x = reference_sweep(K, b, x, blocks, P, n_t)
    r = b - K @ x
    bc = restrict(lev, r)
    xc = np.zeros_like(bc)
    xc = reference_vcycle(levels, l + 1, xc, bc, nu_pre, nu_post, nu_coarse, adjoint, coarse_reduction,
                          coarse_direct, counts)
    x = x + prolong(lev, xc)
    for _ in range(nu_post):
        x = reference_sweep(K, b, x, blocks, P, n_t)
    return x


def solve_by_vcycles(levels, x0, b, tol=1e-10, max_cycles=50, adjoint=False, **kw):
    """Repeat V-cycles until sqrt(N / N0) <= tol; returns (x, history)."""
    lev = levels[0]
    K = operator(lev, adjoint)
    x = np.array(x0, dtype=complex)
    n0 = kkt.residual_norm(lev.system, b - K @ x)
    hist = [1.0]
    if n0 == 0.0:
        return x, hist
    for _ in range(max_cycles):
        x = reference_vcycle(levels, 0, x, b, adjoint=adjoint, **kw)
        ratio = np.sqrt(kkt.residual_norm(lev.system, b - K @ x) / n0)
        hist.append(ratio)
        if ratio <= tol:
            break
    return x, hist
