"""The least-action system of one time step, assembled and solved directly.

Sec. "Review of the Least Action Principle":

* action S = sum C_in [i O_ij Q_nm - H_ij U_nm - V_ijnm] C*_jm;
* stationarity, Eq. (stationaryphase): for every (j, m)
      sum_{i,n} C_in [i O_ij Q_nm - H_ij U_nm - V_ijnm] = 0;
* initial condition by one Lagrange multiplier per spatial function:
  S' = S + sum_i lambda_i f_i*, f_i = sum_n C_in T_n(t0) - <chi_i|psi(t0)>,
  which adds lambda_j T_m(t0)* to row (j, m) and the row f_j = 0;
* action residual, Eq. (actionresidual), and its norm, Eq. (residnorm),
  N = r_in O_ij U_nm r*_jm.

Sec. "Iterative relaxation to the least action solution": N_x (N_t + 1)
unknowns per step, including the multipliers.

Ordering: unknown (j, n) -> j*N_t + n, multiplier j -> P*N_t + j; row (j, m)
-> j*N_t + m, constraint row j -> P*N_t + j.  With O = identity on the grid
and V(x, t) = V0(x) + z E(t):

    K = [[ I (x) iQ^T - H (x) U - Z (x) W,   I (x) s ],
         [ I (x) s^T,                        0       ]],     b = (0, psi0),

with H = T + diag(V0), Z = diag(z), W_nm = int T_n T_m E dt, s_n = T_n(t0).
The residual is the full system residual b - K x (the multiplier term is part
of it; at a solution of the constrained problem the paper's r_jm alone is not
zero).  N weights the stationarity rows with U and the constraint rows with 1.

Parity: pinned.  The assembly by brute force from the action and by closed
forms of the step (tests/test_oracle_kkt.py, tests/test_oracle_physics.py);
the pointwise checkers residual_at_points and block_system against the rows
and sub-matrices of the assembled system (tests/test_oracle_pointwise.py).
"""
from dataclasses import dataclass, field as dc_field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import timebasis as tb
from .grid import Grid, hamiltonian


@dataclass
class StepSystem:
    grid: Grid
    v0: np.ndarray
    n_t: int
    dt: float
    t0: float = 0.0
    field: object = None          # callable E(t) or None
    U: np.ndarray = dc_field(init=False)
    Q: np.ndarray = dc_field(init=False)
    s: np.ndarray = dc_field(init=False)
    e: np.ndarray = dc_field(init=False)
    W: np.ndarray = dc_field(init=False)
    K: sp.csr_matrix = dc_field(init=False)

    def __post_init__(self):
        self.v0 = np.asarray(self.v0, dtype=float).ravel()
        n_t, dt = self.n_t, self.dt
        self.U = tb.overlap_U(n_t, dt)
        self.Q = tb.derivative_Q(n_t, dt)
        self.s = tb.start_values(n_t)
        self.e = tb.end_values(n_t)
        if self.field is None:
            self.W = np.zeros((n_t, n_t))
        else:
            self.W = tb.field_matrix(n_t, self.t0, dt, self.field)
        self.K = assemble(self.grid, self.v0, self.U, self.Q, self.s, self.W)

    @property
    def npts(self):
        return self.grid.npts

    @property
    def size(self):
        return self.grid.npts * (self.n_t + 1)


def assemble(grid, v0, U, Q, s, W, z=None):
    """Sparse K of the step (see module docstring); z overrides the dipole coordinate."""
    P = grid.npts
    n_t = U.shape[0]
    I = sp.identity(P, format="csr")
    H = hamiltonian(grid, v0)
    Z = sp.diags(grid.z() if z is None else np.asarray(z, float).ravel())
    A = (sp.kron(I, 1j * Q.T) - sp.kron(H, U) - sp.kron(Z, W)).tocsr()
    B = sp.kron(I, s.reshape(-1, 1)).tocsr()          # multiplier columns
    C = sp.kron(I, s.reshape(1, -1)).tocsr()          # constraint rows
    K = sp.bmat([[A, B], [C, None]], format="csr")
    return K.astype(complex)


def split(x, npts, n_t):
    x = np.asarray(x)
    return x[: npts * n_t].reshape(npts, n_t), x[npts * n_t:]


def join(c, lam):
    return np.concatenate([np.asarray(c, dtype=complex).ravel(), np.asarray(lam, dtype=complex).ravel()])


def rhs(system, psi0, stat_rhs=None):
    """b = (stationarity right-hand side, psi0); the former is zero for a step."""
    P, n_t = system.npts, system.n_t
    top = np.zeros(P * n_t, complex) if stat_rhs is None else np.asarray(stat_rhs, complex).ravel()
    return np.concatenate([top, np.asarray(psi0, dtype=complex).ravel()])


def initial_guess(system, psi0):
    """c_j0 = psi0_j / s_0, c_jn = 0 for n >= 1, lambda = 0: meets the IC rows."""
    P, n_t = system.npts, system.n_t
    c = np.zeros((P, n_t), complex)
    c[:, 0] = np.asarray(psi0, complex).ravel() / system.s[0]
    return join(c, np.zeros(P, complex))


def residual(K, b, x):
    return b - K @ x


def residual_norm(system, r):
    """N = sum_j r_j^H U r_j over stationarity rows + sum_j |sigma_j|^2."""
    rho, sigma = split(r, system.npts, system.n_t)
    stat = np.einsum("jm,mn,jn->", rho.conj(), system.U, rho).real
    return float(stat + np.sum(np.abs(sigma) ** 2))


def solve_direct(K, b):
    """Direct solution: dense LAPACK for small systems, sparse LU otherwise."""
    n = K.shape[0]
    if n <= 6000:
        return np.linalg.solve(K.toarray(), b)
    return spla.splu(K.tocsc(), permc_spec="COLAMD").solve(b)


def end_state(system, x):
    """psi(t0 + dt)_j = sum_n T_n(t0 + dt) c_jn."""
    c, _ = split(x, system.npts, system.n_t)
    return c @ system.e


def step(grid, v0, psi0, n_t, dt, t0=0.0, field=None):
    sysm = StepSystem(grid, v0, n_t, dt, t0, field)
    x = solve_direct(sysm.K, rhs(sysm, psi0))
    return end_state(sysm, x), x, sysm


def propagate(grid, v0, psi0, n_t, dt, n_steps, field=None, t_start=0.0):
    """Repeated direct steps; returns the list [psi_0, ..., psi_K]."""
    psis = [np.asarray(psi0, complex).ravel()]
    for k in range(n_steps):
        psi, _, _ = step(grid, v0, psis[-1], n_t, dt, t_start + k * dt, field)
        psis.append(psi)
    return psis


def residual_at_points(grid, v0, n_t, dt, t0, field, c, lam, psi0, points, stat_rhs=None, adjoint=False):
    """Residual rows of the points ``points`` only, from the definition.

    For every requested point j: rho_jm = rhs_jm - [ i (Q^T c_j)_m - (U ((T + V0) c)_j)_m
    - z_j (W c_j)_m + s_m lambda_j ] and sigma_j = psi0_j - sum_n s_n c_jn, with the
    neighbours of j gathered explicitly; usable on grids too large to assemble.
    For adjoint=True the time block is (iQ^T)^H = -iQ and the right-hand side is
    g_j on every row (pass g as stat_rhs, one value per point) with psi0 = 0.
    c: (P, n_t), lam: (P,), psi0: (P,), points: iterable of point indices.
    Returns rho (len(points), n_t) and sigma (len(points),).
    """
    U = tb.overlap_U(n_t, dt)
    Q = tb.derivative_Q(n_t, dt)
    s = tb.start_values(n_t)
    W = np.zeros((n_t, n_t)) if field is None else tb.field_matrix(n_t, t0, dt, field)
    shape = grid.n
    z_axis = grid.field_axis % grid.dim
    kin = 0.5 / grid.mass / grid.h ** 2
    pts = np.asarray(points, dtype=np.int64)
    rho = np.zeros((len(pts), n_t), complex)
    sig = np.zeros(len(pts), complex)
    tmat = (-1j * Q) if adjoint else (1j * Q.T)
    for k, j in enumerate(pts):
        idx = np.unravel_index(int(j), shape)
        lap = -2.0 * grid.dim * c[j]
        for a in range(grid.dim):
            for d in (-1, 1):
                nb = list(idx)
                nb[a] += d
                if grid.periodic:
                    nb[a] %= shape[a]
                elif not 0 <= nb[a] < shape[a]:
                    continue
                lap = lap + c[np.ravel_multi_index(tuple(nb), shape)]
        Hc = -kin * lap + v0[j] * c[j]
        z = (idx[z_axis] - 0.5 * (shape[z_axis] - 1)) * grid.h
        row = tmat @ c[j] - U @ Hc - z * (W @ c[j]) + s * lam[j]
        rhs = np.zeros(n_t, complex) if stat_rhs is None else stat_rhs[j]
        rho[k] = rhs - row
        sig[k] = psi0[j] - s @ c[j]
    return rho, sig


def block_system(grid, v0, n_t, dt, t0, field, points):
    """Dense K restricted to the rows and columns of one box of points.

    The box's own kinetic stencil with everything outside held at zero, its
    V0 and z, and the time operators of the step: exactly the block of K on
    those rows and columns (Dirichlet grids).
    """
    pts = np.asarray(points)
    coords = np.array(np.unravel_index(pts, grid.n)).T
    lo = coords.min(axis=0)
    bshape = tuple(int(x) for x in coords.max(axis=0) - lo + 1)
    order = np.ravel_multi_index(tuple((coords - lo).T), bshape)
    if not np.array_equal(np.sort(order), np.arange(len(pts))):
        raise ValueError("points must form a box")
    sub = Grid(bshape, grid.h, False, grid.mass, grid.field_axis)
    z_axis = grid.field_axis % grid.dim
    zfull = (coords[:, z_axis] - 0.5 * (grid.n[z_axis] - 1)) * grid.h
    inv = np.empty(len(pts), int)
    inv[order] = np.arange(len(pts))
    v_sub = np.asarray(v0)[pts][inv]
    z_sub = zfull[inv]
    U = tb.overlap_U(n_t, dt)
    Q = tb.derivative_Q(n_t, dt)
    s = tb.start_values(n_t)
    W = np.zeros((n_t, n_t)) if field is None else tb.field_matrix(n_t, t0, dt, field)
    K = assemble(sub, v_sub, U, Q, s, W, z=z_sub).toarray()
    # rows/cols of ``sub`` are in box C order; entry k of ``points`` is box point order[k]
    rows = np.concatenate([(order[:, None] * n_t + np.arange(n_t)[None, :]).ravel(),
                           len(pts) * n_t + order])
    return K[np.ix_(rows, rows)]
