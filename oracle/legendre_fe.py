"""Legendre finite elements and the plane-wave relaxation experiment (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Implementation with Legendre Polynomials": on one element [-1, 1] of the
dimensionless coordinate y (space) and of the dimensionless time, the basis is
P_i(y) (i < N_x) times P_n(t) (n < N_t), with

* overlaps O_ij = int P_i P_j dy, U_nm = int P_n P_m dt (orthogonality),
* Q_nm = int P_n' P_m dt (n differentiated, the trial index),
* the kinetic matrix T_ij = <P_j | -(1/2) d^2/dy^2 | P_i> (trial i, test j, as
  the action of Sec. "Review of the Least Action Principle" pairs them; by
  parts this is (1/2)[int P_j' P_i' - P_j P_i' |_{-1}^{1}]),

and one element's least-action equations in the dimensionless form
Eq. (leastaction_dimensionless),

    sum_{i,n} C_in [ i O_ij Q_nm - 2 kappa T_ij U_nm - nu O_ij U_nm ] = 0   for all (j, m).

Element transfer (two children [-1, 0], [0, 1] of one parent): interpolation
I^(L/R)_ij = int P_i((y' -+ 1)/2) P_j(y') dy' and projection P^(L/R), the
transposes scaled so that (P^(L) + P^(R)) (I^(L) + I^(R)) = identity.
Continuity between elements, Eq. (eltcontinuity); initial and boundary
conditions, and the continuity-enforcing projection, Eq. (continuityprojection).

Sec. "Convergence": a trial function f = exp(i(k x + w t)) is expanded into
one element [-1, 1] or two elements [-1, 0], [0, 1], relaxed once (correction
form, Eq. (leastaction_correction), with Eqs. (ic_correction),
(bc1_correction), (bc2_correction) and the internal continuity), and the
residual norm and the magnitude of the action are compared before and after.

Readings (the paper is ambiguous or garbled here):

* T_ij: the closed form the paper prints, (j(j+1) - i(i+1))/(2m) for i > j with
  i - j even, is the entry that multiplies the trial coefficient C_in in the
  test row (j, m); the integral printed next to it has i and j exchanged.  We
  take the closed form's convention (m = 1 in the dimensionless form).
* The elements of the two-element calculation carry the same (kappa, nu), and
  the trial function is written in each element's own coordinate:
  x = (y - 1)/2 on the left element, x = (y + 1)/2 on the right one.
* Projection of f: the L2 projection (Galerkin: (O (x) U) C = overlaps) onto the
  elements, with continuity across the interface enforced by one multiplier
  per time function (the L2 form of Eq. (continuityprojection)).
* Constraints of a relaxation: the correction vanishes at the initial time and
  on the boundary of the relaxation volume (left and right ends), and is
  continuous inside it.  These rows are redundant at the corners (and at the
  interface's initial point); the correction is found in the null space of the
  constraint rows (an orthonormal basis from the SVD), which leaves it unique:
  N^T A N y = N^T r, delta = N y.
* Residual r_jm = -sum_in C_in A_(jm),(in) (the left side of the least-action
  equations, without the multiplier terms) and its norm N = r^H (O (x) U) r
  summed over elements, Eq. (residnorm); the action S = C^H A C = -C^H r.
  Ratios reported: sqrt(N_after / N_before) and |S_after| / |S_before|.
* Relaxation modes: "one" (one element, the whole [-1, 1]), "simultaneous"
  (both elements at once, interface continuity as a constraint), "intergrid"
  (Eqs. (residual_rough), (correction_fine): the residual projected from the
  two elements to their parent with P^(L/R), the parent's correction found
  with the Galerkin operator P A I under the parent's constraints and
  interpolated with I^(L/R), then each element relaxed separately with its
  interface held fixed).  P is applied to the residual as the paper writes it
  (the normalised transpose, P I = identity).
* The PDE behind Eq. (leastaction_dimensionless) is i d/dt phi = -kappa
  d^2/dy^2 phi + nu phi, so the plane wave exp(i(k y + w t)) solves it on the
  curve -w = kappa k^2 + nu (the paper prints this curve garbled).

Parity: pinned (tests/test_oracle_legendre_fe.py): the matrices against the
paper's closed forms and identities, the transfers by exact polynomial
reproduction and P I = identity, the relaxation by its constraints, its
stationarity on the admissible subspace and the equivalent direct form of
Eq. (leastaction_relaxedfunction), the experiment by its limits (a trial on
the dispersion curve has a vanishing residual; a basis too small to move).  The paper's figures are
absent: the maps themselves are parity unpinned.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def _P(n, y):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(y, c)


def _dP(n, y):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(y, npleg.legder(c))


def _d2P(n, y):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(y, npleg.legder(c, 2))


def _gauss(npts):
    return npleg.leggauss(npts)


def overlap(n):
    """O_ij = int_{-1}^{1} P_i P_j (also U for the time functions), by quadrature."""
    y, w = _gauss(n + 2)
    P = np.array([_P(i, y) for i in range(n)])
    return (P * w) @ P.T


def derivative(n):
    """Q_nm = int P_n' P_m (n differentiated), by quadrature."""
    y, w = _gauss(n + 2)
    P = np.array([_P(i, y) for i in range(n)])
    D = np.array([_dP(i, y) for i in range(n)])
    return (D * w) @ P.T


def kinetic(n):
    """T_ij = <P_j | -(1/2) d^2/dy^2 | P_i> on [-1, 1] (trial i, test j), by quadrature."""
    y, w = _gauss(n + 2)
    P = np.array([_P(i, y) for i in range(n)])
    D2 = np.array([_d2P(i, y) for i in range(n)])
    # entry [i, j] = int P_j (-1/2 P_i'')
    return -0.5 * (D2 * w) @ P.T


def transfer(n):
    """Interpolation and projection between a parent element and its children.

    Children: left [-1, 0] with y = (y' - 1)/2, right [0, 1] with y = (y' + 1)/2,
    y' the child's own coordinate.  The paper's I^(L/R)_ij = int P_i((y' -+ 1)/2)
    P_j(y') dy' is the overlap of parent function i with child function j; the
    parent function is a polynomial of degree i on the child, so its child
    coefficients are I_ij / O_jj.  Returned as operators on coefficient vectors:
    IL, IR [child j, parent i] = I^(L/R)_ij / O_jj, and the projections PL, PR
    [parent, child] = G^{-1} I^T O (the transposes in the overlap metric, G =
    IL^T O IL + IR^T O IR), so that PL IL + PR IR is the identity of the parent
    basis.
    """
    y, w = _gauss(2 * n + 2)
    O = overlap(n)
    out = {}
    for side, shift in (("L", -1.0), ("R", 1.0)):
        M = np.zeros((n, n))
        for j in range(n):          # child function
            for i in range(n):      # parent function
                M[j, i] = np.sum(w * _P(i, 0.5 * (y + shift)) * _P(j, y)) / O[j, j]
        out[side] = M
    G = out["L"].T @ O @ out["L"] + out["R"].T @ O @ out["R"]
    Gi = np.linalg.inv(G)
    proj = {s: Gi @ out[s].T @ O for s in ("L", "R")}
    return out["L"], out["R"], proj["L"], proj["R"]


def element_operator(nx, nt, kappa, nu):
    """A[(j, m), (i, n)] = i O_ij Q_nm - 2 kappa T_ij U_nm - nu O_ij U_nm (row: test
    (j, m); column: trial (i, n)); index (i, n) -> i * nt + n."""
    O, U, Q, T = overlap(nx), overlap(nt), derivative(nt), kinetic(nx)
    A = np.zeros((nx * nt, nx * nt), complex)
    for j in range(nx):
        for m in range(nt):
            for i in range(nx):
                for n in range(nt):
                    A[j * nt + m, i * nt + n] = 1j * O[i, j] * Q[n, m] - 2 * kappa * T[i, j] * U[n, m] \
                        - nu * O[i, j] * U[n, m]
    return A


def _block_diag(*Ms):
    n = sum(M.shape[0] for M in Ms)
    m = sum(M.shape[1] for M in Ms)
    out = np.zeros((n, m), dtype=np.result_type(*Ms))
    r = c = 0
    for M in Ms:
        out[r:r + M.shape[0], c:c + M.shape[1]] = M
        r += M.shape[0]
        c += M.shape[1]
    return out


def constraint_rows(nx, nt, ne, fix_left=True, fix_right=True, interface="continuous"):
    """Rows B (real) of the constraints on a correction over ne (1 or 2) elements
    [element][i][n]: zero at the initial time in every element (sum_n (-1)^n C_in
    = 0 for all i), zero at the left end (sum_i (-1)^i C_in = 0 for all n) and at
    the right end (sum_i C_in = 0), and for two elements either continuity at the
    interface (sum_i C^L_in = sum_i (-1)^i C^R_in) or, interface="fixed", zero there
    on both sides."""
    nel = nx * nt
    rows = []

    def row():
        return np.zeros(ne * nel)
    for e in range(ne):
        for i in range(nx):
            r = row()
            for n in range(nt):
                r[e * nel + i * nt + n] = (-1.0) ** n
            rows.append(r)
    for n in range(nt):
        if fix_left:
            r = row()
            for i in range(nx):
                r[i * nt + n] = (-1.0) ** i
            rows.append(r)
        if fix_right:
            r = row()
            for i in range(nx):
                r[(ne - 1) * nel + i * nt + n] = 1.0
            rows.append(r)
        if ne == 2:
            if interface == "continuous":
                r = row()
                for i in range(nx):
                    r[i * nt + n] = 1.0
                    r[nel + i * nt + n] = -(-1.0) ** i
                rows.append(r)
            else:
                for e, sgn in ((0, None), (1, -1.0)):
                    r = row()
                    for i in range(nx):
                        r[e * nel + i * nt + n] = 1.0 if sgn is None else sgn ** i
                    rows.append(r)
    return np.array(rows)


def null_space(B, tol=1e-10):
    """Orthonormal basis of {x : B x = 0} from the SVD (rank by singular values)."""
    u, s, vt = np.linalg.svd(B)
    rank = int(np.sum(s > tol * max(s.max(), 1.0)))
    return vt[rank:].T


def relax_operator(A, B):
    """M with delta = M r: the correction in the null space of B that makes the
    residual orthogonal to it, N^T (r - A N y) = 0."""
    N = null_space(B)
    if N.shape[1] == 0:
        return np.zeros_like(A)
    Ar = N.T @ A @ N
    return N @ np.linalg.solve(Ar, N.T)


def metric(nx, nt, ne):
    """Diagonal of O (x) U over the elements (the norm N = r^H diag r)."""
    d = np.kron(np.diag(overlap(nx)), np.diag(overlap(nt)))
    return np.tile(d, ne)


def mode_operators(nx, nt, kappa, nu, mode):
    """(A, M) of a relaxation mode over its elements: A the (block-diagonal)
    least-action operator, M the linear map from the residual to the correction."""
    A1 = element_operator(nx, nt, kappa, nu)
    if mode == "one":
        return A1, relax_operator(A1, constraint_rows(nx, nt, 1))
    A = _block_diag(A1, A1)
    if mode == "simultaneous":
        return A, relax_operator(A, constraint_rows(nx, nt, 2))
    if mode == "intergrid":
        IL, IR, PL, PR = transfer(nx)
        I_nt = np.eye(nt)
        # parent <- children projection and child <- parent interpolation, in the [i][n]
        # coefficient layout (space transfer, time identity); coarse problem of
        # Eq. (residual_rough): (P A I) delta_c = P r, corrected by Eq. (correction_fine)
        Pr = np.hstack([np.kron(PL, I_nt), np.kron(PR, I_nt)])
        Ip = np.vstack([np.kron(IL, I_nt), np.kron(IR, I_nt)])
        Mc = relax_operator(Pr @ A @ Ip, constraint_rows(nx, nt, 1))
        Mf = relax_operator(A, constraint_rows(nx, nt, 2, interface="fixed"))
        Mcoarse = Ip @ Mc @ Pr
        M = Mcoarse + Mf @ (np.eye(A.shape[0]) - A @ Mcoarse)
        return A, M
    raise ValueError(mode)


def _wave_overlaps(n, k, npts=64):
    """int_{-1}^{1} P_i(y) exp(i k y) dy, i < n."""
    y, w = _gauss(npts)
    e = np.exp(1j * k * y)
    return np.array([np.sum(w * _P(i, y) * e) for i in range(n)])


def trial_coefficients(nx, nt, ne, k, w):
    """L2 projection of f = exp(i(k x + w t)) onto the elements (continuous across
    the interface for two elements); layout [element][i][n]."""
    b = _wave_overlaps(nt, w)
    if ne == 1:
        a = _wave_overlaps(nx, k)
        f = np.kron(a, b)
    else:
        # x = (y -+ 1)/2 on the left / right element: exp(i k x) = exp(-+ i k/2) exp(i (k/2) y)
        a = _wave_overlaps(nx, 0.5 * k)
        f = np.concatenate([np.exp(-0.5j * k) * np.kron(a, b), np.exp(0.5j * k) * np.kron(a, b)])
    G = metric(nx, nt, ne)
    C = f / G
    if ne == 2:
        Bc = constraint_rows(nx, nt, 2, fix_left=False, fix_right=False)[2 * nx:]   # continuity rows
        # min (C' - C)^H G (C' - C) subject to Bc C' = 0
        Gi = 1.0 / G
        S = (Bc * Gi) @ Bc.T
        C = C - Gi * (Bc.T @ np.linalg.solve(S, Bc @ C))
    return C


def relax_ratios(nx, nt, kappa, nu, mode, k, w, ops=None):
    """(sqrt(N_after / N_before), |S_after| / |S_before|) for one trial function."""
    A, M = ops if ops is not None else mode_operators(nx, nt, kappa, nu, mode)
    ne = 1 if mode == "one" else 2
    C = trial_coefficients(nx, nt, ne, k, w)
    G = metric(nx, nt, ne)
    r = -A @ C
    d = M @ r
    C2 = C + d
    r2 = -A @ C2
    n0 = np.real(np.sum(G * np.abs(r) ** 2))
    n1 = np.real(np.sum(G * np.abs(r2) ** 2))
    s0 = np.vdot(C, A @ C)
    s1 = np.vdot(C2, A @ C2)
    return np.sqrt(n1 / n0), abs(s1) / abs(s0)


# the (kappa, nu) regimes of the paper's figures
REGIMES = [(0.0, 0.0), (0.1, 0.0), (1.0, 0.0), (10.0, 0.0), (0.0, 1.0), (0.0, -1.0), (1.0, 1.0), (1.0, -1.0)]
