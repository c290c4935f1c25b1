"""Legendre finite-element oracle pinned against the paper's closed forms and identities.

Sec. "Implementation with Legendre Polynomials": orthogonality, the pattern of
Q, the closed form of the kinetic matrix (with the reading of its indices),
element transfers that reproduce polynomials and invert each other; the
relaxation of the plane-wave experiment (Sec. "Convergence") by its
constraints, its stationarity, the equivalent direct form and its limits.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import legendre_fe as L


@pytest.mark.parametrize("n", [1, 3, 8])
def test_overlap_is_orthogonality(n):
    np.testing.assert_allclose(L.overlap(n), np.diag([2.0 / (2 * i + 1) for i in range(n)]), atol=1e-14)


def test_derivative_pattern():
    n = 8
    Q = L.derivative(n)
    ref = np.array([[2.0 if (a > b and (a - b) % 2) else 0.0 for b in range(n)] for a in range(n)])
    np.testing.assert_allclose(Q, ref, atol=1e-13)


def test_kinetic_closed_form():
    """The paper's closed form: (j(j+1) - i(i+1))/2 for i > j with i - j even (m = 1),
    zero otherwise, as the entry of trial i in test row j."""
    n = 9
    T = L.kinetic(n)
    ref = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i > j and (i - j) % 2 == 0:
                ref[i, j] = (j * (j + 1) - i * (i + 1)) / 2.0
    np.testing.assert_allclose(T, ref, atol=1e-12)


def test_kinetic_acts_as_the_second_derivative_on_polynomials():
    """sum_i c_i T_ij = int P_j (-(1/2) phi'') for phi = sum_i c_i P_i, with phi''
    and the integral taken by numpy's Legendre-series calculus (an independent route)."""
    n = 7
    rng = np.random.default_rng(0)
    c = rng.normal(size=n)
    d2 = npleg.legder(c, 2)
    ref = np.empty(n)
    for j in range(n):
        e = np.zeros(j + 1)
        e[j] = 1.0
        prod = npleg.legmul(-0.5 * d2, e)
        integ = npleg.legint(prod)
        ref[j] = npleg.legval(1.0, integ) - npleg.legval(-1.0, integ)
    np.testing.assert_allclose(c @ L.kinetic(n), ref, atol=1e-12)


@pytest.mark.parametrize("n", [2, 4, 7])
def test_transfer_reproduces_parent_polynomials_and_inverts(n):
    IL, IR, PL, PR = L.transfer(n)
    rng = np.random.default_rng(n)
    c = rng.normal(size=n)
    y = np.linspace(-1, 1, 11)
    # the parent polynomial on each child, in the child's coordinate
    np.testing.assert_allclose(npleg.legval(y, IL @ c), npleg.legval(0.5 * (y - 1), c), atol=1e-12)
    np.testing.assert_allclose(npleg.legval(y, IR @ c), npleg.legval(0.5 * (y + 1), c), atol=1e-12)
    np.testing.assert_allclose(PL @ IL + PR @ IR, np.eye(n), atol=1e-12)
    # the projection of two children that hold one parent polynomial returns it
    np.testing.assert_allclose(PL @ (IL @ c) + PR @ (IR @ c), c, atol=1e-12)


@pytest.mark.parametrize("mode", ["one", "simultaneous", "intergrid"])
@pytest.mark.parametrize("nx,nt", [(3, 3), (4, 5), (6, 6)])
def test_relaxation_correction_meets_its_constraints(mode, nx, nt):
    A, M = L.mode_operators(nx, nt, 1.0, -1.0, mode)
    ne = 1 if mode == "one" else 2
    C = L.trial_coefficients(nx, nt, ne, 1.7, 0.9)
    r = -A @ C
    d = M @ r
    B = L.constraint_rows(nx, nt, ne)
    # the correction vanishes at the initial time and the ends, and is continuous inside
    assert np.abs(B @ d).max() <= 1e-12 * np.abs(d).max()
    if mode != "intergrid":
        # the new residual is orthogonal to every admissible correction
        N = L.null_space(B)
        assert np.abs(N.T @ (r - A @ d)).max() <= 1e-10 * np.abs(r).max()


def test_trial_projection_is_continuous_and_exact_for_polynomials():
    nx, nt = 5, 4
    C = L.trial_coefficients(nx, nt, 2, 2.3, -0.7).reshape(2, nx, nt)
    # continuity: value at the right end of the left element = value at the left end of the right one
    left_end = C[0].sum(axis=0)
    right_start = (C[1] * ((-1.0) ** np.arange(nx))[:, None]).sum(axis=0)
    np.testing.assert_allclose(left_end, right_start, atol=1e-13)
    # one element, k = w = 0: the constant 1 is exactly C_00 = 1
    C1 = L.trial_coefficients(nx, nt, 1, 0.0, 0.0)
    ref = np.zeros(nx * nt)
    ref[0] = 1.0
    np.testing.assert_allclose(C1, ref, atol=1e-14)


def test_direct_form_gives_the_same_relaxed_function():
    """Eq. (leastaction_relaxedfunction): solving for the relaxed coefficients C'
    with the trial's initial and boundary values (B C' = B C) and the equations on
    the admissible subspace gives C + delta of the correction form."""
    nx, nt = 5, 5
    A, M = L.mode_operators(nx, nt, 0.1, 1.0, "one")
    C = L.trial_coefficients(nx, nt, 1, -2.2, 1.1)
    B = L.constraint_rows(nx, nt, 1)
    N = L.null_space(B)
    # C' = C_p + N y with B C_p = B C (C_p = C itself) and N^T A C' = 0
    y = np.linalg.solve(N.T @ A @ N, -N.T @ A @ C)
    C_direct = C + N @ y
    np.testing.assert_allclose(C_direct, C + M @ (-A @ C), atol=1e-12 * np.abs(C).max())


def test_small_basis_cannot_move():
    """N_x = N_t = 2 on one element: the initial and boundary rows leave no
    admissible correction, so relaxation changes nothing (ratio exactly 1)."""
    A, M = L.mode_operators(2, 2, 1.0, 0.0, "one")
    assert np.abs(M).max() == 0.0
    rn, ra = L.relax_ratios(2, 2, 1.0, 0.0, "one", 1.1, -0.4)
    assert rn == 1.0 and ra == 1.0


@pytest.mark.parametrize("kappa,nu", [(1.0, 0.5), (0.1, -1.0), (1.0, 0.0)])
def test_plane_wave_on_the_dispersion_curve_has_a_vanishing_residual(kappa, nu):
    """exp(i(k y + w t)) solves i d/dt phi = -kappa phi'' + nu phi when -w = kappa k^2 + nu:
    its projection's residual falls with the basis size (spectral accuracy), while a
    trial off the curve keeps an O(1) residual.  A wrong sign or index in Q, T or
    the operator fails this."""
    k = 1.3
    w_on = -(kappa * k * k + nu)
    norms = []
    for n in (4, 12):
        A = L.element_operator(n, n, kappa, nu)
        G = L.metric(n, n, 1)
        for w in (w_on, w_on + 1.0, -w_on):
            r = -A @ L.trial_coefficients(n, n, 1, k, w)
            norms.append(np.sqrt(np.sum(G * np.abs(r) ** 2)))
    on4, off4, flip4, on12, off12, flip12 = norms
    assert on12 < 1e-6 * min(off12, flip12)
    assert on12 < 1e-5 * on4


@pytest.mark.parametrize("ne", [1, 2])
def test_trial_projection_reproduces_the_plane_wave(ne):
    """The projected trial evaluated at points of each element, in global
    coordinates (x = y on one element; x = (y -+ 1)/2 on the left / right one),
    equals exp(i(k x + w t)) to spectral accuracy."""
    n, k, w = 12, 2.3, -1.7
    C = L.trial_coefficients(n, n, ne, k, w).reshape(ne, n, n)
    y = np.linspace(-0.95, 0.95, 7)
    t = np.linspace(-0.9, 0.9, 5)
    Py = np.array([npleg.legval(y, np.eye(n)[i]) for i in range(n)])
    Pt = np.array([npleg.legval(t, np.eye(n)[m]) for m in range(n)])
    for e in range(ne):
        phi = Py.T @ C[e] @ Pt                       # [y, t]
        x = y if ne == 1 else 0.5 * (y + (2 * e - 1))
        ref = np.exp(1j * (k * x[:, None] + w * t[None, :]))
        assert np.abs(phi - ref).max() < 1e-7
