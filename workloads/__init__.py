"""Seeded synthetic inputs for the least-action propagator workloads.

This module only produces input arrays (grids, potentials, initial states,
pulse coefficients, reference states); it holds none of the propagator's
arithmetic and imports neither the oracle nor the HIP library, so both sides
can take their inputs from here.

Workloads (the paper reports no problem sizes; these are the synthetic
stand-ins, all in atomic units with m = 1):

  1d_harmonic      1D 256 points on [-20, 20] (h = 40/256), V = x^2/2, N_t = 8,
                   dt = 0.05, blocks of 8, Gaussian x0 = -5, k0 = 1, sigma = 1.
  2d_softcoulomb   2D 512 x 512, h = 0.2, V = -1/sqrt(r^2 + 1), N_t = 8,
                   dt = 0.05, 8 x 8 blocks, 2..5 levels, 20 steps,
                   random-phase Gaussian (sigma = 2, phase per point, seed 0).
  3d_laser         3D 128^3, h = 0.3, soft-Coulomb, E(t) = E0 sin^2(pi t/T)
                   cos(w t) with E0 = 0.05, w = 0.057, T = 20 dt, N_t = 6,
                   4^3 blocks, 5 levels, Gaussian sigma = 1.
  2d_adjoint       2D 256 x 256, h = 0.2, soft-Coulomb, E(t) = sum_q a_q
                   sin(q pi t/T), 16 a_q ~ N(0, 0.02^2) seed 0, T = 40 dt,
                   N_t = 8, 8 x 8 blocks, 4 levels, 40 steps; initial state and
                   reference state = the grid ground state.
  3d_large         3D 256^3, h = 0.25, E0 = 0.1 sin^2 laser plus 32 Fourier
                   amplitudes ~ N(0, 0.02^2) seed 0, N_t = 8, 4^3 blocks,
                   6 levels, 20 steps, Gaussian sigma = 1.

``scaled(name, n)`` gives the same workload (same h, dt, N_t, blocks,
potential and state recipe) on n points per axis, for sizes a CPU direct
solve can finish.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

WORKLOADS = {
    "1d_harmonic": dict(dim=1, n=256, h=40.0 / 256, n_t=8, dt=0.05, block=8, levels=1,
                        steps=1, potential="harmonic", state="gauss_moving", pulse=None),
    "2d_softcoulomb": dict(dim=2, n=512, h=0.2, n_t=8, dt=0.05, block=8, levels=5,
                           steps=20, potential="softcoulomb", state="random_phase", pulse=None),
    "3d_laser": dict(dim=3, n=128, h=0.3, n_t=6, dt=0.05, block=4, levels=5, steps=20,
                     potential="softcoulomb", state="gauss",
                     pulse=dict(kind="sin2", e0=0.05, omega=0.057, n_coef=0)),
    "2d_adjoint": dict(dim=2, n=256, h=0.2, n_t=8, dt=0.05, block=8, levels=4, steps=40,
                       potential="softcoulomb", state="ground",
                       pulse=dict(kind="fourier", e0=0.0, omega=0.0, n_coef=16, sigma=0.02, seed=0)),
    "3d_large": dict(dim=3, n=256, h=0.25, n_t=8, dt=0.05, block=4, levels=6, steps=20,
                     potential="softcoulomb", state="gauss",
                     pulse=dict(kind="sin2+fourier", e0=0.1, omega=0.057, n_coef=32, sigma=0.02, seed=0)),
}


def config(name, n=None, levels=None, steps=None):
    cfg = dict(WORKLOADS[name])
    cfg["name"] = name
    if n is not None:
        cfg["n"] = int(n)
    if levels is not None:
        cfg["levels"] = int(levels)
    if steps is not None:
        cfg["steps"] = int(steps)
    cfg["shape"] = (cfg["n"],) * cfg["dim"]
    cfg["t_total"] = cfg["steps"] * cfg["dt"]
    # the coarsest-level solve of a V-cycle: colour sweeps until its residual norm
    # has fallen by 1e3, at most four of them
    cfg["nu_coarse"] = 4
    cfg["coarse_reduction"] = 1e-3
    return cfg


def coords(shape, h):
    axes = [(np.arange(n) - 0.5 * (n - 1)) * h for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def potential(cfg):
    X = coords(cfg["shape"], cfg["h"])
    r2 = sum(x * x for x in X)
    if cfg["potential"] == "harmonic":
        return (0.5 * r2).ravel()
    if cfg["potential"] == "softcoulomb":
        return (-1.0 / np.sqrt(r2 + 1.0)).ravel()
    raise ValueError(cfg["potential"])


def _normalise(psi, h, dim):
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * h ** dim)


def ground_state(shape, h, v0):
    """Lowest eigenvector of -(1/2) Lap_h + V0 (5/7-point, zero outside)."""
    d = len(shape)
    L = None
    for a in range(d):
        n = shape[a]
        D = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]) / h ** 2
        mats = [sp.identity(shape[b]) for b in range(d)]
        mats[a] = D
        term = mats[0]
        for m in mats[1:]:
            term = sp.kron(term, m)
        L = term if L is None else L + term
    H = (-0.5 * L + sp.diags(v0)).tocsc()
    w, V = spla.eigsh(H, k=1, sigma=float(v0.min()) - 1.0, which="LM")
    g = V[:, 0]
    g = g * np.sign(g[np.argmax(np.abs(g))])
    return _normalise(g.astype(complex), h, d)


def initial_state(cfg, v0=None, seed=0):
    X = coords(cfg["shape"], cfg["h"])
    r2 = sum(x * x for x in X)
    d = cfg["dim"]
    st = cfg["state"]
    if st == "gauss_moving":
        x = X[0]
        psi = np.exp(-(x + 5.0) ** 2 / 2.0 + 1j * x)
    elif st == "random_phase":
        rng = np.random.default_rng(seed)
        psi = np.exp(-r2 / (2 * 2.0 ** 2)) * np.exp(1j * rng.uniform(0, 2 * np.pi, r2.shape))
    elif st == "gauss":
        psi = np.exp(-r2 / 2.0).astype(complex)
    elif st == "ground":
        if v0 is None:
            v0 = potential(cfg)
        return ground_state(cfg["shape"], cfg["h"], v0)
    else:
        raise ValueError(st)
    return _normalise(psi.ravel(), cfg["h"], d)


def pulse_coefficients(cfg):
    p = cfg["pulse"]
    if not p or p.get("n_coef", 0) == 0:
        return np.zeros(0)
    rng = np.random.default_rng(p.get("seed", 0))
    return rng.normal(0.0, p.get("sigma", 0.02), p["n_coef"])


def random_complex(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * (rng.normal(size=n) + 1j * rng.normal(size=n))


def random_real(n, seed, scale=1.0):
    return scale * np.random.default_rng(seed).normal(size=n)


def random_state_device(npts, n_t, seed, device, scale=1.0):
    """Seeded random (c, lambda) generated on the device (torch Philox stream).

    For full-size workloads where a host copy would be large; tests read back
    only the entries they sample.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    c = torch.randn(npts * n_t, dtype=torch.complex128, device=device, generator=gen) * scale
    lam = torch.randn(npts, dtype=torch.complex128, device=device, generator=gen) * scale
    return c, lam
