"""Benchmark of the least-action relaxation path on one MI355X.

Headline workload (the largest single-GPU configuration): 3d_large, a 3D
256^3 grid, h = 0.25, soft-Coulomb V0 = -1/sqrt(r^2 + 1) plus a dipole field
E(t) = 0.1 sin^2(pi t/T) cos(0.057 t) + 32 Fourier sine amplitudes
(N(0, 0.02^2), seed 0), N_t = 8 Legendre time functions, dt = 0.05, 4^3
subvolumes, 6-level V(1,1) cycles, Gaussian initial state, steps solved to
sqrt(N/N0) <= 1e-10.  A "step" is one propagation time step: every kernel of
the path (residual, colour sweeps on all levels, projection, interpolation,
coarse sweeps, step I/O) until the tolerance, inputs resident in HBM.

value: finest-level Munknowns*sweeps/s = P * N_t * (finest full sweeps done
in the timed steps) / (wall time of the timed steps) / 1e6, on the mixed path
(FP32 subvolume solves, FP64 state, residual, transfers and coarsest level),
which is what the workload names.  The FP64 path is reported next to it, with
the time to reach the 1e-10 residual per step for both, the adjoint step, and
the 2D soft-Coulomb 512^2 workload as an extra block.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Munknowns·sweeps/s + time-to-action-residual 1e-10 (FP64 vs mixed) per step"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_1111_4363_amd", "csrc", "lam_kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "sweep_counters.json")
HEADLINE = "3d_large"


def sweep_launch_bytes(shape, block, n_t, colour, precision):
    """Algorithmic HBM bytes of one finest-level colour launch (forward step).

    Per block of b points: its eigenvectors, b^2 reals (8 B FP64, 4 B mixed),
    its b eigenvalues (FP64), its id (4 B, only when the colour's blocks come
    from a table: an odd block count along the last axis) and its inner-pass
    count (1 B written).  Per own point: read c (N_t complex FP64), lambda,
    the constraint right-hand side (complex) and V0 (real); write c and
    lambda.  Per distinct halo point of the launch: read c (N_t complex).
    The time factor records (one per slab of blocks along the field axis, or
    one for the whole launch; a few hundred KB at most) are read once per
    launch and not counted.
    """
    import numpy as np
    nblk = [s // b for s, b in zip(shape, block)]
    b = int(np.prod(block))
    rb = 8 if precision == "fp64" else 4
    coords = np.indices(nblk).reshape(len(nblk), -1).T
    ncol = int(np.sum(coords.sum(axis=1) % 2 == colour))
    per_block = b * b * rb + b * 8 + (4 if nblk[-1] % 2 else 0) + 1
    per_point = (n_t * 16 + 16 + 16 + 8) + (n_t * 16 + 16)
    # distinct halo points: points outside a colour block, face-adjacent to one
    owner_colour = np.zeros(shape, dtype=np.int8)
    idx = np.indices(shape, dtype=np.int16)
    for a in range(len(shape)):
        owner_colour += (idx[a] // block[a]).astype(np.int8)
    del idx
    owner_colour %= 2
    inside = owner_colour == colour
    del owner_colour
    halo = np.zeros(shape, bool)
    for a in range(len(shape)):
        for d in (-1, 1):
            sh = np.roll(inside, d, axis=a)
            # no wrap on a Dirichlet grid
            sl = [slice(None)] * len(shape)
            sl[a] = 0 if d == 1 else -1
            sh[tuple(sl)] = False
            halo |= sh & ~inside
    nhalo = int(halo.sum())
    return ncol * (per_block + b * per_point) + nhalo * n_t * 16, ncol


def counters_for_current_kernel(key):
    """Traffic per launch from committed rocprofv3 counters (entry `key`, e.g.
    "3d_large/mixed"), if they were taken on this kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    try:
        with open(COUNTERS) as f:
            rec = json.load(f)
        with open(KERNEL_SOURCE, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
        if rec.get("kernel_source_sha256") != digest:
            return None
        ent = rec.get("entries", {}).get(key)
        return ent.get("traffic_bytes_per_launch") if ent else None
    except Exception:
        return None


def threads_in_use():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def field_of(cfg):
    """The workload's field E(t) as a host function for the oracle (None without)."""
    import workloads as W
    from oracle import timebasis as tb
    p = cfg["pulse"]
    if not p:
        return None
    parts = []
    if p["kind"] in ("sin2", "sin2+fourier"):
        parts.append(tb.pulse_sin2_cos(p["e0"], p["omega"], cfg["t_total"]))
    if p["kind"] in ("fourier", "sin2+fourier"):
        parts.append(tb.pulse_fourier_sine(list(W.pulse_coefficients(cfg)), cfg["t_total"]))
    return parts[0] if len(parts) == 1 else (lambda t: parts[0](t) + parts[1](t))


def cpu_baseline(name, budget_s=15.0):
    """The oracle, untuned, on a window of the workload: plain-loop colour sweeps
    (dense local solves of its subvolumes) on a 16^3 (3D) or 64^2 (2D) window,
    and its direct step solve on an 8^3 (3D) or 32^2 (2D) window, median of 3."""
    import numpy as np
    import workloads as W
    from oracle import grid as G
    from oracle import kkt, relax
    threads = threads_in_use()
    full = W.config(name)
    field = field_of(full)
    t0 = 0.35 * full["t_total"]
    win = 16 if full["dim"] == 3 else 64
    cfg = W.config(name, n=win)
    v0 = W.potential(cfg)
    psi0 = W.initial_state(cfg, v0)
    g = G.Grid(cfg["shape"], cfg["h"])
    sysm = kkt.StepSystem(g, v0, cfg["n_t"], cfg["dt"], t0, field)
    b = kkt.rhs(sysm, psi0)
    x = kkt.initial_guess(sysm, psi0)
    bl = G.blocks(g, (cfg["block"],) * cfg["dim"])
    sweeps = 0
    t_a = time.perf_counter()
    while True:
        x = relax.reference_sweep(sysm.K, b, x, bl, g.npts, cfg["n_t"])
        sweeps += 1
        if time.perf_counter() - t_a > budget_s or sweeps >= 60:
            break
    dt = time.perf_counter() - t_a
    value = g.npts * cfg["n_t"] * sweeps / dt / 1e6
    # direct solve of one step (assembly + factorisation + solve) on a smaller window
    dwin = 8 if full["dim"] == 3 else 32
    dcfg = W.config(name, n=dwin)
    dv0 = W.potential(dcfg)
    dpsi = W.initial_state(dcfg, dv0)
    dg = G.Grid(dcfg["shape"], dcfg["h"])
    times = []
    for _ in range(3):
        t_b = time.perf_counter()
        kkt.step(dg, dv0, dpsi, dcfg["n_t"], dcfg["dt"], t0, field)
        times.append(time.perf_counter() - t_b)
    t_direct = float(np.median(times))
    unknowns = dg.npts * (dcfg["n_t"] + 1)
    shape = "x".join(str(k) for k in cfg["shape"])
    dshape = "x".join(str(k) for k in dcfg["shape"])
    return {"value": value, "unit": "Munknowns·sweeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{sweeps} full colour sweeps (plain-loop dense local solves of the "
                      f"{cfg['block']}^{cfg['dim']} subvolumes, field on) of the same workload on a {shape} "
                      f"window, {dt:.1f} s",
            "direct_step": {"window": dshape, "unknowns": unknowns, "s_per_step_median_of_3": t_direct,
                            "munknowns_per_s": unknowns / t_direct / 1e6,
                            "method": "assembly + dense LAPACK (<= 6000 unknowns) or SuperLU solve of the "
                                      "step system, the oracle's kkt.step"}}


def oracle_direct_2d(sizes=(64, 128), repeats=3):
    """The oracle's direct solve of one step of the 2D soft-Coulomb workload
    (same h, dt, N_t, potential, state) at reduced sizes: SuperLU factorisation
    (COLAMD) and solve timed separately, median of `repeats`."""
    import numpy as np
    import scipy.sparse.linalg as spla
    import workloads as W
    from oracle import grid as G
    from oracle import kkt
    out = {"workload": "2d_softcoulomb", "threads": threads_in_use(), "cores": os.cpu_count(),
           "method": "scipy.sparse.linalg.splu (SuperLU, COLAMD) of the assembled step system", "sizes": {}}
    for n in sizes:
        cfg = W.config("2d_softcoulomb", n=n)
        v0 = W.potential(cfg)
        psi0 = W.initial_state(cfg, v0)
        g = G.Grid(cfg["shape"], cfg["h"])
        sysm = kkt.StepSystem(g, v0, cfg["n_t"], cfg["dt"])
        b = kkt.rhs(sysm, psi0)
        Kc = sysm.K.tocsc()
        tf, ts = [], []
        for _ in range(repeats):
            t_a = time.perf_counter()
            lu = spla.splu(Kc, permc_spec="COLAMD")
            tf.append(time.perf_counter() - t_a)
            t_a = time.perf_counter()
            x = lu.solve(b)
            ts.append(time.perf_counter() - t_a)
        res = float(np.abs(sysm.K @ x - b).max())
        out["sizes"][f"{n}x{n}"] = {"unknowns": sysm.size, "factor_s": float(np.median(tf)),
                                    "solve_s": float(np.median(ts)), "max_residual": res}
        print(f"[oracle-direct] {n}^2: factor {np.median(tf):.2f} s, solve {np.median(ts):.3f} s",
              file=sys.stderr, flush=True)
    return out


# Relaxation variants over groups of 2^d elements (Sec. "Convergence"): each
# element relaxed separately (blocks of edge e), the group relaxed
# simultaneously (blocks of edge 2e), or separately after a correction found
# on the coarse grid whose element is the group (one more level: the residual
# projected, the coarse element relaxed, the correction interpolated, then the
# fine elements relaxed separately; the paper's intergrid-transfer variant).
VARIANT_PROBLEMS = {
    "2d": dict(workload="2d_softcoulomb", n=256, edge=4),
    "3d": dict(workload="3d_laser", n=128, edge=2),
}


def relaxation_variants(torch, lam, precision="fp64", iters=6, problems=("2d", "3d")):
    """Residual reduction per iteration and GPU time per iteration of the three
    variants, from the same initial guess of one step (the workloads' potential,
    h, dt and N_t, without field)."""
    import numpy as np
    import workloads as W
    out = {}
    dev = torch.device("cuda:0")
    for key in problems:
        spec = VARIANT_PROBLEMS[key]
        cfg = W.config(spec["workload"], n=spec["n"])
        v0 = W.potential(cfg)
        psi0 = W.initial_state(cfg, v0)
        d, e = cfg["dim"], spec["edge"]
        v0_t = torch.as_tensor(v0, device=dev)
        psi_t = torch.as_tensor(psi0, device=dev)
        P, nt = int(np.prod(cfg["shape"])), cfg["n_t"]
        c0 = torch.zeros(P * nt, dtype=torch.complex128, device=dev)
        c0.view(P, nt)[:, 0] = psi_t
        l0 = torch.zeros(P, dtype=torch.complex128, device=dev)
        res = {}
        for name, block, levels, (pre, post, coarse) in (
                ("separate", e, 1, (0, 0, 1)),
                ("simultaneous", 2 * e, 1, (0, 0, 1)),
                ("intergrid", e, 2, (0, 1, 1))):
            prop = lam.Propagator(cfg["shape"], cfg["h"], v0_t, nt, cfg["dt"], (block,) * d, levels=levels,
                                  nu_pre=pre, nu_post=post, nu_coarse=coarse, precision=precision)
            _, _, n0 = prop.residual_action(0.0, psi_t, c0, l0, want_fields=False)
            prop.set_state(0.0, psi_t, c0, l0)
            prop.vcycle(norm=False)                       # warm-up
            prop.set_state(0.0, psi_t, c0, l0)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(prop.stream)
            for _ in range(iters):
                prop.vcycle(norm=False)
            ev[1].record(prop.stream)
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / iters
            c, l_ = prop.get_state()
            _, _, nk = prop.residual_action(0.0, psi_t, c, l_, want_fields=False)
            rate = (nk / n0) ** (0.5 / iters)
            res[name] = {"block": "x".join([str(block)] * d), "levels": levels, "ms_per_iteration": ms,
                         "residual_ratio_per_iteration": rate,
                         "decades_per_ms": -np.log10(rate) / ms if rate > 0 else None}
            prop.close()
        sep = res["separate"]["ms_per_iteration"]
        for r in res.values():
            r["cost_vs_separate"] = r["ms_per_iteration"] / sep
        out[key] = {"problem": f"{spec['workload']} at {'x'.join(str(k) for k in cfg['shape'])}, h={cfg['h']}, "
                               f"N_t={nt}, dt={cfg['dt']}, no field, {precision}", "variants": res}
    return out


# (kappa, nu) regimes of the paper's convergence maps (Sec. "Convergence")
PW_REGIMES = [(0.0, 0.0), (0.1, 0.0), (1.0, 0.0), (10.0, 0.0), (0.0, 1.0), (0.0, -1.0), (1.0, 1.0), (1.0, -1.0)]


def plane_wave_maps(torch, lam, npts=128, kmax=8.0, bases=((3, 3), (4, 4), (6, 6))):
    """The plane-wave convergence maps on an npts x npts grid of (k, w) in
    [-kmax, kmax]^2 (cell centres), for every regime, basis size and mode: the
    fraction of trial waves whose residual norm falls (ratio < 1) and falls ten
    times (< 0.1), the median log10 of the ratio, and the GPU time of the map."""
    import numpy as np
    grid = [-kmax + 2 * kmax * (j + 0.5) / npts for j in range(npts)]
    out = []
    for mode in ("one", "simultaneous", "intergrid"):
        for nx, nt in bases:
            for kappa, nu in PW_REGIMES:
                torch.cuda.synchronize()
                t_a = time.perf_counter()
                rr, ar = lam.plane_wave_map(nx, nt, mode, kappa, nu, grid, grid)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t_a) * 1e3
                r = rr.cpu().numpy().ravel()
                a = ar.cpu().numpy().ravel()
                ok = np.isfinite(r)
                lr = np.log10(r[ok])
                out.append({"mode": mode, "n_x": nx, "n_t": nt, "kappa": kappa, "nu": nu,
                            "frac_resid_below_1": float(np.mean(r[ok] < 1.0)),
                            "frac_resid_below_0.1": float(np.mean(r[ok] < 0.1)),
                            "median_log10_resid_ratio": float(np.median(lr)),
                            "median_log10_action_ratio": float(np.median(np.log10(a[np.isfinite(a)]))),
                            "ms_per_map": ms, "points": npts * npts})
    return out


def adaptive_tree(torch, lam, steps=4, fractions=(1e-10, 1e-8, 1e-6, 1e-4)):
    """The adaptive tree on the 256^3 workload (mixed path): the hierarchy with
    piecewise-constant interpolation and Galerkin coarse operators, first
    unrefined (the reference), then with the finest level refined only on the
    subvolumes that hold all but a fraction f of the Haar detail energy of psi0
    (largest details first).  Per f: subvolumes refined, ms per step over the
    workload's first `steps` steps, V-cycles, and the relative difference of
    psi after them from the unrefined solution.  The default hierarchy (linear
    interpolation, rediscretised coarse operators) is timed for comparison."""
    import numpy as np
    import workloads as W
    cfg = W.config("3d_large")
    v0 = torch.as_tensor(W.potential(cfg), device="cuda")
    psi0 = torch.as_tensor(W.initial_state(cfg, W.potential(cfg)), device="cuda")

    def make(galerkin):
        return lam.Propagator(cfg["shape"], cfg["h"], v0, cfg["n_t"], cfg["dt"], (cfg["block"],) * cfg["dim"],
                              levels=cfg["levels"], nu_coarse=cfg["nu_coarse"],
                              coarse_reduction=cfg["coarse_reduction"], precision="mixed", tol=1e-10,
                              max_cycles=60, pulse=pulse_of(cfg), interp="constant" if galerkin else "linear",
                              coarse_op="galerkin" if galerkin else "rediscretised")

    def run(prop):
        prop.propagate(psi0.clone(), 1)   # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        psi, st = prop.propagate(psi0.clone(), steps)
        torch.cuda.synchronize()
        return psi, (time.perf_counter() - t) / steps * 1e3, st[0]["cycles"] / steps

    rows = []
    prop = make(False)
    _, ms, cyc = run(prop)
    rows.append({"hierarchy": "linear interpolation, rediscretised", "refined": 1.0, "ms_per_step": ms,
                 "cycles_per_step": cyc, "diff_from_unrefined": None})
    prop.close()
    prop = make(True)
    psi_full, ms, cyc = run(prop)
    rows.append({"hierarchy": "constant interpolation, Galerkin", "refined": 1.0, "ms_per_step": ms,
                 "cycles_per_step": cyc, "diff_from_unrefined": 0.0})
    det = prop.block_detail(psi0)
    order = np.argsort(det)[::-1]
    cum = np.cumsum(det[order])
    nfull = float(torch.linalg.vector_norm(psi_full))
    for f in fractions:
        keep = int(np.searchsorted(cum, (1.0 - f) * cum[-1]) + 1)
        mask = np.zeros(det.size, np.uint8)
        mask[order[:keep]] = 1
        prop.set_refinement(mask)
        psi, ms, cyc = run(prop)
        diff = float(torch.linalg.vector_norm(psi - psi_full)) / nfull
        rows.append({"hierarchy": "constant interpolation, Galerkin", "detail_left_out": f,
                     "refined": keep / det.size, "refined_subvolumes": keep, "ms_per_step": ms,
                     "cycles_per_step": cyc, "diff_from_unrefined": diff})
        print(f"[adaptive] f={f:g}: {keep} of {det.size} subvolumes refined, {ms:.2f} ms/step, "
              f"{cyc:.1f} cycles/step, |psi - psi_unrefined| / |psi_unrefined| = {diff:.2e}", file=sys.stderr,
              flush=True)
        prop.set_refinement(None)
    prop.close()
    return rows


def pulse_of(cfg):
    """The workload's pulse as Propagator arguments (None without a field)."""
    import workloads as W
    p = cfg["pulse"]
    if not p:
        return None
    return dict(kind=p["kind"], e0=p.get("e0", 0.0), omega=p.get("omega", 0.0), t_total=cfg["t_total"],
                coef=list(W.pulse_coefficients(cfg)))


def run_precision(args, precision, v0_t, psi0_t, cfg, torch, lam, adjoint_steps=0):
    shape = cfg["shape"]
    torch.cuda.synchronize()
    t_f = time.perf_counter()
    # context creation = hierarchy + factorisation of every block of every level (once per run for a
    # static potential)
    prop = lam.Propagator(shape, cfg["h"], v0_t, cfg["n_t"], cfg["dt"], (cfg["block"],) * cfg["dim"],
                          levels=cfg["levels"], nu_pre=1, nu_post=1, nu_coarse=cfg["nu_coarse"],
                          coarse_reduction=cfg["coarse_reduction"], precision=precision,
                          tol=args.tol, max_cycles=60, pulse=pulse_of(cfg))
    torch.cuda.synchronize()
    factor_ms = (time.perf_counter() - t_f) * 1e3
    # warm-up steps from the start of the pulse, then the timed steps again from the initial
    # state at t = 0: the timed region is the workload's own steps (with a field, its pulse)
    t = 0.0
    if args.warmup:
        prop.propagate(psi0_t.clone(), args.warmup, t_start=t)
    psi = psi0_t.clone()
    torch.cuda.synchronize()
    # HIP events around every 8th finest-level sweep launch of the timed steps (a sample: each
    # event record costs stream time)
    prop.profile(8)
    torch.cuda.synchronize()
    # the timed steps run back to back inside one lam_propagate call
    t_a = time.perf_counter()
    psi, stl = prop.propagate(psi, args.steps, t_start=t)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_a
    st = stl[0]
    launches, sweep_ms = prop.profile_read()
    prop.profile(0)
    # inner passes per subvolume: one more step solved at mid-pulse, outside the timed region
    # (the statistics describe each subvolume's last solve)
    prop.solve_step(0.5 * cfg["t_total"], psi0_t)
    hist, unsolved = prop.pass_stats(0)
    nblk = sum(hist)
    sweeps = st["sweeps_fine"]
    P = 1
    for s in shape:
        P *= s
    value = P * cfg["n_t"] * sweeps / elapsed / 1e6
    kernel_rate = P * cfg["n_t"] * 0.5 / (sweep_ms / launches / 1e3) / 1e6 if sweep_ms > 0 else None
    norm = float(torch.sum(torch.abs(psi) ** 2).item()) * cfg["h"] ** cfg["dim"]
    out = {
        "value": value,
        "ms_per_step": elapsed / args.steps * 1e3,
        "time_to_residual_ms": st["t_solve_ms"] / args.steps,
        "cycles_per_step": st["cycles"] / args.steps,
        "fine_sweeps_per_step": sweeps / args.steps,
        "final_resid_ratio_max": st["resid"] / st["resid0"],
        "sweep_launches": launches,
        "sweep_kernel_ms_avg": sweep_ms / launches if launches else None,
        "sweep_kernel_munk_sweeps_per_s": kernel_rate,
        "coarsest_sweeps_per_cycle": st["coarse_sweeps"] / max(1, st["cycles"]),
        "coarsest_solves_short_of_reduction": st["coarse_unmet"],
        "inner_passes_finest_mean": (sum(k * c for k, c in enumerate(hist)) / nblk) if nblk else 0.0,
        "inner_passes_finest_max": max([k for k, c in enumerate(hist) if c] + [0]),
        "subvolumes_unsolved_finest": unsolved,
        "norm_after": norm,
        "factor_ms": factor_ms,
    }
    if adjoint_steps:
        # backward steps of a loss of the final state (lam_adjoint_step: the step's forward
        # solve recomputed from its checkpoint, then the adjoint solve and the gradients)
        g = (psi / torch.sqrt(torch.sum(torch.abs(psi) ** 2))).contiguous()
        dv0 = torch.zeros(P, dtype=torch.float64, device=psi.device)
        dcoef = [0.0] * prop.n_coef
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        for k in range(adjoint_steps):
            t_k = (args.steps - 1 - k) * cfg["dt"]
            g, _ = prop.adjoint_step(t_k, psi, g, dv0, dcoef)
        torch.cuda.synchronize()
        out["adjoint_ms_per_step"] = (time.perf_counter() - t_b) / adjoint_steps * 1e3
        # the same backward steps from a stored forward solution (lam_adjoint_step_stored:
        # the adjoint solve and the gradients only; a caller keeps P N_t complex values per step)
        t_last = (args.steps - 1) * cfg["dt"]
        prop.solve_step(t_last, psi)
        c_fwd, _ = prop.get_state()
        g = (psi / torch.sqrt(torch.sum(torch.abs(psi) ** 2))).contiguous()
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        for k in range(adjoint_steps):
            t_k = (args.steps - 1 - k) * cfg["dt"]
            g, _ = prop.adjoint_step_stored(t_k, c_fwd, g, dv0, dcoef)
        torch.cuda.synchronize()
        out["adjoint_stored_ms_per_step"] = (time.perf_counter() - t_b) / adjoint_steps * 1e3
        del c_fwd
    prop.close()
    return out


def workload_string(cfg, tol):
    shape = "x".join(str(n) for n in cfg["shape"])
    pot = {"softcoulomb": "V=-1/sqrt(r^2+1)", "harmonic": "V=x^2/2"}[cfg["potential"]]
    p = cfg["pulse"]
    field = ""
    if p:
        field = {"sin2": f", E0={p['e0']} sin^2 pulse w={p['omega']}",
                 "fourier": f", {p['n_coef']}-amplitude Fourier pulse",
                 "sin2+fourier": f", E0={p['e0']} sin^2 pulse + {p['n_coef']} Fourier amplitudes"}[p["kind"]]
    blocks = "x".join([str(cfg["block"])] * cfg["dim"])
    return (f"{cfg['name']} {shape} h={cfg['h']:g} {pot}{field}, N_t={cfg['n_t']}, dt={cfg['dt']}, "
            f"{blocks} subvolumes, {cfg['levels']}-level V(1,1), coarsest level swept to a "
            f"{1 / cfg['coarse_reduction']:.0e} reduction (at most {cfg['nu_coarse']} sweeps), tol {tol:g}")


def sweep_kernel_name(cfg, prec):
    """The finest-level colour sweep kernel the library launches for this workload
    (the FP32 shared-factor sweep takes two time components per lane for N_t = 8 and
    N_t <= 4, with its block geometry fixed at compile time for 4 x 4 x 4 blocks in
    3D (3) and 8 x 8 blocks in 2D (2), else 0)."""
    nt = cfg["n_t"]
    if prec == "mixed" and (nt == 8 or nt <= 4):
        geo = 3 if (cfg["dim"] == 3 and cfg["block"] == 4) else (2 if (cfg["dim"] == 2 and cfg["block"] == 8) else 0)
        return f"k_sweep_pair<{nt}, {geo}>"
    return f"k_sweep<{nt}, {'double' if prec == 'fp64' else 'float'}, false>"


def roofline_of(cfg, prec, r, traffic):
    import numpy as np
    blocks = (cfg["block"],) * cfg["dim"]
    nb0, ncol0 = sweep_launch_bytes(cfg["shape"], blocks, cfg["n_t"], 0, prec)
    nb1, ncol1 = sweep_launch_bytes(cfg["shape"], blocks, cfg["n_t"], 1, prec)
    bytes_per_launch = 0.5 * (nb0 + nb1)
    avg = r["sweep_kernel_ms_avg"]
    achieved = bytes_per_launch / (avg * 1e-3) / 1e9 if avg else None
    # matrix-core work issued per launch and block solve: the two block transforms (points x
    # modes by the 2 N_t reals of the reduced block system) and the two per-mode mixes (modes x
    # 2 N_t by 2 N_t x 2 N_t), each over 16x16 output tiles with 16x16x4 steps, once per
    # solve (1 + the inner passes)
    b = int(np.prod(blocks))
    nc = 2 * cfg["n_t"]
    tiles = -(-b // 16) * -(-nc // 16)
    mfma_per_solve = 2 * tiles * 4 * (-(-b // 16)) + 2 * tiles * ((nc + 3) // 4)
    solves = 1.0 + r["inner_passes_finest_mean"]
    mfma_flops = 0.5 * (ncol0 + ncol1) * mfma_per_solve * solves * 2 * 16 * 16 * 4
    mfma_peak = 78.6 if prec == "fp64" else 157.3
    mfma_tf = mfma_flops / (avg * 1e-3) / 1e12 if avg else None
    kern = sweep_kernel_name(cfg, prec)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic,
            "kernel": f"{kern} (finest level, {ncol0 + ncol1} subvolumes per full sweep)",
            "bytes_per_launch": bytes_per_launch,
            "mfma": {"achieved": mfma_tf, "peak": mfma_peak, "unit": "TFLOP/s",
                     "frac": (mfma_tf / mfma_peak) if mfma_tf else None,
                     "note": "matrix-core FLOPs issued (16x16 tiles, padding included, inner passes counted)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE,
                    help="3d_large (the headline, default), 2d_softcoulomb, 1d_harmonic, 3d_laser, 2d_adjoint")
    ap.add_argument("--n", type=int, default=None, help="points per axis (default: the workload's)")
    ap.add_argument("--levels", type=int, default=None, help="multigrid levels (default: the workload's)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 2D soft-Coulomb extra block")
    ap.add_argument("--adjoint-steps", type=int, default=2,
                    help="backward steps timed on the headline precision (0: none)")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration)")
    ap.add_argument("--oracle-direct", action="store_true",
                    help="only time the oracle's direct step solve (SuperLU factor and solve, median of 3) "
                         "of the 2D soft-Coulomb workload at 64^2 and 128^2, on the host")
    ap.add_argument("--variants", action="store_true",
                    help="only measure the relaxation variants over groups of 2^d elements (separate, "
                         "simultaneous, intergrid transfer): residual ratio and time per iteration")
    ap.add_argument("--adaptive", action="store_true",
                    help="only measure the adaptive tree on the 256^3 workload (Galerkin piecewise-constant "
                         "hierarchy; finest level refined by Haar detail)")
    ap.add_argument("--plane-wave", action="store_true",
                    help="only compute the Legendre-element plane-wave convergence maps (128 x 128 trial "
                         "waves per regime, basis and mode) and summarise them")
    args = ap.parse_args()
    if args.adaptive:
        import torch
        from paper_1111_4363_amd import lam
        lam.load_library()
        print(json.dumps(adaptive_tree(torch, lam)))
        return
    if args.plane_wave:
        import torch
        from paper_1111_4363_amd import lam
        lam.load_library()
        print(json.dumps(plane_wave_maps(torch, lam)))
        return
    if args.variants:
        import torch
        from paper_1111_4363_amd import lam
        lam.load_library()
        print(json.dumps({p: relaxation_variants(torch, lam, p) for p in ("fp64", "mixed")}))
        return
    if args.oracle_direct:
        print(json.dumps(oracle_direct_2d()))
        return
    if args.copy_probe:
        import torch
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_launch": n * 8, "copy_probe_bytes_written_per_launch": n * 8,
                          "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the sharding design is described, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1111_4363_amd import lam
    import workloads as W

    lam.load_library()
    dev = torch.device("cuda:0")

    def run_workload(name, n=None, levels=None, precisions=("fp64", "mixed"), adjoint_for=None):
        cfg = W.config(name, n=n, levels=levels)
        v0 = W.potential(cfg)
        psi0 = W.initial_state(cfg, v0)
        v0_t = torch.as_tensor(v0, dtype=torch.float64, device=dev)
        psi0_t = torch.as_tensor(psi0, dtype=torch.complex128, device=dev)
        res = {}
        for prec in precisions:
            print(f"[bench] {name} {prec}: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr,
                  flush=True)
            res[prec] = run_precision(args, prec, v0_t, psi0_t, cfg, torch, lam,
                                      adjoint_steps=args.adjoint_steps if prec == adjoint_for else 0)
        del v0_t, psi0_t
        torch.cuda.empty_cache()
        return cfg, res

    precs = ("fp64", "mixed") if args.precision == "both" else (args.precision,)
    # the headline precision: mixed for workloads that name it (a field and FP32 block solves), else FP64
    main_prec = "mixed" if ("mixed" in precs and args.workload in ("3d_large", "3d_laser")) else precs[0]
    if main_prec not in precs:
        main_prec = precs[0]
    cfg, res = run_workload(args.workload, args.n, args.levels, precs, adjoint_for=main_prec)
    r = res[main_prec]
    full_size = args.n is None and args.levels is None
    traffic = counters_for_current_kernel(f"{args.workload}/{main_prec}") if full_size else None
    roofline = roofline_of(cfg, main_prec, r, traffic)

    extra = None
    if not args.no_extra and args.workload == HEADLINE and full_size:
        c2, r2 = run_workload("2d_softcoulomb", precisions=precs)
        p2 = "fp64" if "fp64" in r2 else precs[0]
        extra = {"2d_softcoulomb": {"config": workload_string(c2, args.tol), "precisions": r2,
                                    "roofline": roofline_of(c2, p2, r2[p2],
                                                            counters_for_current_kernel(f"2d_softcoulomb/{p2}"))}}

    cpu = None
    if not args.no_cpu_baseline and full_size:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload)

    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "Munknowns·sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload_string(cfg, args.tol), "precision": main_prec,
                   "grid": list(cfg["shape"]), "n_t": cfg["n_t"], "levels": cfg["levels"],
                   "unknowns_per_step": int(np.prod(cfg["shape"])) * (cfg["n_t"] + 1)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_residual_ms": {p: res[p]["time_to_residual_ms"] for p in res},
        "precisions": res,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
