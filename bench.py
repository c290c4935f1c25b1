"""Benchmark of the least-action relaxation path on one MI355X.

Workload: the 2D soft-Coulomb problem, 512 x 512 points, h = 0.2,
V = -1/sqrt(r^2 + 1), N_t = 8 Legendre time functions, dt = 0.05, 8 x 8
subvolumes, 5-level V(1,1) cycles, random-phase Gaussian initial state
(seed 0), steps solved to sqrt(N/N0) <= 1e-10.  A "step" is one propagation
time step: every kernel of the path (residual, colour sweeps on all levels,
projection, interpolation, coarse sweeps, step I/O) until the tolerance.

value: finest-level Munknowns*sweeps/s = P * N_t * (finest full sweeps done
in the timed steps) / (wall time of the timed steps) / 1e6, FP64 path.
The mixed path (FP32 subvolume solves) is reported next to it, with the
time to reach the 1e-10 residual per step for both.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512] [--levels 5]
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


def sweep_launch_bytes(shape, block, n_t, colour, precision):
    """Algorithmic HBM bytes of one finest-level colour launch (forward step).

    Per block of b points: its eigenvectors, b^2 reals (8 B FP64, 4 B mixed),
    its b eigenvalues (FP64) and frozen-field shift (8 B), its id (4 B).  Per
    own point: read c (N_t complex FP64), lambda, the constraint right-hand
    side (complex) and V0 (real); write c and lambda.  Per distinct halo point
    of the launch: read c (N_t complex).  The shared time factor (3 (N_t+1)^2
    complex, under 4 KB) is read once per launch and not counted.
    """
    import numpy as np
    nblk = [s // b for s, b in zip(shape, block)]
    b = int(np.prod(block))
    rb = 8 if precision == "fp64" else 4
    coords = np.indices(nblk).reshape(len(nblk), -1).T
    ncol = int(np.sum(coords.sum(axis=1) % 2 == colour))
    per_block = b * b * rb + b * 8 + 8 + 4
    per_point = (n_t * 16 + 16 + 16 + 8) + (n_t * 16 + 16)
    # distinct halo points: points outside a colour block, face-adjacent to one
    owner_colour = np.zeros(shape, dtype=np.int8)
    idx = np.indices(shape)
    for a in range(len(shape)):
        owner_colour += (idx[a] // block[a]).astype(np.int8)
    owner_colour %= 2
    inside = owner_colour == colour
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


def counters_for_current_kernel():
    """Traffic per launch from committed rocprofv3 counters, if taken on this kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    try:
        with open(COUNTERS) as f:
            rec = json.load(f)
        with open(KERNEL_SOURCE, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
        if rec.get("kernel_source_sha256") != digest:
            return None
        return rec.get("traffic_bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(budget_s=20.0):
    """The oracle's plain-loop colour sweeps on a 64 x 64 window of the workload."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    import workloads as W
    from oracle import grid as G
    from oracle import kkt, relax
    cfg = W.config("2d_softcoulomb", n=64)
    v0 = W.potential(cfg)
    psi0 = W.initial_state(cfg, v0)
    g = G.Grid(cfg["shape"], cfg["h"])
    sysm = kkt.StepSystem(g, v0, cfg["n_t"], cfg["dt"])
    b = kkt.rhs(sysm, psi0)
    x = kkt.initial_guess(sysm, psi0)
    bl = G.blocks(g, (cfg["block"],) * 2)
    sweeps = 0
    t_a = time.perf_counter()
    while True:
        x = relax.reference_sweep(sysm.K, b, x, bl, g.npts, cfg["n_t"])
        sweeps += 1
        if time.perf_counter() - t_a > budget_s or sweeps >= 60:
            break
    dt = time.perf_counter() - t_a
    value = g.npts * cfg["n_t"] * sweeps / dt / 1e6
    return {"value": value, "unit": "Munknowns·sweeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{sweeps} full colour sweeps (plain-loop dense local solves) of the same workload's "
                      f"8x8 subvolumes on a 64x64 window (64 of its 4096 blocks), {dt:.1f} s"}


def pulse_of(cfg):
    """The workload's pulse as Propagator arguments (None without a field)."""
    import workloads as W
    p = cfg["pulse"]
    if not p:
        return None
    return dict(kind=p["kind"], e0=p.get("e0", 0.0), omega=p.get("omega", 0.0), t_total=cfg["t_total"],
                coef=list(W.pulse_coefficients(cfg)))


def run_precision(args, precision, v0_t, psi0_t, cfg, torch, lam):
    shape = cfg["shape"]
    torch.cuda.synchronize()
    t_f = time.perf_counter()
    # context creation = hierarchy + factorisation of every block of every level (once per run for a
    # static potential)
    prop = lam.Propagator(shape, cfg["h"], v0_t, cfg["n_t"], cfg["dt"], (cfg["block"],) * cfg["dim"],
                          levels=cfg["levels"], nu_pre=1, nu_post=1, nu_coarse=cfg["nu_coarse"], precision=precision,
                          tol=args.tol, max_cycles=60, pulse=pulse_of(cfg))
    torch.cuda.synchronize()
    factor_ms = (time.perf_counter() - t_f) * 1e3
    psi = psi0_t.clone()
    t = 0.0
    if args.warmup:
        psi, _ = prop.propagate(psi, args.warmup, t_start=t)
        t += args.warmup * cfg["dt"]
    torch.cuda.synchronize()
    # HIP events around every 8th finest-level sweep launch of the timed steps (a sample: each
    # event record costs stream time, so recording all 16 launches of a step would slow it ~5%)
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
    sweeps = st["sweeps_fine"]
    P = 1
    for s in shape:
        P *= s
    value = P * cfg["n_t"] * sweeps / elapsed / 1e6
    kernel_rate = P * cfg["n_t"] * 0.5 / (sweep_ms / launches / 1e3) / 1e6 if sweep_ms > 0 else None
    norm = float(torch.sum(torch.abs(psi) ** 2).item()) * cfg["h"] ** cfg["dim"]
    prop.close()
    return {
        "value": value,
        "ms_per_step": elapsed / args.steps * 1e3,
        "time_to_residual_ms": st["t_solve_ms"] / args.steps,
        "cycles_per_step": st["cycles"] / args.steps,
        "fine_sweeps_per_step": sweeps / args.steps,
        "final_resid_ratio_max": st["resid"] / st["resid0"],
        "sweep_launches": launches,
        "sweep_kernel_ms_avg": sweep_ms / launches if launches else None,
        "sweep_kernel_munk_sweeps_per_s": kernel_rate,
        "norm_after": norm,
        "factor_ms": factor_ms,
    }


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
            f"{blocks} subvolumes, {cfg['levels']}-level V(1,1) with {cfg['nu_coarse']} coarsest sweep(s), tol {tol:g}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="2d_softcoulomb",
                    help="2d_softcoulomb (the headline, default), 1d_harmonic, 3d_laser, 2d_adjoint, 3d_large")
    ap.add_argument("--n", type=int, default=None, help="points per axis (default: the workload's)")
    ap.add_argument("--levels", type=int, default=None, help="multigrid levels (default: the workload's)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration)")
    args = ap.parse_args()
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
    cfg = W.config(args.workload, n=args.n, levels=args.levels)
    v0 = W.potential(cfg)
    psi0 = W.initial_state(cfg, v0)
    dev = torch.device("cuda:0")
    v0_t = torch.as_tensor(v0, dtype=torch.float64, device=dev)
    psi0_t = torch.as_tensor(psi0, dtype=torch.complex128, device=dev)

    res = {}
    for prec in (["fp64", "mixed"] if args.precision == "both" else [args.precision]):
        print(f"[bench] {prec}: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr, flush=True)
        res[prec] = run_precision(args, prec, v0_t, psi0_t, cfg, torch, lam)
    main_prec = "fp64" if "fp64" in res else "mixed"
    r = res[main_prec]

    blocks = (cfg["block"],) * cfg["dim"]
    nb0, ncol0 = sweep_launch_bytes(cfg["shape"], blocks, cfg["n_t"], 0, main_prec)
    nb1, ncol1 = sweep_launch_bytes(cfg["shape"], blocks, cfg["n_t"], 1, main_prec)
    bytes_per_launch = 0.5 * (nb0 + nb1)
    achieved = bytes_per_launch / (r["sweep_kernel_ms_avg"] * 1e-3) / 1e9 if r["sweep_kernel_ms_avg"] else None
    traffic = counters_for_current_kernel() if (args.workload == "2d_softcoulomb" and args.n is None) else None
    # matrix-core work issued per launch: per block, the two block transforms (points x modes
    # by the 2 N_t reals of the reduced block system) and the two per-mode mixes (modes x
    # 2 N_t by 2 N_t x 2 N_t), each over 16x16 output tiles with 16x16x4 steps
    b = int(np.prod(blocks))
    nc = 2 * cfg["n_t"]
    tiles = -(-b // 16) * -(-nc // 16)
    mfma_per_block = 2 * tiles * 4 * (-(-b // 16)) + 2 * tiles * ((nc + 3) // 4)
    mfma_flops = 0.5 * (ncol0 + ncol1) * mfma_per_block * 2 * 16 * 16 * 4
    mfma_peak = 78.6 if main_prec == "fp64" else 157.3
    mfma_tf = mfma_flops / (r["sweep_kernel_ms_avg"] * 1e-3) / 1e12 if r["sweep_kernel_ms_avg"] else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": traffic,
                "kernel": f"k_sweep<{cfg['n_t']}, {'double' if main_prec == 'fp64' else 'float'}, false> (finest level)",
                "bytes_per_launch": bytes_per_launch,
                "mfma": {"achieved": mfma_tf, "peak": mfma_peak, "unit": "TFLOP/s",
                         "frac": (mfma_tf / mfma_peak) if mfma_tf else None,
                         "note": "matrix-core FLOPs issued (16x16 tiles, padding included)"}}

    cpu = None
    if not args.no_cpu_baseline and args.workload == "2d_softcoulomb":
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

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
        "config": {"workload": workload_string(cfg, args.tol),
                   "grid": list(cfg["shape"]), "n_t": cfg["n_t"], "levels": cfg["levels"],
                   "unknowns_per_step": int(np.prod(cfg["shape"])) * (cfg["n_t"] + 1)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_residual_ms": {p: res[p]["time_to_residual_ms"] for p in res},
        "precisions": res,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
