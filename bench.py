"""Benchmark of the limited D2Q9 step on one MI355X.

Default workload: D2Q9 periodic Taylor-Green vortex plus a seeded random-phase
perturbation on 4096 x 4096 nodes, FP32 shifted SoA storage, nu = 1e-4,
entropy trimming and the 3x3 median filter both on (delta = 1e-4),
polynomial f*, quadratic Delta S, FP64 global reductions every step.  One
step = one fused launch (free flight, collision, Delta S, both limiters,
store, reduction of the previous step's partials).

Prints one JSON line: MLUPS of the whole job, the roofline of the step
kernel (algorithmic bytes / kernel time vs 8 TB/s HBM), and the FP64 CPU
oracle timed on the host on a 1024 x 1024 replica of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_d2q9_f32_4096.json")
KERNEL_SOURCES = ["paper_0704_0043_amd/csrc/step.hip", "paper_0704_0043_amd/csrc/lbm_device.h",
                  "paper_0704_0043_amd/csrc/lbm_common.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def c2_domain(L, wl, n=4096, storage=None):
    nu = 1e-4
    rho, u = wl.taylor_green(n, u0=0.05, mode=1, perturb=1e-3, seed=wl.DEFAULT_SEED)
    return L.Domain(lattice=L.LBM_D2Q9, nx=n, ny=n, beta=wl.beta_from_nu(nu), qe=L.LBM_QE_POLYNOMIAL,
                    limiter=L.LBM_LIM_TRIM | L.LBM_LIM_MEDIAN, ds_form=L.LBM_DS_QUADRATIC, bc=L.LBM_BC_PERIODIC,
                    delta_trim=1e-4, delta_median=1e-4, rho0=1.0, rho_init=rho, u_init=u)


def shear_domain(L, wl, n=8192):
    rho, u = wl.double_shear_layer(n, u0=0.05, kappa=80.0, eps=0.05)
    return L.Domain(lattice=L.LBM_D2Q9, nx=n, ny=n, beta=wl.beta_from_nu(5e-5), qe=L.LBM_QE_POLYNOMIAL,
                    limiter=L.LBM_LIM_TRIM, ds_form=L.LBM_DS_QUADRATIC, bc=L.LBM_BC_PERIODIC,
                    delta_trim=1e-4, rho0=1.0, rho_init=rho, u_init=u)


def time_steps(torch, L, ctx, stream, steps, warmup):
    L.lbm_step(ctx, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.lbm_step(ctx, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)          # ms


def cpu_baseline(wl, seconds=12.0):
    """The FP64 oracle (single thread) on a 1024 x 1024 replica of the workload."""
    from oracle import oracle as orc
    n = 1024
    rho, u = wl.taylor_green(n, u0=0.05, mode=1, perturb=1e-3, seed=wl.DEFAULT_SEED)
    p = orc.make_params(lattice=2, nx=n, ny=n, beta=wl.beta_from_nu(1e-4), qe=0, ds_form=1, limiter=3,
                        delta_trim=1e-4, delta_median=1e-4, bc=0)
    f = orc.init_equilibrium(p, rho, u)
    steps = 0
    t0 = time.perf_counter()
    while True:
        orc.step(p, f, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 1000:
            break
    return {"value": round(n * n * steps / el / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 C oracle, single thread, {steps} steps of a {n}x{n} replica (same nu, U0, mode, "
                      f"limiters, quadratic dS), {el:.1f} s"}


def load_traffic():
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--variants", action="store_true", help="also time FP16/BF16 8192^2 and the cavity batch")
    ap.add_argument("--tile-h", type=int, default=0, help="fixed rows per wave tile instead of autotuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of 1 GiB (known bytes) to scale HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0704_0043_amd import lbm as L
    from paper_0704_0043_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.init()
    stream = torch.cuda.Stream()
    n = args.n
    dom = c2_domain(L, wl, n)
    print(f"[bench] creating {n}x{n} FP32 context", file=sys.stderr, flush=True)
    run = L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, graph_chunk=64)
    if args.tile_h:
        run.tile_h = args.tile_h
    ctx = L.lbm_create([dom], run)
    tile = L.lbm_tile_config(ctx)
    print(f"[bench] tile {tile}; warmup {args.warmup}, timing {args.steps} steps", file=sys.stderr, flush=True)
    ms = time_steps(torch, L, ctx, stream, args.steps, args.warmup)
    stats = L.lbm_entropy_stats(ctx)
    sites = n * n
    ms_step = ms / args.steps
    mlups = sites * args.steps / (ms * 1e3)
    bytes_per_site = 2 * 9 * 4
    bytes_launch = bytes_per_site * sites
    achieved = bytes_launch / (ms_step * 1e-3) / 1e9
    traffic = load_traffic()
    out = {
        "metric": "MLUPS + % HBM roofline, limited D2Q9 step; batched/low-precision vs plain FP32",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"D2Q9 periodic Taylor-Green + random-phase perturbation {n}x{n}, FP32 shifted SoA, "
                        "nu=1e-4, trimming + 3x3 median limiter (delta=1e-4), polynomial f*, quadratic dS, "
                        "FP64 stats every step",
            "nx": n, "ny": n, "storage": "f32_shift", "tile": list(tile), "graph_chunk": 64,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "stats": {"mass": stats["mass"], "n_trimmed": stats["n_trimmed"], "n_filtered": stats["n_filtered"],
                  "max_dS": stats["max_dS"], "n_nonfinite": stats["n_nonfinite"]},
    }
    ctx.close()
    if args.calibrate_copy:
        out["copy_calibration"] = copy_calibration(torch, stream)
    if args.variants:
        out["variants"] = variants(torch, L, wl, stream, args)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def copy_calibration(torch, stream, nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of `nbytes` (read nbytes, write nbytes):
    its FETCH_SIZE / WRITE_SIZE counters give the scale of those counters."""
    a = torch.ones(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        for _ in range(reps):
            b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "launches": reps}


def variants(torch, L, wl, stream, args):
    res = {}
    steps = max(50, args.steps // 4)
    for name, storage in (("f32_8192", L.LBM_F32), ("f16_8192", L.LBM_F16_SHIFT), ("bf16_8192", L.LBM_BF16_SHIFT)):
        print(f"[bench] variant {name}", file=sys.stderr, flush=True)
        dom = shear_domain(L, wl)
        with L.lbm_create([dom], L.Run(storage=storage, stream=stream.cuda_stream)) as ctx:
            ms = time_steps(torch, L, ctx, stream, steps, 16)
        sites = dom.nx * dom.ny
        b = 2 * 9 * L.STORAGE_BYTES[storage]
        res[name] = {"mlups": round(sites * steps / (ms * 1e3), 1), "ms_per_step": round(ms / steps, 5),
                     "hbm_frac": round(b * sites / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "steps": steps}
    return res


if __name__ == "__main__":
    main()
