"""Benchmark of the limited D2Q9 step on one MI355X.

Default workload: D2Q9 periodic Taylor-Green vortex plus a seeded random-phase
perturbation on 4096 x 4096 nodes, FP32 shifted SoA storage, nu = 1e-4,
entropy trimming and the 3x3 median filter both on (delta = 1e-4),
polynomial f*, quadratic Delta S.  One step = the collision kernel (free
flight, moments, f*, over-relaxation, Delta S', trimming, store, one partial
of the reduction terms per workgroup) plus the median kernel (3x3 median of
Delta S', the filtered nodes rescaled in place); every step runs inside
captured HIP graphs (chunks of 64 steps and the powers of two below, captured
when the context is created), and the FP64 global stats of the last step are
formed inside the timed region.

Prints one JSON line: MLUPS of the whole job; the roofline of the dominant
kernel (the collision kernel: algorithmic bytes of the step divided by that
kernel's average duration, measured with HIP events on its stream after half
a second of graph steps has brought the clocks to their sustained level; this
measurement runs before the warm-up and timed steps); the roofline of the
whole step; the same step with the
median filter moving a few (delta_median = 1e-9) and some ten percent
(delta_median = 0) of the nodes, with the two kernels, with the fused step
and adaptively (LBM_RUN_ADAPTIVE); the
max-norm error of a 1024 x 1024 replica against the FP64 CPU oracle; and that
oracle timed on the host on the replica (its OpenMP build on the host's cores,
and one thread).

--variants adds the reduced-precision runs (FP16 / BF16 shifted storage on
an 8192 x 8192 double shear layer, against FP32 on the same input), the
headline step with the median filter active in every tile, the headline step
with each ensemble-dependent limiter added, and the batched ensemble of 256
lid-driven cavities (one launch per step for all of them, against the same
cavities run one by one).

--hopf runs, instead of the benchmark, the first-Hopf-bifurcation experiment
(a batch of 100 x 100 cavities with diffusive walls over a range of Re for
5000 non-dimensional time units each) and prints its analysis;
--hopf-continuation its hysteresis test (continuation down from an
oscillating state and up from a steady one).

--summarize-pmc FETCH_CSV WRITE_CSV turns two rocprofv3 --pmc runs of this
script (FETCH_SIZE, then WRITE_SIZE, with --calibrate-copy) into a table of
each kernel's HBM bytes and the traffic record the roofline reports (not
with --no-record).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE = {0: 144, 1: 72, 2: 36, 3: 36}     # read Q + write Q populations, D2Q9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_collide2d_f32_4096.json")
KERNEL_SOURCES = ["paper_0704_0043_amd/csrc/step.hip", "paper_0704_0043_amd/csrc/lbm_device.h",
                  "paper_0704_0043_amd/csrc/lbm_common.h"]
DOMINANT = "k_collide2d<float, 0, 1, 0, false>"
COPY_BYTES = 1 << 30


def kernel_hash() -> str:
    """Hash of the kernel sources' code: comments and layout left out, so a
    change of wording does not count as a change of the kernel."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def c2_domain(L, wl, n=4096):
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
    """ms for `steps` steps plus the FP64 reduction of the last step's stats
    (the reduction runs on the same stream before the closing event)."""
    L.lbm_step(ctx, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.lbm_step(ctx, steps)
    L.lbm_entropy_stats(ctx, 0)       # forms the stats of every domain
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)          # ms


REPLICA_N = 1024


def replica_params(orc, wl, dom, n=REPLICA_N):
    """Oracle parameters of an n x n replica of the timed domain (same nu,
    U0, mode, perturbation, limiters and Delta S form) and its initial fields."""
    rho, u = wl.taylor_green(n, u0=0.05, mode=1, perturb=1e-3, seed=wl.DEFAULT_SEED)
    p = orc.make_params(lattice=2, nx=n, ny=n, beta=dom.beta, ds_form=dom.ds_form, bc=0, qe=dom.qe,
                        limiter=dom.limiter, delta_trim=dom.delta_trim, delta_median=dom.delta_median,
                        collision=dom.collision, ens_k=dom.ens_k, delta_ens=dom.delta_ens, ens_c=dom.ens_c)
    return p, rho, u


def run_oracle_for(orc, p, f, seconds, handle=None, max_steps=2000):
    """Step the oracle one step at a time until `seconds` have passed; every
    step records its mask and Delta S' (kept for the last).  Returns
    (steps, elapsed, (stats, mask, dS) of the last step)."""
    steps, el, rec = 0, 0.0, None
    t0 = time.perf_counter()
    while steps < max_steps and el < seconds:
        steps += 1
        rec = orc.step(p, f, 1, record=True, handle=handle)
        el = time.perf_counter() - t0
    return steps, el, rec


def cpu_baseline(wl, seconds=24.0, dom=None):
    """The FP64 oracle on a 1024 x 1024 replica of the timed workload, timed
    on the host: its plain build on one thread for half of `seconds`, then its
    OpenMP build (per-node loops over rows, on the host's cores) for the other
    half.  Returns the baseline record and the OpenMP leg's final state (for
    the error statement of the GPU replica)."""
    from oracle import oracle as orc
    n = REPLICA_N
    p, rho, u = replica_params(orc, wl, dom, n)
    f1 = orc.init_equilibrium(p, rho, u)
    s1, e1, _ = run_oracle_for(orc, p, f1, seconds / 2)
    handle = orc.timing_lib()
    threads = int(handle.orc_threads())
    f2 = orc.init_equilibrium(p, rho, u)
    s2, e2, rec = run_oracle_for(orc, p, f2, seconds / 2, handle=handle)
    single = round(n * n * s1 / e1 / 1e6, 3)
    multi = round(n * n * s2 / e2 / 1e6, 3)
    base = {"value": multi, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "per_core": round(multi / threads, 3), "single_thread": single,
            "host_cpus_allowed": len(os.sched_getaffinity(0)),
            "sample": f"FP64 C oracle on a {n}x{n} replica of the timed workload (same nu, U0, mode, perturbation, "
                      f"limiters, dS form): OpenMP build on {threads} threads, {s2} steps in {e2:.1f} s; plain "
                      f"build on one thread, {s1} steps in {e1:.1f} s (a baseline only)"}
    return base, (s2, f2, rec)


def replica_error(L, stream, dom, wl, oracle_run):
    """Max-norm error of the GPU step (FP32 storage) against the FP64 oracle
    on the 1024 x 1024 replica after the oracle's own number of steps:
    rho / rho0, u / max|u_oracle|, Delta S' of the last step / its largest
    oracle value, and the limiter masks of that step."""
    import numpy as np
    steps, f_o, (st_o, mask_o, ds_o) = oracle_run
    n = REPLICA_N
    rho_i, u_i = wl.taylor_green(n, u0=0.05, mode=1, perturb=1e-3, seed=wl.DEFAULT_SEED)
    d = L.Domain(lattice=L.LBM_D2Q9, nx=n, ny=n, beta=dom.beta, qe=dom.qe, limiter=dom.limiter,
                 ds_form=dom.ds_form, bc=L.LBM_BC_PERIODIC, delta_trim=dom.delta_trim,
                 delta_median=dom.delta_median, rho0=1.0, collision=dom.collision, ens_c=dom.ens_c,
                 ens_k=dom.ens_k, delta_ens=dom.delta_ens, rho_init=rho_i, u_init=u_i)
    with L.lbm_create([d], L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, flags=L.LBM_RUN_RECORD)) as ctx:
        L.lbm_step(ctx, steps)
        rho, u = L.lbm_moments(ctx)
        mask, ds = L.lbm_limiter_mask(ctx)
    vx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    vy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    r_o = f_o.sum(axis=0)
    ux_o = np.tensordot(vx, f_o, axes=1) / r_o
    uy_o = np.tensordot(vy, f_o, axes=1) / r_o
    umax = max(np.abs(ux_o).max(), np.abs(uy_o).max())
    dsmax = float(np.abs(ds_o).max())
    return {"replica": f"{n}x{n}", "steps": steps, "storage": "f32_shift",
            "rho_rel": float(np.abs(rho - r_o).max() / 1.0),
            "u_rel": float(max(np.abs(u[0] - ux_o).max(), np.abs(u[1] - uy_o).max()) / umax),
            "dS_rel": float(np.abs(ds - ds_o).max() / dsmax) if dsmax > 0 else 0.0,
            "mask_mismatches": int((mask != mask_o).sum()), "oracle_max_dS": dsmax, "gate_rho_u": 1e-5}


def workload_text(n, workload="headline", delta_median=1e-4):
    """The `config.workload` description of the timed run."""
    limiters = ("trimming + 3x3 median limiter (delta=1e-4)" if delta_median == 1e-4 else
                f"trimming (delta=1e-4) + 3x3 median limiter (delta={delta_median:g})")
    if workload == "smooth":
        limiters += " + smooth ensemble factor (k=0.5, delta=0.01)"
    elif workload == "elbm":
        limiters = "ELBM collisions, no limiter"
    feq = "entropic f*" if workload == "elbm" else "polynomial f*"
    return (f"D2Q9 periodic Taylor-Green + random-phase perturbation {n}x{n}, FP32 shifted SoA, "
            f"nu=1e-4, {limiters}, {feq}, quadratic dS, "
            "per-workgroup partials every step, FP64 global stats of the last step")


def kernel_times_warm(L, ctx, steps=50, warm_seconds=0.5):
    """Average collision and second-pass kernel durations (ms) over `steps`
    eager steps with HIP events on the context's stream, after graph steps
    have kept the GPU busy for at least `warm_seconds` (clocks settled)."""
    t0 = time.perf_counter()
    warm = 0
    while time.perf_counter() - t0 < warm_seconds:
        L.lbm_step(ctx, 256)
        L.lbm_synchronize(ctx)
        warm += 256
    k1, k2 = L.lbm_kernel_times(ctx, steps)
    return k1, k2, {"warmup_graph_steps": warm, "warmup_s": round(time.perf_counter() - t0, 3),
                    "timed_steps": steps, "mode": "eager launches, HIP events on the context stream"}


def median_active(torch, L, wl, stream, n, steps=200, warmup=192):
    """The headline step with the median tolerance below the Delta S' of most
    nodes (delta_median = 1e-9, and 0): the filter moves a few percent (some
    fifteen percent) of the nodes every step.  Timed with the two kernels as
    tuned (the second pass rescales the moved nodes' stored states), with the
    fused step (tile_x = 248, collision and filter in one pass), and adaptive
    (LBM_RUN_ADAPTIVE: the two kernels first, the fused step from the second
    64-step point on once the filter moves more than 0.5 % of the nodes),
    each after `warmup` steps from the start."""
    sites = n * n
    out = {}
    for dmed in (1e-9, 0.0):
        res = {}
        for name, tile_x, flags in (("two_kernels", 0, 0), ("fused", 248, 0), ("adaptive", 0, L.LBM_RUN_ADAPTIVE)):
            dom = c2_domain(L, wl, n)
            dom.delta_median = dmed
            with L.lbm_create([dom], L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, tile_x=tile_x,
                                           flags=flags)) as ctx:
                ms = time_steps(torch, L, ctx, stream, steps, warmup)
                tile = L.lbm_tile_config(ctx)
                st = L.lbm_entropy_stats(ctx)
                k1, k2, _ = kernel_times_warm(L, ctx, 20, 0.2)
            res[name] = {"mlups": round(sites * steps / (ms * 1e3), 1), "ms_per_step": round(ms / steps, 5),
                         "tile": list(tile), "first_kernel_ms": round(k1, 5), "second_kernel_ms": round(k2, 5),
                         "filtered_fraction": round(st["n_filtered"] / sites, 4),
                         "step_hbm_frac": round(72 * sites / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        out[f"delta_median_{dmed:g}"] = dict(res, steps=steps, warmup=warmup)
    return out


def load_traffic():
    """HBM bytes per launch of the dominant kernel from the committed PMC
    record, or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def copy_calibration(torch, stream, nbytes=COPY_BYTES, reps=3):
    """A plain elementwise kernel over `nbytes` (reads nbytes, writes nbytes):
    its FETCH_SIZE / WRITE_SIZE counters give the scale of those counters."""
    a = torch.rand(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(reps):
            torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "launches": reps}


def shear_run(torch, L, wl, stream, storage, steps, warmup=16):
    """The 8192^2 double shear layer (trimming only) in one storage type."""
    dom = shear_domain(L, wl)
    with L.lbm_create([dom], L.Run(storage=storage, stream=stream.cuda_stream, graph_chunk=64)) as ctx:
        ms = time_steps(torch, L, ctx, stream, steps, warmup)
        k1, k2, _ = kernel_times_warm(L, ctx, 20, 0.2)
    sites = dom.nx * dom.ny
    b = BYTES_PER_SITE[storage] * sites
    return {"mlups": round(sites * steps / (ms * 1e3), 1), "ms_per_step": round(ms / steps, 5),
            "step_hbm_frac": round(b / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "collide_ms": round(k1, 5), "steps": steps}


SHEAR_STORAGE = {"shear-f32": "f32", "shear-f16": "f16", "shear-bf16": "bf16"}


def variants(torch, L, wl, stream, args):
    res = {}
    steps = max(50, args.steps // 4)
    shear = {}
    for name, storage in (("f32", L.LBM_F32), ("f16", L.LBM_F16_SHIFT), ("bf16", L.LBM_BF16_SHIFT)):
        print(f"[bench] variant shear 8192^2 {name}", file=sys.stderr, flush=True)
        shear[name] = shear_run(torch, L, wl, stream, storage, steps)
    for name in ("f16", "bf16"):
        shear[name]["vs_f32"] = round(shear[name]["mlups"] / shear["f32"]["mlups"], 3)
    res["shear_8192"] = shear

    # the headline step with the median filter working in every tile: delta
    # below the Delta S' of most nodes (the headline's delta is above all of
    # them, so there every median tile finds no candidate and skips)
    print("[bench] variant 4096^2 with the median filter active", file=sys.stderr, flush=True)
    act = {}
    for dmed in (1e-9, 0.0):
        dom = c2_domain(L, wl, 4096)
        dom.delta_median = dmed
        with L.lbm_create([dom], L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, graph_chunk=64)) as ctx:
            ms = time_steps(torch, L, ctx, stream, steps, 16)
            st = L.lbm_entropy_stats(ctx)
            k1, k2, _ = kernel_times_warm(L, ctx, 20, 0.2)
        sites = dom.nx * dom.ny
        act[f"delta_median={dmed:g}"] = {
            "mlups": round(sites * steps / (ms * 1e3), 1), "ms_per_step": round(ms / steps, 5),
            "collide_ms": round(k1, 5), "median_ms": round(k2, 5),
            "filtered_fraction": round(st["n_filtered"] / sites, 4), "steps": steps}
    res["median_active_4096"] = act

    # the headline grid with each ensemble-dependent limiter added to trimming
    # and the median filter: E(Delta S') reduced every step, then (budget) the
    # radix selection of the threshold, then the second pass with the factors
    print("[bench] variant 4096^2 with ensemble-dependent limiters", file=sys.stderr, flush=True)
    ens = {}
    for name, lim, kw in (("threshold_cE", L.LBM_LIM_ENS_THRESHOLD, dict(ens_c=5.0)),
                          ("smooth_k0.5", L.LBM_LIM_ENS_SMOOTH, dict(ens_k=0.5, delta_ens=0.01)),
                          ("rational_k1", L.LBM_LIM_ENS_RATIONAL, dict(ens_c=2.0, ens_k=1.0)),
                          ("budget", L.LBM_LIM_ENS_BUDGET, dict(ens_c=0.05))):
        dom = c2_domain(L, wl, 4096)
        dom.limiter |= lim
        for k, v in kw.items():
            setattr(dom, k, v)
        with L.lbm_create([dom], L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, graph_chunk=64)) as ctx:
            ms = time_steps(torch, L, ctx, stream, steps, 16)
            st = L.lbm_entropy_stats(ctx)
            k1, k2, _ = kernel_times_warm(L, ctx, 20, 0.2)
        sites = dom.nx * dom.ny
        ens[name] = {"mlups": round(sites * steps / (ms * 1e3), 1), "ms_per_step": round(ms / steps, 5),
                     "collide_ms": round(k1, 5), "rest_ms": round(k2, 5),
                     "moved_fraction": round(st["n_ensemble"] / sites, 4),
                     "threshold": st["ens_threshold"], "mean_dS": st["mean_dS"], "steps": steps}
    res["ensemble_limiters_4096"] = ens

    # ELBM collisions (a root solve per node: arithmetic-bound) on the
    # headline grid without limiters, FP32 storage, against LBGK on the same
    print("[bench] variant 4096^2 ELBM vs LBGK", file=sys.stderr, flush=True)
    coll = {}
    for name, cv in (("lbgk", L.LBM_COLL_LBGK), ("elbm", L.LBM_COLL_ELBM)):
        dom = c2_domain(L, wl, 4096)
        dom.qe, dom.limiter, dom.collision = L.LBM_QE_ENTROPIC, L.LBM_LIM_NONE, cv
        with L.lbm_create([dom], L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, graph_chunk=64)) as ctx:
            ms = time_steps(torch, L, ctx, stream, steps, 16)
            st = L.lbm_entropy_stats(ctx)
            k1, _, _ = kernel_times_warm(L, ctx, 20, 0.2)
        sites = dom.nx * dom.ny
        coll[name] = {"mlups": round(sites * steps / (ms * 1e3), 1), "ms_per_step": round(ms / steps, 5),
                      "collide_ms": round(k1, 5), "n_positivity": st["n_positivity"], "steps": steps}
    coll["elbm"]["vs_lbgk"] = round(coll["elbm"]["mlups"] / coll["lbgk"]["mlups"], 3)
    res["collision_4096_entropic"] = coll

    print("[bench] variant cavity ensemble (256 domains)", file=sys.stderr, flush=True)
    res["cavity_ensemble_256"] = cavity_batch(torch, L, wl, stream, 200, one_by_one=True)
    return res


def batch_domains(L, wl, batch):
    doms = []
    for s in batch.specs:
        rho, u = wl.cavity_rest(s.n, s.n, rho0=1.0)
        doms.append(L.Domain(lattice=L.LBM_D2Q9, nx=s.n, ny=s.n, beta=s.beta, qe=L.LBM_QE_ENTROPIC,
                             limiter=L.LBM_LIM_MEDIAN, ds_form=L.LBM_DS_QUADRATIC, bc=L.LBM_BC_CAVITY,
                             delta_median=1e-3, rho0=1.0, lid_ux=0.1, rho_init=rho, u_init=u, probe=s.probe))
    return doms


def cavity_batch(torch, L, wl, stream, bsteps, one_by_one=False, kernel_steps=50, tile_x=0, tile_h=0):
    """The seeded ensemble of 256 lid-driven cavities (N in {64, 100, 128,
    192, 256}, Re in [2000, 7500], entropic f*, median filter delta = 1e-3),
    FP32, all domains in one launch per kernel per step, shapes chosen by the
    tuner; optionally against the same cavities run one context at a time."""
    batch = wl.cavity_batch(256)
    doms = batch_domains(L, wl, batch)
    with L.lbm_create(doms, L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, graph_chunk=50,
                                  probe_capacity=bsteps + 64, tile_x=tile_x, tile_h=tile_h)) as ctx:
        shape = L.lbm_tile_config(ctx)
        k1, k2, _ = kernel_times_warm(L, ctx, kernel_steps, 0.5)
        ms_batch = time_steps(torch, L, ctx, stream, bsteps, 20)
    sites = batch.sites
    alg = 72 * sites
    res = {
        "sites": sites, "steps": bsteps, "tile": list(shape),
        "batched_mlups": round(sites * bsteps / (ms_batch * 1e3), 1),
        "ms_per_step": round(ms_batch / bsteps, 5),
        "collide_ms": round(k1, 5), "second_pass_ms": round(k2, 5),
        "collide_hbm_frac": round(alg / (k1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_hbm_frac": round(alg * bsteps / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    if one_by_one:
        ms_single = 0.0
        for d in doms:
            with L.lbm_create([d], L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, graph_chunk=50,
                                         probe_capacity=bsteps + 64)) as ctx:
                ms_single += time_steps(torch, L, ctx, stream, bsteps, 20)
        res["one_by_one_mlups"] = round(sites * bsteps / (ms_single * 1e3), 1)
        res["speedup"] = round(ms_single / ms_batch, 2)
    return res


def summarize_pmc(fetch_csv, write_csv, record=True):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of every kernel, scaled by
    what the counters read for the calibration kernel (a plain elementwise
    multiply of COPY_BYTES in, COPY_BYTES out), printed as a table; with
    record, the dominant kernel's bytes are stored as the traffic record the
    roofline reports."""
    def per_kernel(path, counter):
        out = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return out

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")

    def pick(d, key, last=None):
        names = [k for k in d if key in k]
        if not names:
            raise SystemExit(f"no dispatch of a kernel matching {key!r}")
        vals = d[names[0]]
        return vals[-last:] if last else vals

    cal_f = pick(fetch, "MulFunctor", 3)
    cal_w = pick(write, "MulFunctor", 3)
    sf = COPY_BYTES / (sum(cal_f) / len(cal_f))
    sw = COPY_BYTES / (sum(cal_w) / len(cal_w))
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetch MB (scaled) | write MB (scaled) |")
    print("|---|---|---|---|---|---|")
    for name, vf in fetch.items():
        if "MulFunctor" in name:
            continue
        vw = write.get(name, [0.0])
        mf, mw = sum(vf) / len(vf), sum(vw) / len(vw)
        print(f"| {short_name(name)} | {len(vf)} | {mf / 1024:,.0f} | {mw / 1024:,.0f} | "
              f"{sf * mf / 1e6:,.1f} | {sw * mw / 1e6:,.1f} |")
    if not record:
        return
    k_f = pick(fetch, DOMINANT)
    k_w = pick(write, DOMINANT)
    fb = sf * sum(k_f) / len(k_f)
    wb = sw * sum(k_w) / len(k_w)
    rec = {"kernel": DOMINANT, "kernel_hash": kernel_hash(), "bytes_per_launch": round(fb + wb),
           "fetch_bytes": round(fb), "write_bytes": round(wb), "fetch_scale": round(sf, 4),
           "write_scale": round(sw, 4), "dispatches": [len(k_f), len(k_w)]}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def short_name(kernel):
    """A kernel's name without its return type and parameter list."""
    name = kernel.split("(")[0]
    return name[5:] if name.startswith("void ") else name


def np_arange_inclusive(a, b, c):
    k = int(round((b - a) / c))
    return [a + i * c for i in range(k + 1)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="host seconds for the oracle (half on one thread, half on the OpenMP build)")
    ap.add_argument("--kernel-steps", type=int, default=50, help="eager steps timed per kernel for the roofline")
    ap.add_argument("--kernel-warmup", type=float, default=0.5,
                    help="seconds of graph steps before the per-kernel timing (clocks settle)")
    ap.add_argument("--no-active", action="store_true", help="skip the active-median companion run")
    ap.add_argument("--variants", action="store_true", help="also time FP16/BF16 8192^2 and the cavity ensemble")
    ap.add_argument("--tile-h", type=int, default=0, help="rows per second-pass tile (16, 32, 64; 0: tuned)")
    ap.add_argument("--tile-x", type=int, default=0,
                    help="collision row blocks: 64 narrow, 256 full rows, 248 the fused step, 0 tuned")
    ap.add_argument("--adaptive", action="store_true",
                    help="LBM_RUN_ADAPTIVE: two kernels or the fused step, chosen every 64 steps")
    ap.add_argument("--delta-median", type=float, default=None,
                    help="median tolerance instead of 1e-4 (below the Delta S' of most nodes the filter acts)")
    ap.add_argument("--workload", choices=("headline", "elbm", "smooth", "batch") + tuple(SHEAR_STORAGE),
                    default="headline",
                    help="elbm: entropic f*, ELBM collisions, no limiter; smooth: the headline limiters plus "
                         "the smooth ensemble factor (k = 1/2, delta = 0.01); batch: only the ensemble of 256 "
                         "cavities (its own JSON line); shear-f32/-f16/-bf16: only the 8192^2 double shear "
                         "layer in that storage (its own JSON line)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain elementwise kernel over 1 GiB (known bytes) to scale HBM counters")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--no-record", action="store_true",
                    help="with --summarize-pmc: print the table only (a workload other than the headline)")
    ap.add_argument("--hopf", action="store_true",
                    help="instead of the step benchmark: the first-Hopf-bifurcation experiment (diffusive walls)")
    ap.add_argument("--hopf-re", default="6000:9000:250", help="Reynolds numbers, start:stop:step (inclusive)")
    ap.add_argument("--hopf-units", type=float, default=5000.0, help="non-dimensional time units per run")
    ap.add_argument("--hopf-n", type=int, default=100)
    ap.add_argument("--hopf-continuation", action="store_true",
                    help="instead of the benchmark: the hysteresis test of the Hopf onset (continuation down from "
                         "an oscillating state, up from a steady one)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, record=not args.no_record)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no multi-GPU path",
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
    if args.hopf_continuation:
        from paper_0704_0043_amd import hopf
        res = hopf.continuation(L, n=args.hopf_n, stream=stream.cuda_stream)
        print(json.dumps({"hopf_continuation": res}), flush=True)
        return
    if args.hopf:
        from paper_0704_0043_amd import hopf
        a, b, c = (float(v) for v in args.hopf_re.split(":"))
        res = hopf.run(L, list(np_arange_inclusive(a, b, c)), n=args.hopf_n, time_units=args.hopf_units,
                       stream=stream.cuda_stream)
        print(json.dumps({"hopf": res}), flush=True)
        return
    if args.workload in SHEAR_STORAGE:
        name = SHEAR_STORAGE[args.workload]
        storage = {"f32": L.LBM_F32, "f16": L.LBM_F16_SHIFT, "bf16": L.LBM_BF16_SHIFT}[name]
        res = {"shear_8192": {name: shear_run(torch, L, wl, stream, storage, args.steps, args.warmup)}}
        if args.calibrate_copy:
            res["copy_calibration"] = copy_calibration(torch, stream)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "batch":
        res = cavity_batch(torch, L, wl, stream, args.steps, kernel_steps=args.kernel_steps, tile_x=args.tile_x,
                           tile_h=args.tile_h)
        if args.calibrate_copy:
            res["copy_calibration"] = copy_calibration(torch, stream)
        print(json.dumps({"cavity_ensemble_256": res}), flush=True)
        return
    n = args.n
    dom = c2_domain(L, wl, n)
    dmed = 1e-4 if args.delta_median is None else args.delta_median
    dom.delta_median = dmed
    if args.workload == "elbm":
        dom.qe, dom.limiter, dom.collision = L.LBM_QE_ENTROPIC, L.LBM_LIM_NONE, L.LBM_COLL_ELBM
    elif args.workload == "smooth":
        dom.limiter |= L.LBM_LIM_ENS_SMOOTH
        dom.ens_k, dom.delta_ens = 0.5, 0.01
    default = args.workload == "headline" and dmed == 1e-4 and not args.adaptive and args.tile_x in (0, 256)
    print(f"[bench] creating {n}x{n} FP32 context", file=sys.stderr, flush=True)
    run = L.Run(storage=L.LBM_F32, stream=stream.cuda_stream, graph_chunk=64)
    if args.tile_h:
        run.tile_h = args.tile_h
    if args.tile_x:
        run.tile_x = args.tile_x
    if args.adaptive:
        run.flags |= L.LBM_RUN_ADAPTIVE
    ctx = L.lbm_create([dom], run)
    tile = L.lbm_tile_config(ctx)
    # the per-kernel timing first: its warm-up brings the clocks to their
    # sustained level, so the timed steps below run on a settled GPU
    print(f"[bench] per-kernel timing over {args.kernel_steps} eager steps after {args.kernel_warmup} s of "
          "graph steps", file=sys.stderr, flush=True)
    k1_ms, k2_ms, ktiming = kernel_times_warm(L, ctx, args.kernel_steps, args.kernel_warmup)
    ktiming["before_timed_region"] = True
    print(f"[bench] tile {tile}; warmup {args.warmup}, timing {args.steps} steps", file=sys.stderr, flush=True)
    ms = time_steps(torch, L, ctx, stream, args.steps, args.warmup)
    stats = L.lbm_entropy_stats(ctx)
    sites = n * n
    ms_step = ms / args.steps
    mlups = sites * args.steps / (ms * 1e3)
    alg_bytes = BYTES_PER_SITE[L.LBM_F32] * sites          # per step = per collision launch
    achieved = alg_bytes / (k1_ms * 1e-3) / 1e9
    step_achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    # the recorded traffic belongs to the default tolerance (no wave stores Delta S')
    traffic = load_traffic() if default else None
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
            "workload": workload_text(n, args.workload, dmed),
            "nx": n, "ny": n, "storage": "f32_shift", "tile": list(tile),
            "graphs": "every step inside captured HIP graphs (64-step chunks and powers of two below)",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "kernels": {"dominant": DOMINANT, "collide_ms": round(k1_ms, 5), "median_ms": round(k2_ms, 5),
                    "algorithmic_bytes_per_launch": alg_bytes, "timing": ktiming},
        "step_roofline": {"achieved": round(step_achieved, 1), "frac": round(step_achieved / HBM_PEAK_GBS, 4),
                          "unit": "GB/s"},
        "stats": {"mass": stats["mass"], "n_trimmed": stats["n_trimmed"], "n_filtered": stats["n_filtered"],
                  "max_dS": stats["max_dS"], "n_nonfinite": stats["n_nonfinite"]},
    }
    ctx.close()
    if not default:
        # the roofline object is defined for the headline's collision kernel;
        # these workloads are reported by kernel time only
        if args.workload == "elbm":
            out["kernels"]["dominant"] = "k_collide2d<float, 1, 1, 0, true>"
        out["roofline"] = None
        out["note"] = "not the headline workload: kernel times only (no roofline, no traffic record)"
    if default and not args.no_active:
        print("[bench] the same step with the median filter acting (delta_median = 1e-9 and 0; two kernels "
              "and the fused step)", file=sys.stderr, flush=True)
        out["median_active"] = median_active(torch, L, wl, stream, n)
    if args.calibrate_copy:
        out["copy_calibration"] = copy_calibration(torch, stream)
    if args.variants:
        out["variants"] = variants(torch, L, wl, stream, args)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        base, orun = cpu_baseline(wl, args.cpu_seconds, dom)
        out["cpu_baseline"] = base
        print(f"[bench] GPU replica against the oracle ({orun[0]} steps)", file=sys.stderr, flush=True)
        out["error"] = replica_error(L, stream, dom, wl, orun)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
