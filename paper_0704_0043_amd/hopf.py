"""First Hopf bifurcation of the lid-driven cavity (Sec. 4.4.2).

A batch of N x N cavities with diffusive Maxwell walls, entropic f*, density
1, lid speed u0 and the median filter (delta = 1e-3), one per Reynolds
number, runs in one context for T non-dimensional time units (T L / u0 steps)
while the velocity at the node nearest (L/16, 13L/16) is recorded every step.
From the last 1 % of each signal:

  * the energy of eq. (energy): E_u = || sqrt(L / (u0 |u_sig|)) (u_sig - mean) ||_2,
    i.e. E_u^2 = (L / u0) times the variance of u_sig (|u_sig| samples, one per
    step, so |u_sig| u0 / L is the signal's non-dimensional duration);
  * the critical Reynolds number: a Hopf bifurcation has E_u^2 growing
    linearly in Re past it, so Re_c is where the least-squares line through
    the oscillating runs crosses E_u^2 = 0;
  * the dominant frequency: the largest peak of the amplitude spectrum of
    u_sig - mean, in cycles per non-dimensional time unit;
  * the energy of an earlier window of the same length (ending at 90 % of the
    run), which shows whether the signal has settled.

L is N (the length in Re = u0 N / nu); the signal is in lattice units.
"""
from __future__ import annotations

import math
import sys
import time

import numpy as np

from . import workloads as wl


def probe_node(n: int) -> tuple:
    """node nearest (L/16, 13L/16) with node i at i / (N - 1)"""
    return int(round((n - 1) / 16)), int(round(13 * (n - 1) / 16))


def energy(u_sig, length: float, u0: float) -> float:
    """eq. (energy)"""
    u = np.asarray(u_sig, dtype=np.float64)
    return math.sqrt(length / (u0 * len(u))) * float(np.linalg.norm(u - u.mean()))


def critical_reynolds(re, e2, frac: float = 0.05):
    """Re where the least-squares line through the oscillating runs (E_u^2
    above `frac` of the largest) meets E_u^2 = 0; returns (Re_c, slope,
    the Re values used), or (nan, nan, []) with fewer than two such runs."""
    re = np.asarray(re, dtype=np.float64)
    e2 = np.asarray(e2, dtype=np.float64)
    osc = e2 > frac * e2.max() if e2.size and e2.max() > 0 else np.zeros(e2.shape, dtype=bool)
    if osc.sum() < 2:
        return math.nan, math.nan, []
    slope, icpt = np.polyfit(re[osc], e2[osc], 1)
    return float(-icpt / slope), float(slope), [float(r) for r in re[osc]]


def onset(re, e2, frac: float = 0.05):
    """(largest Re of a steady run below the smallest Re of an oscillating
    one, that smallest Re): the bracket of the transition when the
    oscillation appears with a finite amplitude (E_u^2 above `frac` of the
    largest counts as oscillating)"""
    re = np.asarray(re, dtype=np.float64)
    e2 = np.asarray(e2, dtype=np.float64)
    if not e2.size or e2.max() <= 0:
        return math.nan, math.nan
    osc = e2 > frac * e2.max()
    if not osc.any():
        return math.nan, math.nan
    first = float(re[osc].min())
    below = re[(~osc) & (re < first)]
    return (float(below.max()) if below.size else math.nan), first


def dominant_frequency(u_sig, length: float, u0: float) -> float:
    """cycles per non-dimensional time unit of the largest spectral peak
    (Hann window, mean removed, rest frequency excluded)"""
    u = np.asarray(u_sig, dtype=np.float64)
    u = (u - u.mean()) * np.hanning(len(u))
    amp = np.abs(np.fft.rfft(u))
    k = int(np.argmax(amp[1:])) + 1
    dt = u0 / length                  # non-dimensional time per step
    return k / (len(u) * dt)


def hopf_domains(L, re_values, n: int = 100, u0: float = 0.1, delta: float = 1e-3, qe=None):
    doms = []
    px, py = probe_node(n)
    for re in re_values:
        rho, u = wl.cavity_rest(n, n, rho0=1.0)
        doms.append(L.Domain(lattice=L.LBM_D2Q9, nx=n, ny=n, beta=wl.beta_from_nu(u0 * n / re),
                             qe=L.LBM_QE_ENTROPIC if qe is None else qe, limiter=L.LBM_LIM_MEDIAN,
                             ds_form=L.LBM_DS_EXACT, bc=L.LBM_BC_CAVITY_DIFFUSIVE, delta_median=delta,
                             rho0=1.0, lid_ux=u0, rho_init=rho, u_init=u, probe=(px, py)))
    return doms


def run(L, re_values, n: int = 100, u0: float = 0.1, time_units: float = 5000.0, tail: float = 0.01,
        storage: int = 0, stream=None, chunk: int = 200000, log=sys.stderr) -> dict:
    """Run the batch and analyse the probe signals; prints progress to `log`."""
    steps = int(round(time_units * n / u0))
    keep = max(2, int(round(tail * steps)))
    # the probes hold the last 10 tails, so the energy of an earlier window
    # (ending at 90 % of the run) shows whether the signal is still changing
    cap = min(steps, 10 * keep)
    doms = hopf_domains(L, re_values, n, u0)
    run_desc = L.Run(storage=storage, graph_chunk=100, probe_capacity=cap, tile_h=16,
                     stream=stream if stream is not None else 0)
    t0 = time.perf_counter()
    out = {"n": n, "u0": u0, "time_units": time_units, "steps": steps, "signal_steps": keep,
           "re": [float(r) for r in re_values], "probe": list(probe_node(n))}
    with L.lbm_create(doms, run_desc) as ctx:
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            L.lbm_step(ctx, k)
            L.lbm_synchronize(ctx)
            done += k
            print(f"[hopf] {done}/{steps} steps, {time.perf_counter() - t0:.1f} s", file=log, flush=True)
        wall = time.perf_counter() - t0
        full = [L.lbm_probe_trace(ctx, k, cap) for k in range(len(doms))]
        sig = [s[-keep:] for s in full]
        early = [s[:keep] for s in full] if cap >= 2 * keep else sig
        stats = [L.lbm_entropy_stats(ctx, k) for k in range(len(doms))]
    e = [energy(s[:, 0], n, u0) for s in sig]
    out["E_u_earlier"] = [energy(s[:, 0], n, u0) for s in early]
    out["earlier_window_end"] = 1.0 - (cap - keep) / steps
    e2 = [v * v for v in e]
    rec, slope, used = critical_reynolds(re_values, e2)
    out["onset"] = list(onset(re_values, e2))
    out.update({
        "E_u": e, "E_u2": e2, "Re_c": rec, "slope": slope, "fit_re": used,
        "frequency": [dominant_frequency(s[:, 0], n, u0) for s in sig],
        "u_mean": [float(s[:, 0].mean()) for s in sig], "v_mean": [float(s[:, 1].mean()) for s in sig],
        "n_filtered_last": [int(s["n_filtered"]) for s in stats],
        "wall_s": wall, "mlups": len(doms) * n * n * steps / wall / 1e6,
    })
    return out


def continuation(L, re_osc: float = 6400.0, re_steady: float = 6200.0, down=(6300.0, 6100.0, 5900.0, 5600.0),
                 up=(6300.0, 6500.0, 6700.0, 7000.0), n: int = 100, u0: float = 0.1, time_units: float = 3000.0,
                 tail: float = 0.01, stream=None, chunk: int = 250000, log=sys.stderr) -> dict:
    """Hysteresis test of the onset: run re_osc (oscillating from rest) and
    re_steady (steady from rest) for `time_units`, then continue from the
    oscillating state at each Re of `down` and from the steady state at each
    Re of `up` (the state carried over, only nu changed) for as long again;
    E_u^2 and the dominant frequency of the last `tail` of every run."""
    steps = int(round(time_units * n / u0))
    keep = max(2, int(round(tail * steps)))

    def go(doms):
        t0 = time.perf_counter()
        rd = L.Run(storage=0, graph_chunk=100, probe_capacity=keep, tile_h=16,
                   stream=stream if stream is not None else 0)
        with L.lbm_create(doms, rd) as ctx:
            done = 0
            while done < steps:
                k = min(chunk, steps - done)
                L.lbm_step(ctx, k)
                L.lbm_synchronize(ctx)
                done += k
                print(f"[hopf continuation] {done}/{steps} steps, {time.perf_counter() - t0:.1f} s", file=log,
                      flush=True)
            sig = [L.lbm_probe_trace(ctx, k, keep)[:, 0] for k in range(len(doms))]
            fs = [L.lbm_get_populations(ctx, k) for k in range(len(doms))]
        return sig, fs

    sig1, f1 = go(hopf_domains(L, [re_osc, re_steady], n, u0))
    doms = []
    for re, f in [(r, f1[0]) for r in down] + [(r, f1[1]) for r in up]:
        d = hopf_domains(L, [re], n, u0)[0]
        d.rho_init = d.u_init = None
        d.f_init = np.ascontiguousarray(f)
        doms.append(d)
    sig2, _ = go(doms)
    e2 = [energy(s, n, u0) ** 2 for s in sig2]
    fr = [dominant_frequency(s, n, u0) for s in sig2]
    nd = len(down)
    return {"n": n, "u0": u0, "time_units_each": time_units, "tail": tail,
            "from_rest": {"re": [re_osc, re_steady], "E_u2": [energy(s, n, u0) ** 2 for s in sig1]},
            "down_from_oscillating": {"re": list(down), "E_u2": e2[:nd], "frequency": fr[:nd]},
            "up_from_steady": {"re": list(up), "E_u2": e2[nd:], "frequency": fr[nd:]}}
