"""Helpers of the GPU parity tests: run the same seeded input through the HIP
library (via the C ABI binding) and through the FP64 oracle, and compare."""
from __future__ import annotations

import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def lbm():
    from paper_0704_0043_amd import lbm as L
    L.lib()                      # fails loudly when the library is not built
    return L


def orc():
    from oracle import oracle
    oracle.build()
    return oracle


def oracle_params(d, entropy=False):
    o = orc()
    return o.make_params(lattice=d.lattice, nx=d.nx, ny=d.ny, beta=d.beta, qe=d.qe, ds_form=d.ds_form,
                         limiter=d.limiter, trim_mode=d.trim_mode, median_mode=d.median_mode, bc=d.bc,
                         delta_trim=d.delta_trim, delta_median=d.delta_median, rho0=d.rho0, lid_ux=d.lid_ux,
                         entropy=entropy, ens_c=d.ens_c, ens_k=d.ens_k, delta_ens=d.delta_ens,
                         collision=d.collision, homothety=d.homothety, top_k=d.top_k)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Pair:
    """GPU and oracle results after `steps` steps from the same state."""

    def __init__(self, dom, f0, steps=1, storage=0, tile=None, flags=None, entropy=False, tile_x=0):
        L = lbm()
        o = orc()
        say(f"[case] lattice={dom.lattice} n={dom.nx}x{dom.ny} bc={dom.bc} qe={dom.qe} ds={dom.ds_form} "
            f"lim={dom.limiter} modes={dom.trim_mode}/{dom.median_mode} storage={storage} steps={steps} tile={tile} "
            f"tile_x={tile_x}")
        dom.f_init = np.ascontiguousarray(f0)
        fl = L.LBM_RUN_RECORD | (L.LBM_RUN_ENTROPY if entropy else 0) if flags is None else flags
        run = L.Run(storage=storage, flags=fl, tile_x=tile_x)
        if tile:
            run.tile_h = int(tile)     # rows per D2Q9 second-pass (or fused) tile
        with L.lbm_create([dom], run) as ctx:
            self.tile = L.lbm_tile_config(ctx)
            L.lbm_step(ctx, steps)
            self.f = L.lbm_get_populations(ctx)
            self.stats = L.lbm_entropy_stats(ctx, allow_unstable=True)
            if fl & L.LBM_RUN_RECORD:
                self.mask, self.ds = L.lbm_limiter_mask(ctx)
            self.rho, self.u = L.lbm_moments(ctx)
        p = oracle_params(dom, entropy)
        self.fo = np.ascontiguousarray(f0, dtype=np.float64).copy()
        st, self.mo, self.dso = o.step(p, self.fo, steps, record=True)
        self.so = st.as_dict()
        self.neq = neq_l1(dom, f0) if steps == 1 else None
        dom.f_init = None


def neq_l1(dom, f0):
    """sum_i |f'_i - f*_i| per node for one step from f0 (oracle equilibria):
    the scale of the rounding error of Delta S(f') in any FP64 evaluation."""
    o = orc()
    f0 = np.asarray(f0, dtype=np.float64)
    rho, ux, uy = o.moments(dom.lattice, f0)
    c = 2 * dom.beta - 1
    out = np.zeros(rho.shape)
    for (y, x), r in np.ndenumerate(rho):
        fs = o.equilibrium(dom.lattice, dom.qe, r, ux[y, x], uy[y, x])
        out[y, x] = abs(c) * np.abs(fs - f0[:, y, x]).sum()
    return out


def stats_equal(a, b):
    """dict equality with NaN == NaN (total_entropy is NaN when not computed)"""
    if a.keys() != b.keys():
        return False
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, float) and isinstance(y, float) and np.isnan(x) and np.isnan(y):
            continue
        if x != y:
            return False
    return True


# Delta S' of a node at equilibrium up to rounding is (eps f*)^2 / f* per
# population: any two FP64 evaluations may differ by that much
DS_NOISE = 1e-28


def assert_masks_equal(pr, ens_noise=False):
    """Masks equal node by node.  With ens_noise, the ensemble bit may differ
    at nodes whose Delta S' is rounding noise on either side (a limiter that
    moves every node with Delta S' > 0 sees 0 on one side and 1e-30 on the
    other; the move changes the node by far less than one ulp)."""
    diff = pr.mask != pr.mo
    if ens_noise:
        quiet = (np.maximum(np.abs(pr.ds), np.abs(pr.dso)) <= DS_NOISE) & ((pr.mask ^ pr.mo) == 16)
        diff &= ~quiet
    mism = np.nonzero(diff)
    if len(mism[0]):
        k = (mism[0][0], mism[1][0])
        raise AssertionError(f"{len(mism[0])} mask mismatches; first at {k}: gpu {pr.mask[k]} oracle {pr.mo[k]} "
                             f"dS gpu {pr.ds[k]!r} oracle {pr.dso[k]!r}")




def assert_ds_close(pr, rtol):
    """Delta S' within rtol, or within the rounding bound 32 eps sum|f' - f*|
    where the nonequilibrium part is so small that one ulp of f* matters, or
    within the rounding noise of a node at equilibrium."""
    a, b = pr.ds, pr.dso
    fin = np.isfinite(b)
    assert np.array_equal(np.isfinite(a), fin)
    assert np.array_equal(np.isinf(a), np.isinf(b))
    tol = rtol * np.abs(b[fin]) + DS_NOISE
    if pr.neq is not None:
        tol = tol + 32 * np.finfo(np.float64).eps * pr.neq[fin]
    err = np.abs(a[fin] - b[fin])
    bad = err > tol
    if bad.any():
        k = np.argmax(np.where(bad, err - tol, -np.inf))
        raise AssertionError(f"{bad.sum()} dS mismatches; worst: gpu {a[fin][k]!r} oracle {b[fin][k]!r} "
                             f"tol {tol[k]:.3e}")


def assert_stats_close(pr, rtol=1e-11, counts=True, skip=()):
    g, o = pr.stats, pr.so
    assert g["mass"] == pytest.approx(o["mass"], rel=rtol)
    m = abs(o["mass"])
    assert abs(g["mom_x"] - o["mom_x"]) <= rtol * m
    assert abs(g["mom_y"] - o["mom_y"]) <= rtol * m
    for k in ("sum_dS_pre", "sum_dS_post", "max_dS"):
        assert g[k] == pytest.approx(o[k], rel=rtol, abs=1e-300), k
    assert abs(g["limiter_production"] - o["limiter_production"]) <= rtol * max(o["sum_dS_post"], 1e-300) * 10
    if counts:
        for k in ("n_trimmed", "n_filtered", "n_nonpositive", "n_nonfinite", "n_fluid", "n_ensemble",
                  "n_positivity"):
            if k in skip:
                continue
            assert g[k] == o[k], (k, g[k], o[k])
    assert g["mean_dS"] == pytest.approx(o["mean_dS"], rel=rtol, abs=1e-300)
    assert g["ens_threshold"] == pytest.approx(o["ens_threshold"], rel=rtol, abs=1e-300)
