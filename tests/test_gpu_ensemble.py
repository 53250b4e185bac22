"""Ensemble-dependent limiters on the GPU (threshold c E, smooth eq. smooth1,
rational eq. phiExamp; Sec. 3.3, 3.4, 4.3.2) against the FP64 oracle.

E(Delta S') is a global FP64 sum on both sides, summed in different orders;
a node whose Delta S' lies within rounding of a threshold c E could take
the other decision, which these inputs (continuous random values) make
vanishingly unlikely; masks are compared exactly.
"""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl
from tests.gpu_util import DS_NOISE, Pair, assert_ds_close, assert_masks_equal, assert_stats_close, lbm, orc, require_gpu, say

pytestmark = pytest.mark.gpu

D1Q3, D2Q9 = 1, 2
THRESH, SMOOTH, RATIONAL, BUDGET = 4, 8, 16, 32


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def fields_close(pr, rtol=1e-12):
    scale = np.abs(pr.fo).max()
    err = np.abs(pr.f - pr.fo).max() / scale
    assert err <= rtol, f"population max rel err {err:.3e}"


CASES = [
    (THRESH, dict(ens_c=5.0)),
    (THRESH, dict(ens_c=2.0, delta_ens=1e-3)),
    (SMOOTH, dict(ens_k=0.5, delta_ens=0.1)),
    (SMOOTH, dict(ens_k=1.0, delta_ens=0.05)),
    (RATIONAL, dict(ens_c=2.0, ens_k=1.0)),
    (THRESH | 3, dict(ens_c=3.0)),
    (SMOOTH | RATIONAL | THRESH | 1, dict(ens_c=4.0, ens_k=1.0, delta_ens=0.02)),
    (BUDGET, dict(ens_c=0.3)),
    (BUDGET, dict(ens_c=0.05, delta_ens=1e-4)),
    (BUDGET | 2, dict(ens_c=0.9)),
]


@pytest.mark.parametrize("ds", [0, 1])
@pytest.mark.parametrize("limiter,kw", CASES)
def test_d2q9_periodic_single_step_fp64(limiter, kw, ds):
    L = lbm()
    f0 = wl.random_populations(9, 300, 70, seed=21, amp=0.03, spike_frac=0.05, spike_amp=0.35)
    dom = L.Domain(lattice=D2Q9, nx=300, ny=70, beta=0.97, qe=0, ds_form=ds, limiter=limiter,
                   delta_trim=1e-3, delta_median=1e-5, **kw)
    pr = Pair(dom, f0, steps=1, storage=0)
    assert pr.so["n_ensemble"] > 0
    assert_masks_equal(pr)
    assert_ds_close(pr, 1e-12)
    fields_close(pr)
    assert_stats_close(pr)


@pytest.mark.parametrize("ds", [0, 1])
@pytest.mark.parametrize("tile", [1, 3, 5, 16])
@pytest.mark.parametrize("limiter,kw", [(SMOOTH | RATIONAL | THRESH | 3, dict(ens_c=4.0, ens_k=1.0, delta_ens=0.02)),
                                        (BUDGET | 2, dict(ens_c=0.9))])
def test_tile_heights_fp64(limiter, kw, tile, ds):
    """The second pass walks each tile's rows in short chunks and rescales a
    chunk's moved nodes after its decisions: tiles shorter than a chunk, and
    tiles that end inside one, give the oracle's result."""
    L = lbm()
    f0 = wl.random_populations(9, 300, 70, seed=23, amp=0.03, spike_frac=0.05, spike_amp=0.35)
    dom = L.Domain(lattice=D2Q9, nx=300, ny=70, beta=0.97, qe=0, ds_form=ds, limiter=limiter,
                   delta_trim=1e-3, delta_median=1e-5, **kw)
    pr = Pair(dom, f0, steps=1, storage=0, tile=tile)
    assert pr.so["n_ensemble"] > 0 and pr.so["n_filtered"] > 0
    assert_masks_equal(pr)
    assert_ds_close(pr, 1e-12)
    fields_close(pr)
    assert_stats_close(pr)


@pytest.mark.parametrize("limiter,kw", [(THRESH, dict(ens_c=5.0)), (SMOOTH, dict(ens_k=0.5, delta_ens=0.01)),
                                        (BUDGET, dict(ens_c=0.5))])
def test_cavity_multistep_fp64(limiter, kw):
    """64 x 64 cavity from rest (Re = 3000 scaled), an ensemble limiter
    combined with the median filter, 60 steps."""
    L = lbm()
    o = orc()
    rho, u = wl.cavity_rest(64, rho0=1.0)
    d = L.Domain(lattice=D2Q9, nx=64, ny=64, beta=wl.beta_from_nu(0.1 * 64 / 3000), qe=1, limiter=limiter | 2,
                 bc=1, rho0=1.0, lid_ux=0.1, delta_median=1e-4, **kw)
    f0 = o.init_equilibrium(o.make_params(lattice=2, nx=64, ny=64, qe=1, bc=1), rho, u)
    pr = Pair(d, f0, steps=60)
    assert pr.so["n_ensemble"] > 0
    assert_masks_equal(pr, ens_noise=True)
    fields_close(pr, rtol=1e-11)
    assert_stats_close(pr, rtol=1e-10, skip=("n_ensemble",))
    assert abs(pr.stats["n_ensemble"] - pr.so["n_ensemble"]) <= (pr.dso <= DS_NOISE).sum()


@pytest.mark.parametrize("limiter,kw", [(THRESH, dict(ens_c=5.0)), (THRESH, dict(ens_c=20.0)),
                                        (SMOOTH, dict(ens_k=0.5, delta_ens=0.01)),
                                        (RATIONAL, dict(ens_c=3.0, ens_k=1.0)), (BUDGET, dict(ens_c=0.5))])
def test_shock_tube_fp64(limiter, kw):
    """The shock-tube runs of Sec. 4.3.2 (800 sites, nu = 1e-9, entropic
    f*, tube ends), 100 steps from the 1:2 density step."""
    L = lbm()
    o = orc()
    rho, u = wl.shock_tube(800, 400)
    d = L.Domain(lattice=D1Q3, nx=800, ny=1, beta=wl.beta_from_nu(1e-9), qe=1, ds_form=0, limiter=limiter, bc=2,
                 **kw)
    f0 = o.init_equilibrium(o.make_params(lattice=1, nx=800, beta=d.beta, qe=1, bc=2), rho, u)
    pr = Pair(d, f0, steps=100)
    say(f"[shock tube] n_ensemble {pr.so['n_ensemble']} threshold {pr.so['ens_threshold']:.3e}")
    assert pr.so["n_ensemble"] > 0
    assert_masks_equal(pr, ens_noise=True)
    fields_close(pr, rtol=1e-11)
    assert_stats_close(pr, rtol=1e-9, skip=("n_ensemble",))
    assert abs(pr.stats["n_ensemble"] - pr.so["n_ensemble"]) <= (pr.dso <= DS_NOISE).sum()


def test_batched_domains_use_their_own_mean():
    """Two domains with different amplitudes in one launch: E (hence the
    threshold) is per domain."""
    L = lbm()
    o = orc()
    doms, f0s = [], []
    for k, amp in enumerate((0.01, 0.05)):
        f0 = wl.random_populations(9, 130, 40, seed=40 + k, amp=amp, spike_frac=0.05, spike_amp=0.3)
        f0s.append(f0)
        doms.append(L.Domain(lattice=D2Q9, nx=130, ny=40, beta=0.95, qe=0, ds_form=1, limiter=THRESH, ens_c=4.0,
                             f_init=f0))
    with L.lbm_create(doms, L.Run(storage=0, flags=L.LBM_RUN_RECORD)) as ctx:
        L.lbm_step(ctx, 1)
        res = [(L.lbm_get_populations(ctx, k), L.lbm_limiter_mask(ctx, k)[0], L.lbm_entropy_stats(ctx, k))
               for k in range(2)]
    thr = []
    for k, d in enumerate(doms):
        p = o.make_params(lattice=2, nx=130, ny=40, beta=0.95, qe=0, ds_form=1, limiter=THRESH, ens_c=4.0)
        f = f0s[k].copy()
        st, mo, _ = o.step(p, f, 1, record=True)
        fg, mg, sg = res[k]
        assert np.array_equal(mg, mo)
        assert np.abs(fg - f).max() <= 1e-12 * np.abs(f).max()
        assert sg["ens_threshold"] == pytest.approx(st.ens_threshold, rel=1e-12)
        thr.append(st.ens_threshold)
    assert thr[1] > 1.2 * thr[0]      # the two means differ, each domain used its own


@pytest.mark.parametrize("storage", [1, 2])
def test_reduced_precision_smooth_limiter(storage):
    """FP32 / FP16 shift storage with the smooth limiter: Delta S' and the
    moved-node count against the FP64 oracle after one step (every node with
    Delta S' > 0 moves, so counts agree exactly)."""
    L = lbm()
    f0 = wl.random_populations(9, 300, 70, seed=23, amp=0.03, spike_frac=0.05, spike_amp=0.35)
    dom = L.Domain(lattice=D2Q9, nx=300, ny=70, beta=0.97, qe=0, ds_form=1, limiter=SMOOTH, ens_k=0.5,
                   delta_ens=0.1)
    pr = Pair(dom, f0, steps=1, storage=storage)
    assert pr.stats["n_ensemble"] == pr.so["n_ensemble"]
    assert pr.stats["mean_dS"] == pytest.approx(pr.so["mean_dS"], rel=1e-4 if storage == 1 else 2e-2)
    scale = np.abs(pr.fo).max()
    tol = 1e-6 if storage == 1 else 3e-3
    assert np.abs(pr.f - pr.fo).max() <= tol * scale


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("frac", [0.0, 0.02, 0.4, 1.0, 50.0])
def test_budget_threshold(storage, frac):
    """eq. (EntThresh) on the device: the threshold against the oracle's exact
    solution on the empirical distribution, from no budget (the threshold at
    the largest value) to a budget beyond sum Delta S' (every node to f*).
    FP32 storage takes the decision on FP32 Delta S' values, so there only
    the threshold's defining equation is checked, on the device's values."""
    L = lbm()
    f0 = wl.random_populations(9, 520, 90, seed=31, amp=0.03, spike_frac=0.05, spike_amp=0.35)
    dom = L.Domain(lattice=D2Q9, nx=520, ny=90, beta=0.9, qe=0, ds_form=1, limiter=BUDGET, ens_c=frac)
    pr = Pair(dom, f0, steps=1, storage=storage)
    t = pr.stats["ens_threshold"]
    say(f"[budget] frac {frac} threshold gpu {t!r} oracle {pr.so['ens_threshold']!r} moved {pr.stats['n_ensemble']}")
    if storage == 0:
        assert t == pytest.approx(pr.so["ens_threshold"], rel=1e-12, abs=1e-300)
        assert_masks_equal(pr)
        fields_close(pr)
        assert_stats_close(pr)
    else:
        d = pr.ds.astype(np.float32).astype(np.float64).ravel()
        c = 2 * 0.9 - 1
        budget = frac * (1 - c * c) * pr.stats["sum_dS_post"]
        if frac == 0.0:
            assert t == pytest.approx(d.max(), rel=1e-7)
        elif budget >= d.sum():
            assert t == 0.0
        else:
            assert np.maximum(d - t, 0).sum() == pytest.approx(budget, rel=1e-6)
        # the device compares Delta S' with the threshold rounded to FP32
        assert pr.stats["n_ensemble"] == int((d > float(np.float32(t))).sum())
