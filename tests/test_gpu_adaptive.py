"""Adaptive runs (LBM_RUN_ADAPTIVE): the context keeps the two-kernel step and
the fused step (Sec. 3.5 median filter in one pass) and chooses between them
at every multiple of graph_chunk steps, from the number of nodes the filter
moved at the previous such point: the fused step above 0.5 % of the fluid
nodes, the two kernels again below 0.1 %.

The forms take the same decisions and agree to rounding, so an adaptive run
is checked against the FP64 oracle like any multi-step run; the choice of
form depends only on the states at those points, so the same steps split
into different calls (with stats reads between them) give bit-identical
states, and so do graph replays and eager launches.
"""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl
from tests.gpu_util import lbm, oracle_params, orc, require_gpu, say

pytestmark = pytest.mark.gpu

D2Q9 = 2
FUSED = 248


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def dom(**kw):
    L = lbm()
    base = dict(lattice=D2Q9, nx=300, ny=70, beta=0.97, qe=0, ds_form=1, limiter=3, delta_trim=1e-4,
                delta_median=1e-12)
    base.update(kw)
    return L.Domain(**base)


def spiky(nx=300, ny=70, seed=7):
    return wl.random_populations(9, nx, ny, seed=seed, amp=0.05, spike_frac=0.05, spike_amp=0.4)


def create(d, f0, chunk=8, flags=0, storage=0):
    L = lbm()
    d.f_init = np.ascontiguousarray(f0)
    ctx = L.lbm_create([d], L.Run(storage=storage, graph_chunk=chunk, flags=L.LBM_RUN_ADAPTIVE | flags))
    d.f_init = None
    return ctx


def rest_state(nx, ny, rho=1.0):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return np.ascontiguousarray(np.broadcast_to((rho * w)[:, None, None], (9, ny, nx)))


def test_adaptive_takes_the_fused_step_while_the_filter_acts_and_leaves_it_after():
    L = lbm()
    d = dom()
    say("[case] adaptive form switching, 300x70 periodic, chunk 8")
    with create(d, spiky()) as ctx:
        assert L.lbm_tile_config(ctx)[0] != FUSED          # the two kernels first
        L.lbm_step(ctx, 16)                                  # points at 0 and 8: nothing read back yet
        assert L.lbm_tile_config(ctx)[0] != FUSED
        st = L.lbm_entropy_stats(ctx)
        assert st["n_filtered"] > 0.005 * st["n_fluid"]
        L.lbm_step(ctx, 1)                                   # point 16: the count of point 8 decides
        assert L.lbm_tile_config(ctx)[0] == FUSED
        L.lbm_step(ctx, 7)
        # at step 24 a state at rest: Delta S' = 0, the filter moves nothing
        L.lbm_set_populations(ctx, rest_state(d.nx, d.ny))
        # point 24 records step 23 (before the reset) and reads point 16;
        # point 32 records step 31 (nothing moved) and reads point 24
        L.lbm_step(ctx, 16)
        assert L.lbm_tile_config(ctx)[0] == FUSED
        assert L.lbm_entropy_stats(ctx)["n_filtered"] == 0
        L.lbm_step(ctx, 1)                                   # point 40 reads point 32
        assert L.lbm_tile_config(ctx)[0] != FUSED
        f = L.lbm_get_populations(ctx)
    # the rest state is a fixed point of either form
    assert np.abs(f - rest_state(d.nx, d.ny)).max() <= 1e-15


@pytest.mark.parametrize("qe,ds", [(0, 1), (1, 0)])
def test_adaptive_run_against_the_oracle(qe, ds):
    """24 steps, the form changing at step 8: the states agree with the oracle
    to FP64 rounding, the masks up to decisions within rounding of a threshold"""
    L = lbm()
    o = orc()
    d = dom(qe=qe, ds_form=ds, nx=250, ny=61)
    f0 = spiky(250, 61, seed=31 + qe)
    steps = 24
    say(f"[case] adaptive vs oracle 250x61 qe={qe} ds={ds} chunk 4, {steps} steps")
    with create(d, f0, chunk=4, flags=L.LBM_RUN_RECORD) as ctx:
        L.lbm_step(ctx, steps)
        assert L.lbm_tile_config(ctx)[0] == FUSED
        f = L.lbm_get_populations(ctx)
        st = L.lbm_entropy_stats(ctx, allow_unstable=True)
        mask, dsg = L.lbm_limiter_mask(ctx)
    fo = np.ascontiguousarray(f0, dtype=np.float64).copy()
    so, mo, dso = o.step(oracle_params(d), fo, steps, record=True)
    so = so.as_dict()
    err = np.abs(f - fo).max() / np.abs(fo).max()
    flips = int((mask != mo).sum())
    say(f"[adaptive] population rel err {err:.3e}, mask flips {flips}")
    assert err <= 1e-12
    assert flips <= max(2, mask.size // 1000)
    fin = np.isfinite(dso)
    assert np.array_equal(np.isfinite(dsg), fin)
    assert np.abs(dsg[fin] - dso[fin]).max() <= 1e-10 * np.abs(dso[fin]).max()
    assert st["mass"] == pytest.approx(so["mass"], rel=1e-12)
    assert st["n_fluid"] == so["n_fluid"]
    assert abs(st["n_filtered"] - so["n_filtered"]) <= max(2, mask.size // 1000)


def test_choices_do_not_depend_on_how_the_steps_are_called():
    L = lbm()
    d = dom(nx=200, ny=45)
    f0 = spiky(200, 45, seed=5)
    say("[case] adaptive call pattern, 200x45, chunk 8, 40 steps")
    with create(d, f0) as a:
        L.lbm_step(a, 40)
        fa = L.lbm_get_populations(a)
        ta = L.lbm_tile_config(a)
    with create(d, f0) as b:
        for n in (3, 5, 13, 1, 18):
            L.lbm_step(b, n)
            L.lbm_entropy_stats(b)
        fb = L.lbm_get_populations(b)
        tb = L.lbm_tile_config(b)
    with create(d, f0, flags=L.LBM_RUN_NO_GRAPH) as c:
        L.lbm_step(c, 40)
        fc = L.lbm_get_populations(c)
    assert ta == tb and ta[0] == FUSED
    assert np.array_equal(fa, fb)
    assert np.array_equal(fa, fc)


def test_adaptive_with_stats_checks_and_kernel_timing():
    """stats read every 5 steps inside lbm_step, and eager steps of
    lbm_kernel_times between calls: the same states as a plain adaptive run
    over the same steps (the checks only read; the timed steps are steps)"""
    L = lbm()
    d = dom(nx=200, ny=45)
    f0 = spiky(200, 45, seed=9)
    say("[case] adaptive with stats_every = 5 and lbm_kernel_times, 200x45, chunk 8")
    d.f_init = np.ascontiguousarray(f0)
    with L.lbm_create([d], L.Run(storage=0, graph_chunk=8, stats_every=5, flags=L.LBM_RUN_ADAPTIVE)) as a:
        L.lbm_step(a, 30)
        L.lbm_kernel_times(a, 4)
        L.lbm_step(a, 6)
        fa = L.lbm_get_populations(a)
        ta = L.lbm_tile_config(a)
    d.f_init = None
    with create(d, f0) as b:
        L.lbm_step(b, 30)
        L.lbm_kernel_times(b, 4)
        L.lbm_step(b, 6)
        fb = L.lbm_get_populations(b)
        tb = L.lbm_tile_config(b)
    assert ta == tb
    assert np.array_equal(fa, fb)


def test_adaptive_fp32_cavity_batch():
    """two cavities of different sizes in one FP32 batch (Sec. 4.4, entropic
    f*, median filter): the adaptive run stays with the plain run to the
    rounding of the moved nodes' FP32 stores"""
    L = lbm()
    doms = []
    for n, seed in ((64, 3), (100, 4)):
        rho, u = wl.cavity_rest(n, n, rho0=1.0)
        doms.append(L.Domain(lattice=D2Q9, nx=n, ny=n, beta=0.99, qe=1, limiter=2, ds_form=1, bc=1,
                             delta_median=1e-12, rho0=1.0, lid_ux=0.1, rho_init=rho, u_init=u))
    say("[case] adaptive FP32 cavity batch 64 + 100, chunk 16, 200 steps")
    with L.lbm_create(doms, L.Run(storage=1, graph_chunk=16, flags=L.LBM_RUN_ADAPTIVE)) as ctx:
        L.lbm_step(ctx, 200)
        shape = L.lbm_tile_config(ctx)
        out = [L.lbm_moments(ctx, k) for k in range(2)]
        sts = [L.lbm_entropy_stats(ctx, k) for k in range(2)]
    with L.lbm_create(doms, L.Run(storage=1)) as ref:
        L.lbm_step(ref, 200)
        outr = [L.lbm_moments(ref, k) for k in range(2)]
    for (rho, u), (rr, ur), st in zip(out, outr, sts):
        say(f"[adaptive] cavity batch shape {shape}, filtered {st['n_filtered']} of {st['n_fluid']}, "
            f"rho diff {np.abs(rho - rr).max():.2e}, u diff {np.abs(u - ur).max():.2e}")
        assert np.all(np.isfinite(rho)) and np.all(np.isfinite(u))
        # the forms differ by the rounding of moved nodes' FP32 stores
        assert np.abs(rho - rr).max() <= 1e-5
        assert np.abs(u - ur).max() <= 1e-5
