"""The fused D2Q9 step (collision, trimming, positivity and the median filter
of Sec. 3.5 in one pass; tile_x = 248) against the FP64 oracle and against the
two-kernel step on the same seeded states.

Both paths take every decision from the same Delta S' values, so the limiter
masks and the recorded Delta S' planes agree bit for bit and so do all
counts.  A moved node's populations are formed differently (the fused step
forms f* - phi c d once with phi the smallest factor, the two kernels rescale
the stored trimmed state), so populations agree with the oracle to the usual
FP64 parity bound and with the other path to rounding.  Sizes put ragged
edges at the wave (62 columns), workgroup (248 columns) and tile-height
boundaries; tiny domains are narrower than one wave and lower than one tile.
"""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl
from tests.gpu_util import Pair, assert_ds_close, assert_masks_equal, assert_stats_close, lbm, require_gpu, say

pytestmark = pytest.mark.gpu

D2Q9 = 2
FUSED = 248


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def dom(**kw):
    L = lbm()
    base = dict(lattice=D2Q9, nx=300, ny=70, beta=0.97, qe=0, ds_form=1, limiter=3, delta_trim=1e-4,
                delta_median=1e-5)
    base.update(kw)
    return L.Domain(**base)


def fields_close(a, b, rtol):
    scale = np.abs(b).max()
    err = np.abs(a - b).max() / scale
    assert err <= rtol, f"population max rel err {err:.3e}"


def run_gpu(d, f0, storage, steps, tile_x, tile_h, flags):
    L = lbm()
    d.f_init = np.ascontiguousarray(f0)
    run = L.Run(storage=storage, tile_x=tile_x, tile_h=tile_h, flags=flags | L.LBM_RUN_NO_TUNE)
    with L.lbm_create([d], run) as ctx:
        shape = L.lbm_tile_config(ctx)
        L.lbm_step(ctx, steps)
        out = dict(f=L.lbm_get_populations(ctx), st=L.lbm_entropy_stats(ctx, allow_unstable=True), shape=shape)
        if flags & L.LBM_RUN_RECORD:
            out["mask"], out["ds"] = L.lbm_limiter_mask(ctx)
    d.f_init = None
    return out


def compare_paths(d, f0, storage=0, steps=1, tile_h=32, rtol=1e-13):
    """fused and two-kernel runs of the same input.  One step: identical
    decisions, Delta S' and counts (both take them from the same collision),
    populations to rtol.  More steps: the rounding-level difference of the
    moved nodes feeds the next collisions, so Delta S' agrees to rounding and
    a decision may flip only where Delta S' lies within rounding of its
    threshold; populations to rtol."""
    L = lbm()
    say(f"[case] fused vs two-kernel {d.nx}x{d.ny} bc={d.bc} qe={d.qe} ds={d.ds_form} lim={d.limiter} "
        f"modes={d.trim_mode}/{d.median_mode} storage={storage} steps={steps} th={tile_h}")
    a = run_gpu(d, f0, storage, steps, FUSED, tile_h, L.LBM_RUN_RECORD)
    b = run_gpu(d, f0, storage, steps, 256, 64, L.LBM_RUN_RECORD)
    assert a["shape"] == (FUSED, 1, tile_h)
    if steps == 1:
        assert np.array_equal(a["mask"], b["mask"])
        assert np.array_equal(a["ds"], b["ds"], equal_nan=True)
        for k in ("n_trimmed", "n_filtered", "n_nonpositive", "n_nonfinite", "n_fluid", "n_positivity"):
            assert a["st"][k] == b["st"][k], k
    else:
        flips = int((a["mask"] != b["mask"]).sum())
        assert flips <= max(2, a["mask"].size // 1000), f"{flips} mask mismatches"
        fin = np.isfinite(b["ds"])
        assert np.array_equal(np.isfinite(a["ds"]), fin)
        scale = np.abs(b["ds"][fin]).max()
        # one rounding of the stored state moves Delta S' by about 2 u / |f - f*| relative
        unit = {0: 2.0 ** -53, 1: 2.0 ** -24, 2: 2.0 ** -11, 3: 2.0 ** -8}[storage]
        assert np.abs(a["ds"][fin] - b["ds"][fin]).max() <= max(1e-11, 64 * unit) * scale
    for k in ("mass", "sum_dS_pre", "sum_dS_post", "max_dS"):
        assert a["st"][k] == pytest.approx(b["st"][k], rel=1e-12 if storage == 0 else 1e-5, abs=1e-300), k
    fields_close(a["f"], b["f"], rtol)
    return a, b


@pytest.mark.parametrize("qe", [0, 1])
@pytest.mark.parametrize("ds", [0, 1])
@pytest.mark.parametrize("limiter", [2, 3])
def test_fused_periodic_fp64_against_oracle(qe, ds, limiter):
    f0 = wl.random_populations(9, 300, 70, seed=101 + qe + 2 * ds, amp=0.05, spike_frac=0.05, spike_amp=0.4)
    pr = Pair(dom(qe=qe, ds_form=ds, limiter=limiter), f0, tile=32, tile_x=FUSED)
    assert pr.tile == (FUSED, 1, 32)
    assert_masks_equal(pr)
    assert_ds_close(pr, 1e-12)
    fields_close(pr.f, pr.fo, 1e-13)
    assert_stats_close(pr)
    assert pr.so["n_filtered"] > 0


@pytest.mark.parametrize("trim_mode,median_mode", [(1, 0), (0, 1), (1, 1)])
def test_fused_limiter_modes_fp64(trim_mode, median_mode):
    f0 = wl.random_populations(9, 130, 90, seed=105, amp=0.05, spike_frac=0.05, spike_amp=0.4)
    pr = Pair(dom(nx=130, ny=90, qe=1, trim_mode=trim_mode, median_mode=median_mode, delta_trim=3e-4,
                  delta_median=2e-5), f0, tile=64, tile_x=FUSED)
    assert_masks_equal(pr)
    assert_ds_close(pr, 1e-12)
    fields_close(pr.f, pr.fo, 1e-13)
    assert_stats_close(pr)


def test_fused_exact_homothety_and_nonpositive_fp64():
    """exact Delta S with the homothety reached by a root solve, and sites with
    a negative population (Delta S = +inf, moved to f*)"""
    f0 = wl.random_populations(9, 96, 40, seed=107, amp=0.05, spike_frac=0.05, spike_amp=0.4, negative_frac=0.02)
    pr = Pair(dom(nx=96, ny=40, qe=1, ds_form=0, homothety=1), f0, tile=32, tile_x=FUSED)
    assert_masks_equal(pr)
    assert_ds_close(pr, 1e-12)
    fields_close(pr.f, pr.fo, 1e-13)
    assert_stats_close(pr)


def test_fused_positivity_with_median_fp64():
    """the positivity factor joins the trimming and median factors in the
    minimum (eq. LimGenF with all three); with the exact Delta S, which this
    combination requires"""
    L = lbm()
    f0 = wl.random_populations(9, 130, 50, seed=109, amp=0.05, spike_frac=0.08, spike_amp=0.9)
    pr = Pair(dom(nx=130, ny=50, beta=1.0, ds_form=0, limiter=3 | L.LBM_LIM_POSITIVITY), f0, steps=2, tile=32,
              tile_x=FUSED)
    assert_masks_equal(pr)
    fields_close(pr.f, pr.fo, 1e-13)
    assert_stats_close(pr)
    assert pr.so["n_positivity"] > 0 and pr.so["n_filtered"] > 0


@pytest.mark.parametrize("qe", [0, 1])
@pytest.mark.parametrize("diffusive", [0, 1])
def test_fused_cavity_fp64(qe, diffusive):
    """walls, lid (equilibrium or diffusive) and the near-wall stencils of Sec. 4.4"""
    L = lbm()
    f0 = wl.random_populations(9, 100, 100, seed=111 + qe, rho0=2.7, amp=0.05, spike_frac=0.05, spike_amp=0.4)
    bc = L.LBM_BC_CAVITY_DIFFUSIVE if diffusive else L.LBM_BC_CAVITY
    d = L.Domain(lattice=D2Q9, nx=100, ny=100, beta=0.97087, qe=qe, limiter=3, bc=bc, rho0=2.7, lid_ux=0.1,
                 delta_trim=1e-4, delta_median=1e-5)
    pr = Pair(d, f0, steps=3, tile=32, tile_x=FUSED)
    assert_masks_equal(pr)
    fields_close(pr.f, pr.fo, 1e-13)
    assert_stats_close(pr)


@pytest.mark.parametrize("nx,ny,th", [(40, 20, 32), (62, 33, 32), (63, 64, 64), (124, 31, 32), (125, 97, 96),
                                      (247, 128, 128), (248, 65, 64), (249, 70, 32), (520, 129, 64),
                                      (130, 9, 1), (250, 23, 3), (300, 42, 4)])
def test_fused_ragged_sizes_against_two_kernels(nx, ny, th):
    f0 = wl.random_populations(9, nx, ny, seed=nx + ny, amp=0.05, spike_frac=0.05, spike_amp=0.4)
    compare_paths(dom(nx=nx, ny=ny, qe=1), f0, steps=1, tile_h=th)
    compare_paths(dom(nx=nx, ny=ny, qe=1), f0, steps=4, tile_h=th, rtol=1e-12)


@pytest.mark.parametrize("storage,rtol", [(1, 2e-6), (2, 2e-3), (3, 2e-2)], ids=["f32", "f16", "bf16"])
def test_fused_reduced_storage_against_two_kernels(storage, rtol):
    """the fused step stores f* - phi c d once; the two kernels store the trimmed
    state and rescale it, each store rounded to the storage type"""
    f0 = wl.random_populations(9, 300, 70, seed=113, amp=0.05, spike_frac=0.05, spike_amp=0.4)
    compare_paths(dom(qe=1), f0, storage=storage, steps=1, tile_h=64, rtol=rtol)
    compare_paths(dom(qe=1), f0, storage=storage, steps=3, tile_h=64, rtol=rtol)


def test_fused_cavity_fp32_and_probe():
    """a 130 x 130 cavity from rest in FP32 for 200 steps: the two paths give
    the same masks and the same probe trace to rounding"""
    L = lbm()
    rho, u = wl.cavity_rest(130, 130, rho0=1.0)
    res = []
    for tile_x, th in ((FUSED, 64), (256, 64)):
        d = L.Domain(lattice=D2Q9, nx=130, ny=130, beta=wl.beta_from_nu(0.1 * 130 / 5000.0), qe=1, limiter=2,
                     ds_form=1, bc=L.LBM_BC_CAVITY, delta_median=1e-6, rho0=1.0, lid_ux=0.1, rho_init=rho,
                     u_init=u, probe=(8, 105))
        run = L.Run(storage=1, tile_x=tile_x, tile_h=th, flags=L.LBM_RUN_RECORD | L.LBM_RUN_NO_TUNE,
                    probe_capacity=256)
        with L.lbm_create([d], run) as ctx:
            L.lbm_step(ctx, 200)
            res.append((L.lbm_limiter_mask(ctx)[0], L.lbm_probe_trace(ctx), L.lbm_entropy_stats(ctx),
                        L.lbm_get_populations(ctx)))
    (ma, pa, sa, fa), (mb, pb, sb, fb) = res
    say(f"[fused cavity fp32 x200] filtered {sa['n_filtered']} / {sb['n_filtered']}, probe diff "
        f"{np.abs(pa - pb).max():.2e}, mask mismatches {int((ma != mb).sum())}")
    assert sa["n_filtered"] > 0
    assert np.abs(pa - pb).max() <= 1e-6 * 0.1     # FP32 rounding of the lid velocity scale
    fields_close(fa, fb, 1e-5)


def test_fused_batch_of_domains():
    """several domains of different sizes in one fused launch: each domain's
    populations and stats match its own single-domain two-kernel run"""
    L = lbm()
    sizes = [(300, 70), (40, 20), (249, 97), (62, 62)]
    doms, f0s = [], []
    for k, (nx, ny) in enumerate(sizes):
        f0s.append(wl.random_populations(9, nx, ny, seed=200 + k, amp=0.05, spike_frac=0.05, spike_amp=0.4))
        d = dom(nx=nx, ny=ny, qe=1)
        d.f_init = np.ascontiguousarray(f0s[-1])
        doms.append(d)
    run = L.Run(storage=0, tile_x=FUSED, tile_h=64, flags=L.LBM_RUN_RECORD | L.LBM_RUN_NO_TUNE)
    with L.lbm_create(doms, run) as ctx:
        L.lbm_step(ctx, 1)
        got = [(L.lbm_get_populations(ctx, k), L.lbm_limiter_mask(ctx, k)[0], L.lbm_entropy_stats(ctx, k))
               for k in range(len(doms))]
    for k, d in enumerate(doms):
        d.f_init = None
        ref = run_gpu(d, f0s[k], 0, 1, 256, 64, L.LBM_RUN_RECORD)
        assert np.array_equal(got[k][1], ref["mask"])
        fields_close(got[k][0], ref["f"], 1e-13)
        assert got[k][2]["n_filtered"] == ref["st"]["n_filtered"]
        assert got[k][2]["mass"] == pytest.approx(ref["st"]["mass"], rel=1e-13)


def test_fused_rejected_where_it_does_not_apply():
    L = lbm()
    f0 = wl.random_populations(9, 64, 16, seed=3, amp=0.05)
    for kw in (dict(limiter=1), dict(limiter=2 | L.LBM_LIM_ENS_SMOOTH, ens_k=0.5, delta_ens=0.01)):
        d = dom(nx=64, ny=16, **kw)
        d.f_init = f0
        with pytest.raises(L.LbmError):
            L.lbm_create([d], L.Run(storage=0, tile_x=FUSED))
