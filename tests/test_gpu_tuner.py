"""The shapes the autotuner chooses between change the speed of a step and
nothing it decides: row blocks of 256 columns or several rows of a narrow
domain per workgroup, the tile height of the second pass, and the fused step.
Across the two-kernel shapes fields, masks and the stats that come from the
collision kernel (and E(Delta S'), which the ensemble limiters use) are
bit-identical, and the FP64 sums the second pass adds to agree to rounding;
the fused step takes the same decisions and forms a moved node's state once,
so its populations agree to rounding."""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl
from tests.gpu_util import lbm, require_gpu, say

pytestmark = pytest.mark.gpu

COLLISION_STATS = ("mass", "mom_x", "mom_y", "sum_dS_pre", "sum_dS_post", "max_dS", "mean_dS", "n_fluid",
                   "n_nonpositive", "n_nonfinite")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def cavities(L, limiter, **kw):
    doms = []
    for k, n in enumerate((40, 64, 100, 128, 130, 200, 37, 256)):
        f0 = wl.random_populations(9, n, n - 3 * (k % 3), seed=900 + k, amp=0.03, spike_frac=0.05,
                                   spike_amp=0.35)
        doms.append(L.Domain(lattice=2, nx=n, ny=n - 3 * (k % 3), beta=0.95, qe=1, ds_form=0, limiter=limiter,
                             bc=L.LBM_BC_CAVITY, delta_trim=1e-4, delta_median=1e-5, rho0=1.0, lid_ux=0.1,
                             f_init=f0, **kw))
    return doms


def run(L, doms, storage, steps, tile_x, tile_h, flags=0):
    run_desc = L.Run(storage=storage, tile_x=tile_x, tile_h=tile_h, flags=L.LBM_RUN_RECORD | flags)
    with L.lbm_create(doms, run_desc) as ctx:
        shape = L.lbm_tile_config(ctx)
        L.lbm_step(ctx, steps)
        out = [(L.lbm_get_populations(ctx, k), L.lbm_limiter_mask(ctx, k)[0], L.lbm_entropy_stats(ctx, k))
               for k in range(len(doms))]
    return shape, out


@pytest.mark.parametrize("limiter,kw", [(2, {}), (2 | 32, dict(ens_c=0.1)), (1 | 8, dict(ens_k=0.5, delta_ens=0.05))],
                         ids=["median", "median+budget", "trim+smooth"])
@pytest.mark.parametrize("storage", [0, 1], ids=["f64", "f32"])
def test_shapes_do_not_change_results(limiter, kw, storage):
    L = lbm()
    doms = cavities(L, limiter, **kw)
    ref_shape, ref = run(L, doms, storage, 12, 256, 64, L.LBM_RUN_NO_TUNE)
    assert ref_shape == (256, 1, 64)
    for tile_x, tile_h in ((64, 16), (64, 64), (256, 32), (0, 0)):
        shape, got = run(L, doms, storage, 12, tile_x, tile_h)
        say(f"[tuner] limiter={limiter} storage={storage} asked ({tile_x}, {tile_h}) -> shape {shape}")
        fused = shape[0] == 248
        for (fa, ma, sa), (fb, mb, sb) in zip(ref, got):
            assert np.array_equal(ma, mb)
            for k in ("n_trimmed", "n_filtered", "n_ensemble", "n_positivity", "n_fluid", "n_nonpositive"):
                assert sa[k] == sb[k], k
            if fused:
                # the fused step forms a moved node's state once: rounding-level differences
                scale = np.abs(fa).max()
                assert np.abs(fa - fb).max() <= (1e-13 if storage == 0 else 2e-6) * scale
                for k in ("mass", "sum_dS_post", "max_dS"):
                    assert sb[k] == pytest.approx(sa[k], rel=1e-12 if storage == 0 else 1e-6, abs=1e-300), k
                continue
            assert np.array_equal(fa, fb)
            for k in COLLISION_STATS:
                assert sa[k] == sb[k], k
            assert sb["limiter_production"] == pytest.approx(sa["limiter_production"], rel=1e-12, abs=1e-300)


def test_narrow_blocks_and_the_cached_choice():
    L = lbm()
    doms = cavities(L, 2)[:1]                  # a 40 x 40 cavity: 64-column blocks, 4 rows each
    with L.lbm_create(doms, L.Run(storage=1, tile_x=64, tile_h=16)) as ctx:
        assert L.lbm_tile_config(ctx) == (64, 4, 16)
    big = [L.Domain(lattice=2, nx=300, ny=50, limiter=2, bc=L.LBM_BC_CAVITY, lid_ux=0.1)]
    with L.lbm_create(big, L.Run(storage=1, tile_x=64)) as ctx:
        assert L.lbm_tile_config(ctx)[:2] == (256, 1)   # wider than 128 columns: 256-column blocks
    # the tuner times the candidates once per problem; the next context gets its choice
    a = cavities(L, 2)
    with L.lbm_create(a, L.Run(storage=1)) as ctx:
        first = L.lbm_tile_config(ctx)
    with L.lbm_create(a, L.Run(storage=1)) as ctx:
        assert L.lbm_tile_config(ctx) == first
    say(f"[tuner] batch of 8 cavities: chosen shape {first}")
