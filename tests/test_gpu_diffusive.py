"""The cavity with diffusive Maxwell walls (Sec. 4.4.2) on the device
against the FP64 oracle: populations, masks and stats after many steps,
random states (every wall rule branch with non-trivial values), a batch of
cavities with different lid speeds in one launch, and FP32 storage."""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl
from tests.gpu_util import Pair, assert_masks_equal, assert_stats_close, lbm, orc, require_gpu, say

pytestmark = pytest.mark.gpu

D2Q9, DIFF = 2, 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def fields_close(pr, rtol):
    scale = np.abs(pr.fo).max()
    err = np.abs(pr.f - pr.fo).max() / scale
    assert err <= rtol, f"population max rel err {err:.3e}"


@pytest.mark.parametrize("qe", [0, 1])
def test_diffusive_cavity_from_rest_fp64(qe):
    """100 x 100 cavity from rest at Re = 7000 (u0 = 0.1, rho = 1), median
    filter delta = 1e-3 (the Hopf study's setting), 400 steps."""
    L = lbm()
    o = orc()
    rho, u = wl.cavity_rest(100, rho0=1.0)
    d = L.Domain(lattice=D2Q9, nx=100, ny=100, beta=wl.beta_from_nu(0.1 * 100 / 7000), qe=qe, limiter=2, bc=DIFF,
                 rho0=1.0, lid_ux=0.1, delta_median=1e-3)
    f0 = o.init_equilibrium(o.make_params(lattice=2, nx=100, ny=100, qe=qe, bc=DIFF), rho, u)
    pr = Pair(d, f0, steps=400)
    assert_masks_equal(pr)
    fields_close(pr, 1e-11)
    assert_stats_close(pr, rtol=1e-10)


@pytest.mark.parametrize("limiter", [0, 3])
def test_diffusive_cavity_random_state_fp64(limiter):
    """A random positive state on a 70 x 45 cavity (walls receive and send
    non-trivial mass everywhere), 5 steps."""
    L = lbm()
    f0 = wl.random_populations(9, 70, 45, seed=81, amp=0.05, spike_frac=0.05, spike_amp=0.3)
    d = L.Domain(lattice=D2Q9, nx=70, ny=45, beta=0.95, qe=1, limiter=limiter, bc=DIFF, lid_ux=0.07,
                 delta_trim=1e-3, delta_median=1e-4)
    pr = Pair(d, f0, steps=5)
    assert_masks_equal(pr)
    fields_close(pr, 1e-12)
    assert_stats_close(pr, rtol=1e-11)


def test_batch_of_diffusive_cavities_fp64():
    """Three cavities of different sizes and lid speeds in one launch."""
    L = lbm()
    o = orc()
    specs = [(40, 0.1, 3000.0), (64, 0.05, 5000.0), (33, 0.08, 8000.0)]
    doms, refs = [], []
    for n, u0, re in specs:
        rho, u = wl.cavity_rest(n, rho0=1.0)
        d = L.Domain(lattice=D2Q9, nx=n, ny=n, beta=wl.beta_from_nu(u0 * n / re), qe=1, limiter=2, bc=DIFF,
                     lid_ux=u0, delta_median=1e-3, rho_init=rho, u_init=u)
        doms.append(d)
        p = o.make_params(lattice=2, nx=n, ny=n, beta=d.beta, qe=1, limiter=2, bc=DIFF, lid_ux=u0,
                          delta_median=1e-3)
        f = o.init_equilibrium(p, rho, u)
        st, mo, _ = o.step(p, f, 250, record=True)
        refs.append((f, mo, st))
    with L.lbm_create(doms, L.Run(storage=0, flags=L.LBM_RUN_RECORD)) as ctx:
        L.lbm_step(ctx, 250)
        for k, (f, mo, st) in enumerate(refs):
            fg = L.lbm_get_populations(ctx, k)
            mg, _ = L.lbm_limiter_mask(ctx, k)
            sg = L.lbm_entropy_stats(ctx, k)
            assert np.array_equal(mg, mo)
            assert np.abs(fg - f).max() <= 1e-11 * np.abs(f).max()
            assert sg["mass"] == pytest.approx(st.mass, rel=1e-12)
            assert sg["n_filtered"] == st.n_filtered


def test_diffusive_cavity_fp32_short_horizon():
    """FP32 shifted storage, 64 x 64 at Re = 5000 with the median filter on
    the exact Delta S, 100 steps, against the FP64 oracle: rho / rho0 and
    u / u0 within 1e-5, and the filter's decisions of the last step equal
    except where the oracle's Delta S' lies within 1e-3 (relative) of its
    threshold max(median, delta) (FP32 Delta S' carries an error of order
    1e-4 relative, so such decisions may go either way)."""
    import median_pins as mp
    L = lbm()
    o = orc()
    n, steps = 64, 100
    rho, u = wl.cavity_rest(n, rho0=1.0)
    d = L.Domain(lattice=D2Q9, nx=n, ny=n, beta=wl.beta_from_nu(0.1 * n / 5000), qe=1, limiter=2, bc=DIFF,
                 lid_ux=0.1, delta_median=1e-3, rho_init=rho, u_init=u)
    with L.lbm_create([d], L.Run(storage=1, flags=L.LBM_RUN_RECORD)) as ctx:
        L.lbm_step(ctx, steps)
        rg, ug = L.lbm_moments(ctx)
        mg, _ = L.lbm_limiter_mask(ctx)
    p = o.make_params(lattice=2, nx=n, ny=n, beta=d.beta, qe=1, limiter=2, bc=DIFF, lid_ux=0.1, delta_median=1e-3)
    f = o.init_equilibrium(p, rho, u)
    _, mo, dso = o.step(p, f, steps, record=True)
    ro, ux, uy = o.moments(2, f)
    eu = max(np.abs(ug[0] - ux).max(), np.abs(ug[1] - uy).max()) / 0.1
    er = np.abs(rg - ro).max()
    med = mp.median_cavity(np.where((mo & 8) != 0, 0.0, dso))
    thr = np.maximum(med, 1e-3)
    close = np.abs(dso - thr) <= 1e-3 * thr
    diff = (mg & 2) != (mo & 2)
    say(f"[diffusive fp32 x{steps}] |u - u_ref|/u0 {eu:.2e}  |rho - rho_ref| {er:.2e}  filter decisions "
        f"differing {int(diff.sum())} (all within the margin: {not (diff & ~close).any()})")
    assert er <= 1e-5 and eu <= 1e-5
    assert not (diff & ~close).any()


def test_diffusive_cavity_fp32_drift_report():
    """The same flow over 1000 steps: the FP32 - FP64 difference is reported
    (filter decisions taken on either side of a threshold compound over the
    run; this is a report, and the assertion only guards against a run that
    leaves the FP64 solution altogether)."""
    L = lbm()
    o = orc()
    n = 64
    rho, u = wl.cavity_rest(n, rho0=1.0)
    d = L.Domain(lattice=D2Q9, nx=n, ny=n, beta=wl.beta_from_nu(0.1 * n / 5000), qe=1, limiter=2, bc=DIFF,
                 lid_ux=0.1, delta_median=1e-3, rho_init=rho, u_init=u)
    with L.lbm_create([d], L.Run(storage=1)) as ctx:
        L.lbm_step(ctx, 1000)
        rg, ug = L.lbm_moments(ctx)
    p = o.make_params(lattice=2, nx=n, ny=n, beta=d.beta, qe=1, limiter=2, bc=DIFF, lid_ux=0.1, delta_median=1e-3)
    f = o.init_equilibrium(p, rho, u)
    o.step(p, f, 1000)
    ro, ux, uy = o.moments(2, f)
    eu = max(np.abs(ug[0] - ux).max(), np.abs(ug[1] - uy).max()) / 0.1
    er = np.abs(rg - ro).max()
    say(f"[diffusive fp32 x1000 drift] |u - u_ref|/u0 {eu:.2e}  |rho - rho_ref| {er:.2e}")
    assert eu < 1e-2 and er < 1e-3
