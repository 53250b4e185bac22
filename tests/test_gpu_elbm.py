"""ELBM collisions (eqs. (elbm), (elbmLB)) and the positivity rule (Sec. 2.1)
on the device against the FP64 oracle: the device solves for alpha by a
safeguarded Newton iteration, the oracle by bisection to 1e-15, so states
agree to rounding; masks and counts (including the nodes where no root
exists and the positivity rule takes over) agree exactly."""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl
from tests.gpu_util import Pair, assert_masks_equal, assert_stats_close, lbm, orc, require_gpu, say

pytestmark = pytest.mark.gpu

D1Q3, D2Q9 = 1, 2
ELBM = 1
POS = 64


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def fields_close(pr, rtol):
    scale = np.abs(pr.fo).max()
    err = np.abs(pr.f - pr.fo).max() / scale
    say(f"[elbm] population max rel err {err:.2e}")
    assert err <= rtol


def test_shock_tube_elbm_fp64():
    """The ELBM shock tube of Sec. 4.3.1 (800 sites, nu = 1e-9, entropic f*),
    400 steps."""
    L = lbm()
    o = orc()
    rho, u = wl.shock_tube(800, 400)
    d = L.Domain(lattice=D1Q3, nx=800, ny=1, beta=wl.beta_from_nu(1e-9), qe=1, ds_form=0, limiter=0, bc=2,
                 collision=ELBM)
    f0 = o.init_equilibrium(o.make_params(lattice=1, nx=800, beta=d.beta, qe=1, bc=2), rho, u)
    pr = Pair(d, f0, steps=400)
    say(f"[elbm tube] positivity rule at {pr.so['n_positivity']} sites in the last step")
    assert_masks_equal(pr)
    fields_close(pr, 1e-11)
    assert_stats_close(pr, rtol=1e-9)


@pytest.mark.parametrize("limiter", [0, 3, 2 | POS])
@pytest.mark.parametrize("steps", [1, 4])
def test_d2q9_random_states_elbm_fp64(limiter, steps):
    L = lbm()
    f0 = wl.random_populations(9, 300, 70, seed=91, amp=0.05, spike_frac=0.05, spike_amp=0.35)
    d = L.Domain(lattice=D2Q9, nx=300, ny=70, beta=0.97, qe=1, ds_form=0, limiter=limiter, collision=ELBM,
                 delta_trim=1e-3, delta_median=1e-5)
    pr = Pair(d, f0, steps=steps)
    assert_masks_equal(pr)
    fields_close(pr, 1e-12)
    assert_stats_close(pr, rtol=1e-11)


def test_elbm_without_root_takes_the_positivity_rule_fp64():
    """Spikes of +700 % on a single population: no state of equal entropy on
    the non-negative part of the line, so the positivity rule acts."""
    L = lbm()
    f0 = wl.random_populations(9, 260, 40, seed=92, amp=0.02)
    rng = np.random.default_rng(5)
    pick = rng.random((40, 260)) < 0.03
    f0[5][pick] *= 8.0
    f0[6:9, pick] *= 0.05
    d = L.Domain(lattice=D2Q9, nx=260, ny=40, beta=0.9, qe=1, ds_form=0, collision=ELBM)
    pr = Pair(d, f0, steps=1)
    assert pr.so["n_positivity"] > 0
    assert_masks_equal(pr)
    fields_close(pr, 1e-12)
    assert_stats_close(pr, rtol=1e-11)


@pytest.mark.parametrize("lattice", [D1Q3, D2Q9])
def test_positivity_limiter_fp64(lattice):
    """LBGK at beta = 0.99 on large random deviations overshoots into negative
    populations; the positivity rule moves those nodes to the boundary."""
    L = lbm()
    q, ny = (9, 50) if lattice == D2Q9 else (3, 1)
    f0 = wl.random_populations(q, 400, ny, seed=93, amp=0.6)
    d = L.Domain(lattice=lattice, nx=400, ny=ny, beta=0.99, qe=0, ds_form=0, limiter=POS)
    pr = Pair(d, f0, steps=1)
    assert pr.so["n_positivity"] > 0
    assert_masks_equal(pr)
    fields_close(pr, 1e-12)
    assert_stats_close(pr, rtol=1e-11)
    assert pr.f.min() >= -1e-15


def test_elbm_fp32():
    L = lbm()
    f0 = wl.random_populations(9, 300, 70, seed=94, amp=0.05, spike_frac=0.05, spike_amp=0.35)
    d = L.Domain(lattice=D2Q9, nx=300, ny=70, beta=0.97, qe=1, ds_form=1, collision=ELBM)
    pr = Pair(d, f0, steps=1, storage=1)
    fields_close(pr, 2e-6)
    assert pr.stats["n_positivity"] == pr.so["n_positivity"]
