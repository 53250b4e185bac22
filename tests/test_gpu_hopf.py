"""The Hopf pipeline (Sec. 4.4.2) end to end on the device, shortened: a
batch of diffusive-wall cavities runs with its probes recording, and the
probe signal is the velocity the context reports at the probe node."""
import numpy as np
import pytest

from paper_0704_0043_amd import hopf
from tests.gpu_util import lbm, orc, require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_short_hopf_batch():
    L = lbm()
    n, u0 = 40, 0.1
    res = hopf.run(L, [2000.0, 4000.0, 9000.0], n=n, u0=u0, time_units=60.0, tail=0.05, chunk=8000)
    say(f"[hopf short] E_u {res['E_u']} freq {res['frequency']} {res['mlups']:.0f} MLUPS")
    assert res["steps"] == 24000 and res["signal_steps"] == 1200
    assert all(np.isfinite(res["E_u"])) and all(np.isfinite(res["u_mean"]))
    assert all(abs(u) < u0 for u in res["u_mean"])


def test_probe_signal_is_the_node_velocity():
    L = lbm()
    n = 40
    doms = hopf.hopf_domains(L, [3000.0], n=n)
    with L.lbm_create(doms, L.Run(storage=0, probe_capacity=64)) as ctx:
        L.lbm_step(ctx, 500)
        sig = L.lbm_probe_trace(ctx, 0, 64)
        _, u = L.lbm_moments(ctx)
    px, py = hopf.probe_node(n)
    # the last sample is the velocity of the pre-collision state of the last
    # step; lbm_moments reports the state after it, one step later
    assert len(sig) == 64
    assert abs(sig[-1, 0] - u[0, py, px]) < 2e-3 * 0.1


@pytest.mark.parametrize("re", [3000.0, 7375.0])
def test_probe_trace_against_the_oracle(re):
    """The Hopf setup (diffusive walls, entropic f*, exact Delta S, median
    filter delta = 1e-3, FP64) on a 40 x 40 cavity from rest: the probe trace
    of 600 steps, sample by sample, against the oracle's velocity at the
    probe node before each step."""
    L, o = lbm(), orc()
    n, u0, steps = 40, 0.1, 600
    d = hopf.hopf_domains(L, [re], n=n, u0=u0)[0]
    px, py = hopf.probe_node(n)
    with L.lbm_create([d], L.Run(storage=0, probe_capacity=steps)) as ctx:
        L.lbm_step(ctx, steps)
        sig = L.lbm_probe_trace(ctx, 0, steps)
        st = L.lbm_entropy_stats(ctx)
    p = o.make_params(lattice=2, nx=n, ny=n, beta=d.beta, qe=d.qe, ds_form=d.ds_form, limiter=d.limiter, bc=d.bc,
                      delta_median=d.delta_median, rho0=d.rho0, lid_ux=d.lid_ux)
    f = o.init_equilibrium(p, d.rho_init, d.u_init)
    ref = np.empty((steps, 2))
    filtered = 0
    for k in range(steps):
        _, ux, uy = o.moments(2, f)
        ref[k] = ux[py, px], uy[py, px]
        s, _, _ = o.step(p, f, 1, record=True)
        filtered += s.n_filtered
    err = np.abs(sig - ref)
    say(f"[hopf probe Re={re:.0f}] max |u_gpu - u_oracle| {err.max():.2e} over {steps} samples; |u| up to "
        f"{np.abs(ref).max():.3e}; filtered in the last step {st['n_filtered']} (oracle, all steps: {filtered})")
    # the probe keeps FP32 samples of the FP64 velocity: one rounding
    assert (err <= 2.0 ** -23 * np.abs(ref) + 1e-15).all()
