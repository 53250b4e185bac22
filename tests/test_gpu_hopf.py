"""The Hopf pipeline (Sec. 4.4.2) end to end on the device, shortened: a
batch of diffusive-wall cavities runs with its probes recording, and the
probe signal is the velocity the context reports at the probe node."""
import numpy as np
import pytest

from paper_0704_0043_amd import hopf
from tests.gpu_util import lbm, require_gpu, say

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
