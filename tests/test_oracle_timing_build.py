"""The oracle's OpenMP build (the CPU baseline's timing build, and the oracle
that the long GPU parity runs compare against) gives bit for bit what the
plain build gives: the same source, its per-node loops spread over rows,
every global sum still taken in row-major order.  Populations, the last
step's masks and Delta S', and every stat are compared exactly on each
boundary, limiter family and collision."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_0704_0043_amd import workloads as wl

CASES = [
    ("periodic trim+median poly exact", dict(lattice=o.D2Q9, nx=61, ny=37, qe=0, ds_form=0, limiter=3,
                                             delta_trim=1e-4, delta_median=1e-5), 5),
    ("periodic trim+median entropic quad", dict(lattice=o.D2Q9, nx=61, ny=37, qe=1, ds_form=1, limiter=3,
                                                delta_trim=1e-4, delta_median=1e-5), 5),
    ("periodic GATE median, Ehrenfest trim", dict(lattice=o.D2Q9, nx=48, ny=33, qe=0, ds_form=1, limiter=3,
                                                  trim_mode=o.TRIM_EHRENFEST, median_mode=o.MED_GATE,
                                                  delta_trim=1e-4, delta_median=1e-5), 4),
    ("periodic budget threshold", dict(lattice=o.D2Q9, nx=40, ny=30, qe=0, ds_form=1,
                                       limiter=o.LIM_MEDIAN | o.LIM_ENS_BUDGET, ens_c=0.05,
                                       delta_median=1e-5), 4),
    ("periodic smooth factor", dict(lattice=o.D2Q9, nx=40, ny=30, qe=0, ds_form=1,
                                    limiter=o.LIM_TRIM | o.LIM_ENS_SMOOTH, ens_k=0.5, delta_ens=0.01,
                                    delta_trim=1e-4), 4),
    ("periodic ELBM + positivity", dict(lattice=o.D2Q9, nx=40, ny=30, qe=1, ds_form=0,
                                        limiter=o.LIM_POSITIVITY, collision=o.COLL_ELBM), 3),
    ("bounce-back cavity", dict(lattice=o.D2Q9, nx=33, ny=29, qe=1, ds_form=1, limiter=2, bc=o.BC_CAVITY,
                                delta_median=1e-4, lid_ux=0.1), 8),
    ("diffusive cavity", dict(lattice=o.D2Q9, nx=33, ny=29, qe=0, ds_form=0, limiter=2,
                              bc=o.BC_CAVITY_DIFFUSIVE, delta_median=1e-4, lid_ux=0.1), 8),
    ("shock tube", dict(lattice=o.D1Q3, nx=300, qe=0, ds_form=0, limiter=3, bc=o.BC_TUBE,
                        delta_trim=1e-3, delta_median=1e-3), 20),
]


def _same_stats(a, b):
    for k, v in a.items():
        w = b[k]
        assert v == w or (v != v and w != w), (k, v, w)


@pytest.mark.parametrize("name,kw,steps", CASES, ids=[c[0] for c in CASES])
def test_openmp_build_is_bit_identical(name, kw, steps):
    p = o.make_params(beta=0.97, **kw)
    q = o.q_of(p.lattice)
    f0 = wl.random_populations(q, p.nx, p.ny, seed=17 + steps, amp=0.05, spike_frac=0.05, spike_amp=0.4)
    fa = np.ascontiguousarray(f0, dtype=np.float64).copy()
    fb = fa.copy()
    sa, ma, da = o.step(p, fa, steps, record=True)
    sb, mb, db = o.step(p, fb, steps, record=True, handle=o.timing_lib())
    assert o.timing_lib().orc_threads() >= 1
    assert np.array_equal(fa, fb)
    assert np.array_equal(ma, mb)
    assert np.array_equal(da, db, equal_nan=True)
    _same_stats(sa.as_dict(), sb.as_dict())
