"""Mirror symmetry of the oracle's cavity step (Sec. 4.4).

No printed value fixes the near-wall and corner median stencils of the
cavity, but the rule has to treat the left and right walls alike: reflecting
a state left to right (x -> nx - 1 - x, each velocity's x component negated)
and reversing the lid must give the reflected result, decisions included.
A wall stencil taken on the wrong side, or a corner rule that mixes up its
neighbours, breaks this.  Bounce-back and diffusive walls, trimming and the
median filter in both tolerance readings, exact and quadratic Delta S."""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl

D2Q9 = 2
CAVITY, DIFFUSIVE = 1, 3


def mirror_map(orc):
    v = orc.velocities(D2Q9)
    return [int(np.flatnonzero((v[:, 0] == -v[i, 0]) & (v[:, 1] == v[i, 1]))[0]) for i in range(9)]


def mirrored(f, mp):
    return np.ascontiguousarray(f[mp][:, :, ::-1])


@pytest.mark.parametrize("bc", [CAVITY, DIFFUSIVE])
@pytest.mark.parametrize("median_mode", [0, 1])
@pytest.mark.parametrize("ds", [0, 1])
def test_cavity_step_is_mirror_symmetric(orc, bc, median_mode, ds):
    nx, ny = 40, 30
    mp = mirror_map(orc)
    assert sorted(mp) == list(range(9)) and all(mp[mp[i]] == i for i in range(9))
    f0 = wl.random_populations(9, nx, ny, seed=31, amp=0.02, spike_frac=0.15, spike_amp=0.3)
    kw = dict(lattice=D2Q9, nx=nx, ny=ny, beta=0.98, qe=1, ds_form=ds, limiter=3, median_mode=median_mode,
              bc=bc, delta_trim=2e-3, delta_median=1e-6, rho0=1.0)
    a = f0.copy()
    st_a, m_a, d_a = orc.step(orc.make_params(lid_ux=0.1, **kw), a, 3, record=True)
    b = mirrored(f0, mp)
    st_b, m_b, d_b = orc.step(orc.make_params(lid_ux=-0.1, **kw), b, 3, record=True)
    # the filter acts next to the side walls, so their stencils are exercised
    filt = (m_a & 2) != 0
    assert filt[1:-1, 1].any() and filt[1:-1, -2].any()
    np.testing.assert_array_equal(m_b, m_a[:, ::-1])
    np.testing.assert_allclose(d_b, d_a[:, ::-1], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(b, mirrored(a, mp), rtol=1e-12, atol=1e-15)
    assert st_b.n_filtered == st_a.n_filtered and st_b.n_trimmed == st_a.n_trimmed
    assert st_b.mass == pytest.approx(st_a.mass, rel=1e-14)
    assert st_b.mom_x == pytest.approx(-st_a.mom_x, rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("bc", [CAVITY, DIFFUSIVE])
@pytest.mark.parametrize("median_mode", [0, 1])
def test_corner_stencils_are_mirror_symmetric(orc, bc, median_mode):
    """Strongly nonequilibrium states planted at the four inner corners (each
    with its own pattern) are filtered by the corner rule, and the step stays
    mirror symmetric."""
    nx, ny = 24, 20
    mp = mirror_map(orc)
    f0 = wl.random_populations(9, nx, ny, seed=37, amp=0.01, spike_frac=0.0)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    for k, (y, x) in enumerate([(1, 1), (1, nx - 2), (ny - 2, 1), (ny - 2, nx - 2)]):
        pattern = 2 * wl.uniform(100 + k, 9) - 1
        f0[:, y, x] = w * (1 + 0.4 * pattern)
    kw = dict(lattice=D2Q9, nx=nx, ny=ny, beta=0.98, qe=1, ds_form=0, limiter=2, median_mode=median_mode,
              bc=bc, delta_median=1e-6, rho0=1.0)
    a = f0.copy()
    st_a, m_a, d_a = orc.step(orc.make_params(lid_ux=0.1, **kw), a, 1, record=True)
    b = mirrored(f0, mp)
    st_b, m_b, d_b = orc.step(orc.make_params(lid_ux=-0.1, **kw), b, 1, record=True)
    filt = (m_a & 2) != 0
    assert filt[1, 1] and filt[1, -2] and filt[-2, 1] and filt[-2, -2]
    np.testing.assert_array_equal(m_b, m_a[:, ::-1])
    np.testing.assert_allclose(d_b, d_a[:, ::-1], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(b, mirrored(a, mp), rtol=1e-12, atol=1e-15)
