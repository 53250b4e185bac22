"""Pins of the oracle's exact-entropy homothety (Sec. 3.6: phi solves
S(f* + phi (f - f*)) = S(f*) - Delta S_t) and of top-k trimming (Sec. 3.2:
Ehrenfests' steps at the k nodes of largest Delta S above delta).

The limited states are checked with the Kullback entropy computed here from
its definition, sum f ln(f / f*), not with the oracle's Delta S routine."""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl

D2Q9 = 2
EXACT, QUAD = 0, 1
TRIM, MEDIAN, THRESH = 1, 2, 4


def kullback(f, fs):
    return float(np.sum(f * np.log(f / fs)))


def fstar_of(orc, f, qe=0):
    rho, ux, uy = orc.moments(D2Q9, np.asarray(f, dtype=np.float64).reshape(9, 1, 1))
    return orc.equilibrium(D2Q9, qe, rho.item(), ux.item(), uy.item())


def one_node(orc, f, **kw):
    base = dict(lattice=D2Q9, nx=1, ny=1, beta=0.9, qe=0, ds_form=EXACT)
    base.update(kw)
    p = orc.make_params(**base)
    out = np.ascontiguousarray(f, dtype=np.float64).reshape(9, 1, 1).copy()
    st, mask, ds = orc.step(p, out, 1, record=True)
    return out.ravel(), st, float(ds.ravel()[0])


@pytest.mark.parametrize("amp,delta", [(0.3, 1e-3), (0.6, 1e-2), (0.05, 1e-5)])
def test_exact_homothety_lands_on_the_threshold(orc, amp, delta):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = w * (1 + amp * (wl.uniform(int(amp * 100), 9) * 2 - 1))
    fs = fstar_of(orc, f)
    beta = 0.9
    fp = fs + (2 * beta - 1) * (fs - f)
    d = kullback(fp, fs)
    assert d > delta
    out, st, _ = one_node(orc, f, beta=beta, limiter=TRIM, delta_trim=delta, homothety=1)
    assert st.n_trimmed == 1
    assert kullback(out, fs) == pytest.approx(delta, rel=1e-11)
    # on the line from f* through f'
    phi = (out - fs) / (fp - fs)
    np.testing.assert_allclose(phi, phi[0], rtol=1e-9)
    assert 0.0 < phi[0] < 1.0
    # the quadratic coefficient misses the threshold unless the state is close to f*
    q, _, _ = one_node(orc, f, beta=beta, limiter=TRIM, delta_trim=delta, homothety=0)
    miss = abs(kullback(q, fs) / delta - 1)
    assert miss > 1e-6 if amp > 0.1 else miss < 0.05


def test_exact_homothety_for_the_median_and_threshold_limiters(orc):
    """The median filter's and the threshold limiter's targets are reached
    exactly too (a field with spikes, one step, Delta S of every moved node)."""
    f0 = wl.random_populations(9, 30, 24, seed=41, amp=0.02, spike_frac=0.1, spike_amp=0.4)
    for lim, kw in ((MEDIAN, dict(delta_median=1e-6)), (THRESH, dict(ens_c=3.0))):
        p = orc.make_params(lattice=D2Q9, nx=30, ny=24, beta=0.95, qe=0, ds_form=EXACT, limiter=lim,
                            homothety=1, **kw)
        f = f0.copy()
        st, mask, ds, dsl = orc.step(p, f, 1, record=True, record_lim=True)
        moved = (mask & (2 | 16)) != 0
        assert moved.sum() > 5
        if lim == THRESH:
            np.testing.assert_allclose(dsl[moved], st.ens_threshold, rtol=1e-11)
        else:
            assert np.all(dsl[moved] < ds[moved])
        # every moved node ends at its target: below the unmoved Delta S'
        assert np.all(dsl[~moved] == ds[~moved])


def topk_field(seed, nx=40, ny=30):
    return wl.random_populations(9, nx, ny, seed=seed, amp=0.03, spike_frac=0.2, spike_amp=0.3)


@pytest.mark.parametrize("k", [1, 17, 100])
def test_top_k_trims_the_k_largest(orc, k):
    f0 = topk_field(42)
    p = orc.make_params(lattice=D2Q9, nx=40, ny=30, beta=0.95, qe=0, ds_form=EXACT, limiter=TRIM,
                        trim_mode=1, delta_trim=1e-5, top_k=k)
    f = f0.copy()
    st, mask, ds = orc.step(p, f, 1, record=True)
    trimmed = (mask & 1) != 0
    above = ds > 1e-5
    assert above.sum() > k
    assert trimmed.sum() == k == st.n_trimmed
    assert ds[trimmed].min() > ds[above & ~trimmed].max()
    # Ehrenfests' steps: those nodes went to f* (unlimited: the full set above delta)
    p0 = orc.make_params(lattice=D2Q9, nx=40, ny=30, beta=0.95, qe=0, ds_form=EXACT, limiter=TRIM,
                         trim_mode=1, delta_trim=1e-5)
    g = f0.copy()
    st0, mask0, _ = orc.step(p0, g, 1, record=True)
    assert st0.n_trimmed == above.sum()


def test_top_k_ties_and_infinities(orc):
    """Nodes with equal Delta S' at the k-th value are all trimmed; a node
    with a negative population (Delta S' = +inf) is trimmed whatever k."""
    nx, ny = 20, 10
    f0 = wl.random_populations(9, nx, ny, seed=43, amp=0.03, spike_frac=0.0)
    # three identical spiky nodes, the largest Delta S' of the field
    spike = f0[:, 5, 5] * np.array([1, 1.5, 1, 0.5, 1, 1.6, 1, 0.4, 1])
    for x in (2, 9, 15):
        f0[:, 3, x] = spike
    # a population far above f*: the over-relaxed state goes negative there
    f0[5, 8, 8] *= 4.0
    p = orc.make_params(lattice=D2Q9, nx=nx, ny=ny, beta=0.95, qe=0, ds_form=EXACT, limiter=TRIM,
                        trim_mode=1, delta_trim=1e-6, top_k=2)
    f = f0.copy()
    st, mask, ds = orc.step(p, f, 1, record=True)
    trimmed = (mask & 1) != 0
    assert np.isinf(ds[8, 8]) and trimmed[8, 8]
    assert all(trimmed[3, x] for x in (2, 9, 15))
    assert trimmed.sum() == 4
