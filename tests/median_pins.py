"""Independent checks of the oracle's median entropy filter (Sec. 3.5; the
cavity stencils of Sec. 4.4), written with numpy and shared by the pin tests
of the real oracle and by the tests that plant mistakes in copies of it.

Nothing here calls the oracle's arithmetic except `orc.step` itself: the
post-collision Delta S' of every node is recomputed from the input state
(moments, f* of Sec. 4.1, eq. (collLBGK)), the medians come from np.roll
and np.median, the FLOOR / GATE decisions are taken again from the recorded
values, and the landing of every filtered node on its target is read off the
populations that came out of the step (free flight undone by np.roll).

Each check raises AssertionError when the oracle disagrees."""
from __future__ import annotations

import numpy as np

from paper_0704_0043_amd import workloads as wl

D1Q3, D2Q9 = 1, 2
POLY, ENTROPIC = 0, 1
EXACT, QUAD = 0, 1
TRIM, MEDIAN = 1, 2
FLOOR, GATE = 0, 1
PERIODIC, CAVITY, TUBE = 0, 1, 2
M_TRIM, M_MEDIAN, M_NOTFLUID = 1, 2, 8

# lattices of Sec. 4.1, written out here independently of the oracle
V9 = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
V3 = np.array([0, -1, 1])


def _axis_factor(u, v):
    """1-D factor of eq. (maxwellian): (2 - s) B^v, s = sqrt(1 + 3u^2),
    B = (2u + s) / (1 - u)."""
    s = np.sqrt(1.0 + 3.0 * u * u)
    b = (2.0 * u + s) / (1.0 - u)
    return (2.0 - s) * b ** v


def fstar2d(qe, rho, ux, uy):
    out = np.empty((9,) + np.shape(rho))
    for i, (vx, vy) in enumerate(V9):
        if qe == POLY:
            cu = vx * ux + vy * uy
            out[i] = rho * W9[i] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
        else:
            out[i] = rho * W9[i] * _axis_factor(ux, vx) * _axis_factor(uy, vy)
    return out


def fstar1d(qe, rho, u):
    if qe == POLY:
        return np.stack([2 * rho / 3 * (1 - 1.5 * u * u), rho / 6 * (1 - 3 * u + 3 * u * u),
                         rho / 6 * (1 + 3 * u + 3 * u * u)])
    w = np.array([2 / 3, 1 / 6, 1 / 6])
    return np.stack([rho * w[i] * _axis_factor(u, V3[i]) for i in range(3)])


def fstar_of(lattice, qe, f):
    if lattice == D2Q9:
        rho = f.sum(axis=0)
        ux = np.tensordot(V9[:, 0], f, axes=1) / rho
        uy = np.tensordot(V9[:, 1], f, axes=1) / rho
        return fstar2d(qe, rho, ux, uy)
    rho = f.sum(axis=0)
    u = np.tensordot(V3, f, axes=1) / rho
    return fstar1d(qe, rho, u)


# absolute rounding of sum f ln(f / f*) computed directly (its terms are first
# order in f - f*, the sum second order)
DS_ATOL = 1e-15


def delta_s(form, f, fs):
    """Delta S summed over the population axis: sum f ln(f / f*) (eq. DelS),
    or half the chi-square form of Sec. 3.6."""
    if form == QUAD:
        return 0.5 * np.sum((f - fs) ** 2 / fs, axis=0)
    return np.sum(f * np.log(f / fs), axis=0)


def post_collision(lattice, qe, beta, f):
    fs = fstar_of(lattice, qe, f)
    return fs, fs + (2 * beta - 1) * (fs - f)


def unstream_periodic(lattice, f):
    """Free flight undone on a periodic grid: population i came from x - v_i."""
    out = np.empty_like(f)
    if lattice == D2Q9:
        for i, (vx, vy) in enumerate(V9):
            out[i] = np.roll(np.roll(f[i], -vy, axis=0), -vx, axis=1)
    else:
        for i in range(3):
            out[i] = np.roll(f[i], -V3[i], axis=-1)
    return out


def median_periodic(ds):
    """3x3 (2-D) or 3-point (1-D) median of every node, wrapping at the seams."""
    if ds.shape[0] == 1:
        stack = [np.roll(ds, k, axis=1) for k in (-1, 0, 1)]
    else:
        stack = [np.roll(np.roll(ds, dy, axis=0), dx, axis=1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return np.median(np.stack(stack), axis=0)


def median_cavity(ds):
    """Cavity stencils (Sec. 4.4, as read here): wall and lid nodes are never
    filtered and never enter a stencil; a fluid node next to one wall takes
    itself and its two neighbours along that wall; a fluid node next to two
    walls takes itself and its two inner axis neighbours; all others the 3x3
    block.  NaN marks nodes that are not filtered."""
    ny, nx = ds.shape
    med = np.full(ds.shape, np.nan)
    for y in range(1, ny - 1):
        for x in range(1, nx - 1):
            side = x in (1, nx - 2)
            flat = y in (1, ny - 2)
            if side and flat:
                ix = 1 if x == 1 else -1
                iy = 1 if y == 1 else -1
                vals = [ds[y, x], ds[y, x + ix], ds[y + iy, x]]
            elif side:
                vals = [ds[y - 1, x], ds[y, x], ds[y + 1, x]]
            elif flat:
                vals = [ds[y, x - 1], ds[y, x], ds[y, x + 1]]
            else:
                vals = list(ds[y - 1:y + 2, x - 1:x + 2].ravel())
            med[y, x] = np.median(vals)
    return med


def decide(ds, med, delta, mode):
    """Filter decision and target: FLOOR corrects where Delta S' > max(med, delta)
    to that value; GATE where Delta S' > delta and Delta S' > med, to med."""
    with np.errstate(invalid="ignore"):
        if mode == FLOOR:
            thr = np.maximum(med, delta)
            hit = ds > thr
        else:
            thr = med
            hit = (ds > delta) & (ds > med)
    hit &= ~np.isnan(med)
    return hit, thr


def run_oracle(orc, p, f0):
    f = np.ascontiguousarray(f0, dtype=np.float64).copy()
    st, mask, ds, dsl = orc.step(p, f, 1, record=True, record_lim=True)
    return f, st, mask, ds, dsl


def check_periodic_2d(orc, ds_form, mode, delta, qe=POLY, beta=0.8, nx=26, ny=22, seed=11, homothety=0):
    """One step of a periodic D2Q9 grid with the median filter alone."""
    f0 = wl.random_populations(9, nx, ny, seed=seed, amp=0.05, spike_frac=0.08, spike_amp=0.4)
    p = orc.make_params(lattice=D2Q9, nx=nx, ny=ny, beta=beta, qe=qe, ds_form=ds_form, limiter=MEDIAN,
                        median_mode=mode, delta_median=delta, bc=PERIODIC, homothety=homothety)
    f, st, mask, ds, dsl = run_oracle(orc, p, f0)
    # Delta S' of the post-collision state, recomputed from the input
    fs, fp = post_collision(D2Q9, qe, beta, f0)
    np.testing.assert_allclose(ds, delta_s(ds_form, fp, fs), rtol=1e-9, atol=DS_ATOL)
    med = median_periodic(ds)
    hit, thr = decide(ds, med, delta, mode)
    np.testing.assert_array_equal((mask & M_MEDIAN) != 0, hit)
    assert st.n_filtered == int(hit.sum())
    assert hit.sum() >= 5, "the case must filter some nodes"
    # the filtered states land on the target: read off the step's output
    flim = unstream_periodic(D2Q9, f)
    fsl = fstar_of(D2Q9, qe, flim)
    got = delta_s(ds_form, flim, fsl)
    exact_target = ds_form == QUAD or homothety
    if exact_target:
        np.testing.assert_allclose(got[hit], thr[hit], rtol=1e-8)
        np.testing.assert_allclose(dsl[hit], thr[hit], rtol=1e-11)
        assert np.all(dsl[hit] <= thr[hit] * (1 + 1e-13))
    else:
        # eq. (entrHom): phi = sqrt(t / Delta S') scales f' - f*
        phi = np.sqrt(thr[hit] / ds[hit])
        want = delta_s(ds_form, fs[:, hit] + phi * (fp[:, hit] - fs[:, hit]), fs[:, hit])
        np.testing.assert_allclose(got[hit], want, rtol=1e-8)
    # nodes the filter leaves alone keep the post-collision state
    np.testing.assert_allclose(flim[:, ~hit], fp[:, ~hit], rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(dsl[~hit], ds[~hit])


def check_cavity(orc, ds_form, mode, delta, qe=POLY, beta=0.8, nx=14, ny=12, seed=5):
    """One cavity step from random states: the near-wall and corner stencils."""
    f0 = wl.random_populations(9, nx, ny, seed=seed, amp=0.05, spike_frac=0.15, spike_amp=0.4)
    p = orc.make_params(lattice=D2Q9, nx=nx, ny=ny, beta=beta, qe=qe, ds_form=ds_form, limiter=MEDIAN,
                        median_mode=mode, delta_median=delta, bc=CAVITY, rho0=1.0, lid_ux=0.1)
    f, st, mask, ds, dsl = run_oracle(orc, p, f0)
    fluid = np.zeros((ny, nx), bool)
    fluid[1:ny - 1, 1:nx - 1] = True
    np.testing.assert_array_equal((mask & M_NOTFLUID) != 0, ~fluid)
    fs, fp = post_collision(D2Q9, qe, beta, f0)
    np.testing.assert_allclose(ds[fluid], delta_s(ds_form, fp, fs)[fluid], rtol=1e-9, atol=DS_ATOL)
    med = median_cavity(ds)
    hit, thr = decide(ds, med, delta, mode)
    np.testing.assert_array_equal((mask & M_MEDIAN) != 0, hit)
    edge = hit.copy()
    edge[2:ny - 2, 2:nx - 2] = False
    assert edge.sum() >= 3, "the case must filter nodes next to the walls"
    if ds_form == QUAD:
        np.testing.assert_allclose(dsl[hit], thr[hit], rtol=1e-11)


def check_d1q3(orc, bc, ds_form, mode, delta, qe=POLY, beta=0.75, nx=200, seed=3):
    f0 = wl.random_populations(3, nx, 1, seed=seed, amp=0.05, spike_frac=0.1, spike_amp=0.4)
    # a strongly nonequilibrium state at the left end: a stencil that reached
    # it would filter it
    f0[1, 0, 0] *= 1.5
    p = orc.make_params(lattice=D1Q3, nx=nx, beta=beta, qe=qe, ds_form=ds_form, limiter=MEDIAN,
                        median_mode=mode, delta_median=delta, bc=bc)
    f, st, mask, ds, dsl = run_oracle(orc, p, f0)
    fs, fp = post_collision(D1Q3, qe, beta, f0)
    np.testing.assert_allclose(ds, delta_s(ds_form, fp, fs), rtol=1e-9, atol=DS_ATOL)
    med = median_periodic(ds)
    if bc == TUBE:
        # the left end would be filtered by a 3-point stencil around it
        assert ds[0, 0] > max(med[0, 0], delta)
        med[0, 0] = med[0, -1] = np.nan      # tube ends are not filtered
    hit, thr = decide(ds, med, delta, mode)
    np.testing.assert_array_equal((mask & M_MEDIAN) != 0, hit)
    assert hit.sum() >= 5
    if ds_form == QUAD:
        np.testing.assert_allclose(dsl[hit], thr[hit], rtol=1e-11)
    if bc == PERIODIC:
        flim = unstream_periodic(D1Q3, f)
        got = delta_s(ds_form, flim, fstar_of(D1Q3, qe, flim))
        if ds_form == QUAD:
            np.testing.assert_allclose(got[hit], thr[hit], rtol=1e-8)


def check_translation(orc, ds_form, mode, shift, nx=24, ny=20, seed=17):
    """A periodic step commutes with translations: shifting the input by
    `shift` (across the seams) shifts the output, the masks and Delta S'
    exactly, with trimming and the median filter both on."""
    f0 = wl.random_populations(9, nx, ny, seed=seed, amp=0.05, spike_frac=0.1, spike_amp=0.4)
    p = orc.make_params(lattice=D2Q9, nx=nx, ny=ny, beta=0.85, qe=POLY, ds_form=ds_form,
                        limiter=TRIM | MEDIAN, median_mode=mode, delta_trim=2e-3, delta_median=1e-5,
                        bc=PERIODIC)
    dy, dx = shift
    f_a, st_a, mask_a, ds_a, _ = run_oracle(orc, p, f0)
    f_b, st_b, mask_b, ds_b, _ = run_oracle(orc, p, np.roll(np.roll(f0, dy, axis=1), dx, axis=2))
    np.testing.assert_array_equal(np.roll(np.roll(f_a, dy, axis=1), dx, axis=2), f_b)
    np.testing.assert_array_equal(np.roll(np.roll(mask_a, dy, axis=0), dx, axis=1), mask_b)
    np.testing.assert_array_equal(np.roll(np.roll(ds_a, dy, axis=0), dx, axis=1), ds_b)
    assert st_a.n_filtered == st_b.n_filtered and st_a.n_filtered > 0


def all_checks(orc):
    """Every check above once, for the tests that plant mistakes in the oracle
    (each planted mistake must make at least one of these raise)."""
    for form in (QUAD, EXACT):
        for mode in (FLOOR, GATE):
            for delta in (0.0, 3e-4):
                check_periodic_2d(orc, form, mode, delta, homothety=1 if form == EXACT else 0)
                check_cavity(orc, form, mode, delta)
    for bc in (PERIODIC, TUBE):
        for mode in (FLOOR, GATE):
            check_d1q3(orc, bc, QUAD, mode, 2e-4)
    check_translation(orc, QUAD, FLOOR, (5, -7))
    check_translation(orc, EXACT, GATE, (1, 23))
