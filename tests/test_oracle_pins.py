"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks a property that a plausible slip in the oracle (a dropped
term, a swapped index, a wrong sign, a transposed velocity) would break,
without re-typing the oracle's own formula.
"""
import itertools
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl

mpmath.mp.dps = 50

D1Q3, D2Q9 = 1, 2
POLY, ENT = 0, 1
EXACT, QUAD = 0, 1


def rand_states(k, seed, umax=0.3):
    r = wl.uniform(seed, 3 * k).reshape(k, 3)
    rho = 0.5 + 1.5 * r[:, 0]
    u = umax * (2 * r[:, 1:] - 1)
    return rho, u


@pytest.mark.parametrize("lattice,qe", [(D1Q3, POLY), (D1Q3, ENT), (D2Q9, POLY), (D2Q9, ENT)])
def test_equilibrium_moments(orc, lattice, qe):
    """Sec. 4.1: f* carries the moments it is built from (macro_dis)."""
    v = orc.velocities(lattice)
    rho, u = rand_states(200, 11 + lattice * 2 + qe)
    for r, (ux, uy) in zip(rho, u):
        if lattice == D1Q3:
            uy = 0.0
        fs = orc.equilibrium(lattice, qe, r, ux, uy)
        assert np.all(fs > 0)
        assert abs(fs.sum() - r) <= 4e-16 * 4 * r
        assert abs((v[:, 0] * fs).sum() - r * ux) <= 1e-15 * r
        assert abs((v[:, 1] * fs).sum() - r * uy) <= 1e-15 * r


@pytest.mark.parametrize("lattice", [D1Q3, D2Q9])
def test_polynomial_second_moment_sound_speed(orc, lattice):
    """Polynomial f* has the athermal pressure tensor rho/3 I + rho u u (c_s^2 = 1/3)."""
    v = orc.velocities(lattice)
    rho, u = rand_states(50, 5)
    for r, (ux, uy) in zip(rho, u):
        if lattice == D1Q3:
            uy = 0.0
        fs = orc.equilibrium(lattice, POLY, r, ux, uy)
        pxx = (v[:, 0] ** 2 * fs).sum()
        assert pxx == pytest.approx(r / 3 + r * ux * ux, rel=1e-14)
        if lattice == D2Q9:
            assert (v[:, 1] ** 2 * fs).sum() == pytest.approx(r / 3 + r * uy * uy, rel=1e-14)
            assert (v[:, 0] * v[:, 1] * fs).sum() == pytest.approx(r * ux * uy, rel=1e-13, abs=1e-16)


def test_d1q3_entropic_max_entropy_identity(orc):
    """For H = f1 log(f1/4) + f2 log f2 + f3 log f3 the constrained maximum
    satisfies (f1*/4)^2 = f2* f3*; also pins which mover carries +u."""
    rho, u = rand_states(300, 17, umax=0.5)
    for r, (ux, _) in zip(rho, u):
        fs = orc.equilibrium(D1Q3, ENT, r, ux)
        assert (fs[0] / 4) ** 2 == pytest.approx(fs[1] * fs[2], rel=2e-15)
        # v = +1 mover (index 2) must carry the positive momentum
        assert fs[2] - fs[1] == pytest.approx(r * ux, rel=1e-14, abs=1e-16)


@pytest.mark.parametrize("lattice", [D1Q3, D2Q9])
def test_entropic_equilibrium_is_constrained_entropy_maximum(orc, lattice):
    """ln(f*_i / W_i) is affine in (1, v_i) (Lagrange condition of Sec. 3.6) and
    any moment-preserving perturbation lowers S."""
    v = orc.velocities(lattice).astype(float)
    q = len(v)
    W = np.array([4.0, 1, 1]) if lattice == D1Q3 else np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cols = [np.ones(q), v[:, 0]] + ([v[:, 1]] if lattice == D2Q9 else [])
    A = np.stack(cols, axis=1)
    null = np.linalg.svd(A.T)[2][A.shape[1]:]          # directions with zero moments
    rho, u = rand_states(60, 23, umax=0.4)
    for k, (r, (ux, uy)) in enumerate(zip(rho, u)):
        if lattice == D1Q3:
            uy = 0.0
        fs = orc.equilibrium(lattice, ENT, r, ux, uy)
        y = np.log(fs / W)
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        assert np.abs(A @ coef - y).max() < 5e-15 * max(1.0, np.abs(y).max())
        s0 = orc.entropy(lattice, fs)
        for j in range(len(null)):
            for eps in (1e-3, -1e-3):
                g = fs + eps * r * null[j]
                assert orc.entropy(lattice, g) < s0


def test_maxwellian_is_tensor_product_of_d1q3(orc):
    """eq. (maxwellian) factorises into the D1Q3 entropic equilibria per axis:
    f*_i = rho g(u_x)_{v_ix} g(u_y)_{v_iy} with g = D1Q3 f* at unit density."""
    v = orc.velocities(D2Q9)
    rho, u = rand_states(200, 29, umax=0.45)
    idx = {0: 0, -1: 1, 1: 2}
    for r, (ux, uy) in zip(rho, u):
        f2 = orc.equilibrium(D2Q9, ENT, r, ux, uy)
        gx = orc.equilibrium(D1Q3, ENT, 1.0, ux)
        gy = orc.equilibrium(D1Q3, ENT, 1.0, uy)
        for i in range(9):
            assert f2[i] == pytest.approx(r * gx[idx[v[i, 0]]] * gy[idx[v[i, 1]]], rel=5e-15)


@pytest.mark.parametrize("lattice", [D1Q3, D2Q9])
def test_entropic_minus_polynomial_is_third_order(orc, lattice):
    """Both quasiequilibria agree to second order in u.  The D2Q9 gap is third
    order (cross terms u_x u_y^2 of the product form); in D1Q3 the odd terms
    cancel and the gap is fourth order."""
    def gap(a):
        ux, uy = 0.6 * a, (-0.8 * a if lattice == D2Q9 else 0.0)
        return np.abs(orc.equilibrium(lattice, ENT, 1.0, ux, uy) - orc.equilibrium(lattice, POLY, 1.0, ux, uy)).max()
    r1 = gap(0.02) / gap(0.01)
    r2 = gap(0.04) / gap(0.02)
    order = 4 if lattice == D1Q3 else 3
    assert abs(math.log2(r1) - order) < 0.05 and abs(math.log2(r2) - order) < 0.1


@pytest.mark.parametrize("x", [-0.9, -0.5, -0.2, -0.0501, -0.0499, -0.01, -1e-4, -1e-8, 1e-8, 1e-4,
                               0.01, 0.0499, 0.0501, 0.3, 1.0, 3.0])
def test_h_kernel_matches_high_precision(orc, x):
    """h(x) = (1+x) ln(1+x) - x evaluated to ~1 ulp across the series/closed-form switch."""
    ref = (1 + mpmath.mpf(x)) * mpmath.log1p(mpmath.mpf(x)) - mpmath.mpf(x)
    assert orc.h(x) == pytest.approx(float(ref), rel=4e-15)


def moment_free_perturbation(lattice, fs, seed, scale):
    """f* + d with d orthogonal to the collision invariants."""
    v = oracle_v(lattice)
    q = len(fs)
    cols = [np.ones(q), v[:, 0]] + ([v[:, 1]] if lattice == D2Q9 else [])
    A = np.stack(cols, axis=1)
    null = np.linalg.svd(A.T)[2][A.shape[1]:]
    c = 2 * wl.uniform(seed, len(null)) - 1
    return scale * (c @ null) * fs.sum()


def oracle_v(lattice):
    from oracle import oracle
    return oracle.velocities(lattice).astype(float)


@pytest.mark.parametrize("lattice,qe", [(D1Q3, POLY), (D1Q3, ENT), (D2Q9, POLY), (D2Q9, ENT)])
@pytest.mark.parametrize("scale", [1e-7, 1e-4, 1e-2, 0.1])
def test_delta_s_matches_kullback_definition(orc, lattice, qe, scale):
    """eq. (DelS)/(Kul): Delta S = sum f ln(f/f*) >= 0, computed at 50 digits."""
    rho, u = rand_states(20, 31 + qe, umax=0.2)
    for k, (r, (ux, uy)) in enumerate(zip(rho, u)):
        fs = orc.equilibrium(lattice, qe, r, ux, uy if lattice == D2Q9 else 0.0)
        f = fs + moment_free_perturbation(lattice, fs, 100 + k, scale)
        if np.any(f <= 0):
            continue
        mf = [mpmath.mpf(a) for a in f]
        ms = [mpmath.mpf(a) for a in fs]
        kull = sum(a * mpmath.log(a / b) for a, b in zip(mf, ms))
        drift = sum(a - b for a, b in zip(mf, ms))      # rounding of the moments
        ref = kull - drift
        got = orc.delta_s(EXACT, f, fs)
        assert got >= 0
        assert got == pytest.approx(float(ref), rel=1e-13, abs=1e-300)
        quad = sum((a - b) ** 2 / (2 * b) for a, b in zip(mf, ms))
        assert orc.delta_s(QUAD, f, fs) == pytest.approx(float(quad), rel=1e-14)


@pytest.mark.parametrize("lattice", [D1Q3, D2Q9])
def test_delta_s_quadratic_limit_and_homogeneity(orc, lattice):
    """Sec. 3.6/3.8: exact/quadratic -> 1 as f -> f*, and Delta S(f* + x d) ~ x^2 Delta S."""
    fs = orc.equilibrium(lattice, ENT, 1.3, 0.07, -0.04 if lattice == D2Q9 else 0.0)
    d = moment_free_perturbation(lattice, fs, 7, 0.05)
    ratios = []
    for t in (1e-1, 1e-2, 1e-3, 1e-4):
        f = fs + t * d
        e, qd = orc.delta_s(EXACT, f, fs), orc.delta_s(QUAD, f, fs)
        ratios.append(abs(e / qd - 1))
    assert ratios[-1] < 1e-4 and all(a > b for a, b in zip(ratios, ratios[1:]))
    base = orc.delta_s(EXACT, fs + 1e-3 * d, fs)
    assert orc.delta_s(EXACT, fs + 2e-3 * d, fs) / base == pytest.approx(4.0, rel=1e-2)
    assert orc.delta_s(EXACT, fs, fs) == 0.0


def test_delta_s_nonpositive_is_infinite(orc):
    fs = orc.equilibrium(D2Q9, POLY, 1.0, 0.05, 0.0)
    f = fs.copy()
    f[3] = -1e-3
    assert math.isinf(orc.delta_s(EXACT, f, fs))
    assert math.isfinite(orc.delta_s(QUAD, f, fs))
    bad = fs.copy()
    bad[0] = 0.0
    assert math.isinf(orc.delta_s(QUAD, f, bad))


@pytest.mark.parametrize("n", [3, 9, 27])
def test_median_is_middle_of_sorted(orc, n):
    """Sec. 3.5: after sorting, the 2nd of 3, 5th of 9, 14th of 27 values."""
    for k in range(200):
        r = wl.uniform(1000 + k, n)
        if k % 3 == 0:
            r = np.round(r * 4) / 4          # many ties
        if k % 5 == 0:
            r[k % n] = np.inf
        assert orc.median(r) == sorted(r)[n // 2]


def one_site(orc, **kw):
    """A 1x1 periodic D2Q9 grid: free flight maps the node onto itself, so a
    step returns exactly the limited post-collision state."""
    return orc.make_params(lattice=D2Q9, nx=1, ny=1, **kw)


@pytest.mark.parametrize("qe", [POLY, ENT])
def test_collision_special_betas(orc, qe):
    """eq. (collLBGK): beta = 0 keeps f, 1/2 equilibrates, 1 reflects through f*."""
    fs = orc.equilibrium(D2Q9, qe, 1.1, 0.05, 0.02)
    f0 = fs + moment_free_perturbation(D2Q9, fs, 3, 0.05)
    for beta, expect in ((0.0, f0), (0.5, fs), (1.0, 2 * fs - f0)):
        p = one_site(orc, beta=beta, qe=qe)
        f = f0.reshape(9, 1, 1).copy()
        st, _, _ = orc.step(p, f)
        assert np.allclose(f.ravel(), expect, rtol=4e-15, atol=1e-16)
    # fixed point: f* is not moved by any beta
    for beta in (0.1, 0.7, 1.0):
        f = fs.reshape(9, 1, 1).copy()
        orc.step(orc.make_params(lattice=D2Q9, nx=1, ny=1, beta=beta, qe=qe), f)
        # a few ulp: f* is rebuilt from the rounded moments of f*
        assert np.all(np.abs(f.ravel() - fs) <= 8 * np.spacing(fs))


def test_lbgk_entropy_production_quadratic(orc):
    """Sec. 3.4: in the quadratic form Delta S(f') = (2 beta - 1)^2 Delta S(f)."""
    beta = 0.83
    p = one_site(orc, beta=beta, qe=POLY, ds_form=QUAD)
    fs = orc.equilibrium(D2Q9, POLY, 1.0, 0.03, 0.01)
    f = (fs + moment_free_perturbation(D2Q9, fs, 9, 0.03)).reshape(9, 1, 1).copy()
    st, _, _ = orc.step(p, f)
    assert st.sum_dS_post == pytest.approx((2 * beta - 1) ** 2 * st.sum_dS_pre, rel=1e-12)
    assert st.lbgk_production == pytest.approx((1 - (2 * beta - 1) ** 2) * st.sum_dS_pre, rel=1e-14)


@pytest.mark.parametrize("form", [EXACT, QUAD])
def test_trimming_homothety_hits_threshold_and_keeps_moments(orc, form):
    """eq. (entrHom): the trimmed state keeps rho, u and, in the quadratic form,
    its nonequilibrium entropy equals the threshold; 0 <= phi <= 1."""
    delta = 1e-4
    for k in range(20):
        p = one_site(orc, beta=0.97, qe=ENT, ds_form=form, limiter=1, delta_trim=delta)
        fs = orc.equilibrium(D2Q9, ENT, 1.0, 0.04, -0.02)
        f0 = fs + moment_free_perturbation(D2Q9, fs, 50 + k, 0.02 * (k + 1) / 20)
        f = f0.reshape(9, 1, 1).copy()
        st, mask, ds = orc.step(p, f, record=True)
        out = f.ravel()
        assert out.sum() == pytest.approx(f0.sum(), rel=1e-15)
        v = orc.velocities(D2Q9)
        assert (v[:, 0] * out).sum() == pytest.approx((v[:, 0] * f0).sum(), rel=1e-12, abs=1e-16)
        after = orc.delta_s(form, out, fs)
        if mask[0, 0] & 1:
            assert ds[0, 0] > delta
            if form == QUAD:
                assert after == pytest.approx(delta, rel=1e-12)
            assert after <= ds[0, 0]
            assert st.limiter_production == pytest.approx(ds[0, 0] - after, rel=1e-9)
        else:
            assert after == pytest.approx(ds[0, 0], rel=1e-12)


def test_threshold_limiter_is_double_monotonic(orc):
    """Sec. 3.8: the threshold homothety is dissipative and order preserving:
    the limited Delta S is nondecreasing in the amplitude y of f - f*."""
    fs = orc.equilibrium(D2Q9, POLY, 1.0, 0.02, 0.03)
    d = moment_free_perturbation(D2Q9, fs, 77, 0.01)
    prev = -1.0
    for y in np.linspace(0.05, 3.0, 80):
        p = one_site(orc, beta=1.0, qe=POLY, ds_form=QUAD, limiter=1, delta_trim=2e-5)
        f = (fs + y * d).reshape(9, 1, 1).copy()
        orc.step(p, f)
        after = orc.delta_s(QUAD, f.ravel(), fs)
        before = orc.delta_s(QUAD, fs + y * d, fs)
        assert after <= before * (1 + 1e-12)
        assert after >= prev * (1 - 1e-12)
        prev = after


def test_ehrenfest_step_returns_to_equilibrium(orc):
    """Sec. 3.2: sites above the threshold jump to f*."""
    p = one_site(orc, beta=0.99, qe=POLY, limiter=1, trim_mode=1, delta_trim=1e-6)
    fs = orc.equilibrium(D2Q9, POLY, 1.0, 0.01, 0.02)
    f = (fs + moment_free_perturbation(D2Q9, fs, 5, 0.05)).reshape(9, 1, 1).copy()
    st, mask, _ = orc.step(p, f, record=True)
    assert mask[0, 0] & 1 and st.n_trimmed == 1
    assert np.allclose(f.ravel(), fs, rtol=1e-14)


@pytest.mark.parametrize("bc,lattice,nx,ny", [(0, D2Q9, 7, 5), (0, D1Q3, 11, 1), (2, D1Q3, 9, 1), (1, D2Q9, 6, 5)])
def test_free_flight_is_a_permutation(orc, bc, lattice, nx, ny):
    """Sec. 2: free flight is exact and linear; with edge reflection at the
    non-periodic edges it moves every population value somewhere (bitwise)."""
    p = orc.make_params(lattice=lattice, nx=nx, ny=ny, bc=bc)
    q = orc.q_of(lattice)
    o = wl.uniform(99, q * nx * p.ny).reshape(q, p.ny, nx)
    f = orc.stream(p, o)
    assert np.array_equal(np.sort(f.ravel()), np.sort(o.ravel()))
    if bc == 0:
        g = o.copy()
        period = nx * p.ny
        for _ in range(int(np.lcm(nx, p.ny))):
            g = orc.stream(p, g)
        assert np.array_equal(g, o)
        # each population moves by its velocity
        v = orc.velocities(lattice)
        for i in range(q):
            assert np.array_equal(f[i], np.roll(np.roll(o[i], v[i, 0], axis=1), v[i, 1], axis=0))


def test_tube_ends_bounce_back_halfway(orc):
    """Tube ends: a mover leaving the domain re-enters the same end site reversed."""
    p = orc.make_params(lattice=D1Q3, nx=5, bc=2)
    o = np.zeros((3, 1, 5))
    o[1, 0, 0] = 7.0     # left mover at the left end
    o[2, 0, 4] = 9.0     # right mover at the right end
    f = orc.stream(p, o)
    assert f[2, 0, 0] == 7.0 and f[1, 0, 4] == 9.0 and f.sum() == 16.0


def fr(x):
    return Fraction(x)


def test_tiny_grid_exact_rational_step(orc):
    """A 3x3 periodic D2Q9 polynomial LBGK step in exact rational arithmetic
    (no limiter), written from eq. (polyeq2d), (macro_dis), (lbgkLB)."""
    p = orc.make_params(lattice=D2Q9, nx=3, ny=3, beta=0.75, qe=POLY)
    f = wl.random_populations(9, 3, 3, seed=4, amp=0.1)
    f = np.round(f * 2 ** 20) / 2 ** 20        # exactly representable inputs
    vx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    vy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    w = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4
    beta = Fraction(3, 4)
    out = [[[None] * 3 for _ in range(3)] for _ in range(9)]
    for y in range(3):
        for x in range(3):
            fl = [fr(f[i, y, x]) for i in range(9)]
            rho = sum(fl)
            ux = sum(vx[i] * fl[i] for i in range(9)) / rho
            uy = sum(vy[i] * fl[i] for i in range(9)) / rho
            for i in range(9):
                cu = vx[i] * ux + vy[i] * uy
                fs = rho * w[i] * (1 + 3 * cu + Fraction(9, 2) * cu * cu - Fraction(3, 2) * (ux * ux + uy * uy))
                out[i][(y + vy[i]) % 3][(x + vx[i]) % 3] = fs + (2 * beta - 1) * (fs - fl[i])
    g = f.copy()
    orc.step(p, g)
    ref = np.array([[[float(out[i][y][x]) for x in range(3)] for y in range(3)] for i in range(9)])
    assert np.allclose(g, ref, rtol=1e-14, atol=0)
