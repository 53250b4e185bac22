"""The seeded input generators (CPU): the counter-based generator against
its published recurrence, and each synthetic flow against the properties
that define it (divergence, amplitude, mean density, determinism)."""
import math

import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl

M64 = (1 << 64) - 1


def splitmix64_reference(seed, count):
    """splitmix64 as published (Steele, Lea & Flood 2014): advance the state
    by the golden gamma, then mix; plain Python integers."""
    out, s = [], seed & M64
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


@pytest.mark.parametrize("seed", [0, 1, wl.DEFAULT_SEED, M64])
def test_splitmix64_follows_the_published_recurrence(seed):
    got = [int(v) for v in wl.splitmix64(seed, 200)]
    assert got == splitmix64_reference(seed, 200)


def test_splitmix64_first_output_from_zero():
    assert int(wl.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_uniform_is_in_the_unit_interval_and_unbiased():
    u = wl.uniform(12345, 200_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert np.array_equal(u, wl.uniform(12345, 200_000))
    assert not np.array_equal(u[:100], wl.uniform(12346, 100))


@pytest.mark.parametrize("nu", [1e-9, 1e-4, 0.01, 0.5])
def test_viscosity_and_beta_are_inverse(nu):
    b = wl.beta_from_nu(nu)
    assert 0 < b <= 1
    assert wl.nu_from_beta(b) == pytest.approx(nu, rel=1e-12)
    # nu = c_s^2 (1/(2 beta) - 1/2) with c_s^2 = 1/3
    assert (1 / 3) * (1 / (2 * b) - 0.5) == pytest.approx(nu, rel=1e-12)


def spectral_divergence(u):
    ny, nx = u.shape[1:]
    kx = 2j * math.pi * np.fft.fftfreq(nx)[None, :]
    ky = 2j * math.pi * np.fft.fftfreq(ny)[:, None]
    return np.real(np.fft.ifft2(kx * np.fft.fft2(u[0]) + ky * np.fft.fft2(u[1])))


def test_taylor_green_is_divergence_free_with_the_stated_amplitudes():
    n = 64
    rho, u = wl.taylor_green(n, u0=0.05, mode=2, perturb=1e-3)
    assert rho.shape == (n, n) and u.shape == (2, n, n)
    assert np.abs(spectral_divergence(u)).max() < 1e-14
    assert rho.mean() == pytest.approx(1.0, abs=1e-15)
    # the perturbation alone has max |u'| = perturb
    _, up = wl.taylor_green(n, u0=0.0, perturb=1e-3)
    assert np.sqrt((up ** 2).sum(axis=0)).max() == pytest.approx(1e-3, rel=1e-12)
    # the vortex alone peaks at U0 (x = n / 4, y = 0 for mode 1)
    _, u1 = wl.taylor_green(n, u0=0.05, mode=1, perturb=0.0)
    assert u1[0, 0, n // 4] == pytest.approx(0.05, rel=1e-14)
    assert np.abs(u1).max() == pytest.approx(0.05, rel=1e-14)
    # seeded: same seed, same field; another seed, another perturbation
    assert np.array_equal(u, wl.taylor_green(n, u0=0.05, mode=2, perturb=1e-3)[1])
    assert not np.array_equal(u, wl.taylor_green(n, u0=0.05, mode=2, perturb=1e-3, seed=1)[1])


def test_double_shear_layer():
    n = 128
    rho, u = wl.double_shear_layer(n, u0=0.05, kappa=80.0, eps=0.05)
    # u_x depends on y only and u_y on x only: divergence-free on the grid
    assert np.array_equal(u[0], np.broadcast_to(u[0][:, :1], (n, n)))
    assert np.array_equal(u[1], np.broadcast_to(u[1][:1, :], (n, n)))
    assert np.abs(u[0]).max() <= 0.05 and np.abs(u[0]).max() > 0.049
    assert np.abs(u[1]).max() == pytest.approx(0.05 * 0.05, rel=1e-12)
    # the two layers: u_x < 0 below y = n/4 and above 3n/4, > 0 between
    assert u[0][n // 8, 0] < 0 < u[0][n // 2, 0] and u[0][7 * n // 8, 0] < 0
    assert np.all(rho == 1.0)


def test_random_populations():
    f = wl.random_populations(9, 200, 100, seed=5, amp=0.05, spike_frac=0.1, spike_amp=0.4)
    assert f.shape == (9, 100, 200) and f.flags.c_contiguous
    assert f.min() > 0
    shape = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rel = np.abs(f / shape[:, None, None] - 1).max(axis=0)
    spikes = rel > 0.05 + 1e-12
    assert rel.max() <= 0.4 + 1e-12
    # spikes at about the requested fraction of sites (binomial, 20000 sites)
    assert abs(spikes.mean() - 0.1) < 5 * math.sqrt(0.1 * 0.9 / spikes.size)
    g = wl.random_populations(9, 200, 100, seed=5, amp=0.05, negative_frac=0.05)
    assert (g < 0).any() and ((g < 0).sum(axis=0) <= 1).all()


def test_shock_tube_and_cavity_rest():
    rho, u = wl.shock_tube(800, 400)
    assert rho.shape == (1, 800) and np.all(rho[0, :400] == 1.0) and np.all(rho[0, 400:] == 0.5)
    assert np.all(u == 0)
    rho, u = wl.cavity_rest(100, rho0=2.7)
    assert np.all(rho == 2.7) and np.all(u == 0) and u.shape == (2, 100, 100)


def test_cavity_batch():
    b = wl.cavity_batch(64, sizes=(64, 100), re_range=(2000.0, 7500.0), u0=0.1)
    assert len(b.specs) == 64
    assert b.sites == sum(s.n * s.n for s in b.specs)
    for s in b.specs:
        assert s.n in (64, 100) and 2000.0 <= s.re <= 7500.0
        assert s.nu == pytest.approx(0.1 * s.n / s.re, rel=1e-15)
        assert s.beta == wl.beta_from_nu(s.nu)
        assert 0 <= s.probe[0] < s.n and 0 <= s.probe[1] < s.n
    again = wl.cavity_batch(64, sizes=(64, 100), re_range=(2000.0, 7500.0), u0=0.1)
    assert [(s.n, s.re) for s in again.specs] == [(s.n, s.re) for s in b.specs]
