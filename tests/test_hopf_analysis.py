"""Pins of the Hopf post-processing (Sec. 4.4.2) on signals with known
answers: the energy of eq. (energy) of a sinusoid, the x-intercept of a
linear E_u^2(Re) branch, and the frequency of a sampled oscillation."""
import math

import numpy as np
import pytest

from paper_0704_0043_amd import hopf


@pytest.mark.parametrize("amp,periods", [(1e-3, 7), (0.02, 40)])
def test_energy_of_a_sinusoid(amp, periods):
    """sum (A sin)^2 over whole periods is N A^2 / 2, so
    E_u = A sqrt(L / (2 u0)) whatever the number of samples"""
    n_samp, length, u0 = 50000, 100.0, 0.1
    t = np.arange(n_samp)
    u = 0.03 + amp * np.sin(2 * math.pi * periods * t / n_samp)
    assert hopf.energy(u, length, u0) == pytest.approx(amp * math.sqrt(length / (2 * u0)), rel=1e-9)
    assert hopf.energy(np.full(1000, 0.05), length, u0) == pytest.approx(0.0, abs=1e-12)


def test_critical_reynolds_of_a_linear_branch():
    re = np.arange(6000.0, 9001.0, 250.0)
    rc, s = 7135.0, 2e-6
    e2 = np.where(re > rc, s * (re - rc), 0.0) + 1e-12 * np.cos(re)
    got, slope, used = hopf.critical_reynolds(re, e2)
    assert got == pytest.approx(rc, abs=1.0)
    assert slope == pytest.approx(s, rel=1e-3)
    assert min(used) > rc
    assert math.isnan(hopf.critical_reynolds(re, np.zeros_like(re))[0])


def test_dominant_frequency():
    length, u0 = 100.0, 0.1
    dt = u0 / length
    n_samp = 50000                       # 50 time units
    t = np.arange(n_samp) * dt
    for f in (0.525, 0.3):
        u = 0.01 * np.sin(2 * math.pi * f * t + 0.3) + 0.002 * np.sin(2 * math.pi * 2.7 * f * t)
        got = hopf.dominant_frequency(u, length, u0)
        assert got == pytest.approx(f, abs=1.0 / (n_samp * dt))


def test_probe_node():
    assert hopf.probe_node(100) == (6, 80)
    assert hopf.probe_node(17) == (1, 13)


def test_onset_bracket():
    re = [6000.0, 6250.0, 6300.0, 6350.0, 6500.0]
    e2 = [7e-8, 7.6e-8, 8e-8, 9e-4, 1e-3]
    assert hopf.onset(re, e2) == (6300.0, 6350.0)
    lo, hi = hopf.onset(re, [0.0] * 5)
    assert math.isnan(lo) and math.isnan(hi)
