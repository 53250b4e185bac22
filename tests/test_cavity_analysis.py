"""CPU checks of the cavity post-processing (stream function, vortex
centres) and of the Table 1 fixture it is compared with."""
import os

import numpy as np
import pytest

from tests.cavity_analysis import load_table, stream_function, vortex_centres

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cavity_vortex_centres.txt")


def test_stream_function_is_exact_for_cubics_at_even_nodes():
    n = 41
    y = np.linspace(0.0, 1.0, n)
    # u_x = 1 - 3y + 2y^3 on every column; psi = y - 1.5 y^2 + 0.5 y^4
    ux = np.repeat((1 - 3 * y + 2 * y ** 3)[:, None], 5, axis=1)
    psi = stream_function(ux)
    exact = (y - 1.5 * y ** 2 + 0.5 * y ** 4)[:, None]
    assert np.abs(psi[0::2] - exact[0::2]).max() < 1e-14
    # odd nodes close with one trapezoid: error <= h^3 max|u''| / 12 + Simpson part
    h = 1.0 / (n - 1)
    assert np.abs(psi[1::2] - exact[1::2]).max() <= h ** 3 * 12.0 / 12.0 + 1e-14
    assert np.all(psi[0] == 0.0)


def test_vortex_centres_of_a_synthetic_field():
    n = 101
    s = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(s, s)          # [j, i]
    sig = 0.03

    def bump(cx, cy, a):
        return a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / sig ** 2)

    def dbump_dy(cx, cy, a):
        return bump(cx, cy, a) * (-2.0 * (Y - cy) / sig ** 2)

    # psi = -sin^2(pi x) sin^2(pi y) + three corner bumps that rise above the
    # wall value psi = 0, as counter-rotating corner vortices do
    psi_exact = -np.sin(np.pi * X) ** 2 * np.sin(np.pi * Y) ** 2
    ux = -np.sin(np.pi * X) ** 2 * 2 * np.pi * np.sin(np.pi * Y) * np.cos(np.pi * Y)
    for cx, cy in ((0.1, 0.1), (0.85, 0.12), (0.07, 0.9)):
        psi_exact = psi_exact + bump(cx, cy, 0.2)
        ux = ux + dbump_dy(cx, cy, 0.2)
    psi = stream_function(ux)
    assert np.abs(psi - psi_exact).max() < 2e-2 * 0.2     # trapezoid closes odd nodes: O(h^2) there
    c = vortex_centres(psi)
    assert c["primary"] == (50, 50)
    assert c["lower_left"] == (10, 10)
    assert c["lower_right"] == (85, 12)
    assert c["top_left"] == (7, 90)


def test_table_fixture_lies_on_the_100_node_grid():
    t = load_table(GOLDEN)
    assert len(t) == 14
    for key, entry in t.items():
        for name, xy in entry.items():
            if xy is None:
                continue
            for v in xy:
                k = v * 99.0
                assert abs(k - round(k)) < 0.01, (key, name, v)
    # the filter does not move the Re = 2000 centres (rows a, b, c, e, f agree)
    rows = [t[(2000.0, r)] for r in "abcef"]
    assert all(r == rows[0] for r in rows)
