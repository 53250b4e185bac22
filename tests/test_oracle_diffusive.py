"""Pins of the oracle's diffusive Maxwell walls (Sec. 4.4.2).

The checks follow from the paper's description of the boundary: what a wall
node sends into the fluid carries exactly the mass that arrived there from
the fluid, distributed as the quasiequilibrium of the wall's velocity (the
quasiequilibria themselves are pinned in test_oracle_pins.py); corners
reflect; a fluid at rest in equilibrium with resting walls stays at rest; the
total mass changes only by what is in transit through the walls; and the
steady cavity flow agrees with the bounce-back cavity to within a node.
"""
import numpy as np
import pytest

from paper_0704_0043_amd import workloads as wl
from tests.cavity_analysis import stream_function, vortex_centres

D2Q9 = 2
CAV, DIFF = 1, 3
VX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
VY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def boundary_nodes(nx, ny):
    """(x, y, inward normal, wall velocity) of every non-corner boundary node"""
    out = []
    for x in range(1, nx - 1):
        out.append((x, 0, (0, 1), 0.0))
        out.append((x, ny - 1, (0, -1), None))   # lid
    for y in range(1, ny - 1):
        out.append((0, y, (1, 0), 0.0))
        out.append((nx - 1, y, (-1, 0), 0.0))
    return out


def params(orc, nx, ny, qe, lid, **kw):
    return orc.make_params(lattice=D2Q9, nx=nx, ny=ny, beta=0.9, qe=qe, bc=DIFF, lid_ux=lid, **kw)


@pytest.mark.parametrize("qe", [0, 1])
@pytest.mark.parametrize("rho0", [1.0, 1.3])
def test_rest_state_is_stationary(orc, qe, rho0):
    nx, ny = 23, 19
    p = params(orc, nx, ny, qe, 0.0)
    rho, u = wl.cavity_rest(nx, ny, rho0=rho0)
    f0 = orc.init_equilibrium(p, rho, u)
    f = f0.copy()
    orc.step(p, f, 40)
    assert np.abs(f - f0).max() <= 1e-14 * rho0


@pytest.mark.parametrize("qe", [0, 1])
def test_wall_sends_back_the_arrived_mass_as_wall_equilibrium(orc, qe):
    nx, ny, lid = 21, 17, 0.08
    p = params(orc, nx, ny, qe, lid)
    f0 = wl.random_populations(9, nx, ny, seed=71, amp=0.05)
    f1 = f0.copy()
    orc.step(p, f1, 1)
    for x, y, (mx, my), uw in boundary_nodes(nx, ny):
        uw = lid if uw is None else uw
        arrived = sum(f0[i, y, x] for i in range(9) if VX[i] * mx + VY[i] * my < 0)
        inward = [i for i in range(9) if VX[i] * mx + VY[i] * my > 0]
        sent = np.array([f1[i, y + VY[i], x + VX[i]] for i in inward])
        assert sent.sum() == pytest.approx(arrived, rel=1e-14)
        fs = orc.equilibrium(D2Q9, qe, 1.0, uw, 0.0)[inward]
        np.testing.assert_allclose(sent / sent.sum(), fs / fs.sum(), rtol=1e-13)


def test_corners_reflect_every_population(orc):
    nx, ny = 12, 10
    p = params(orc, nx, ny, 1, 0.1)
    f0 = wl.random_populations(9, nx, ny, seed=72, amp=0.05)
    f1 = f0.copy()
    orc.step(p, f1, 1)
    for cx, cy in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
        for i in range(1, 9):
            tx, ty = cx + VX[i], cy + VY[i]
            if 0 <= tx < nx and 0 <= ty < ny:
                # what leaves the corner along v_i is what arrived along -v_i
                assert f1[i, ty, tx] == f0[OPP[i], cy, cx]


def test_boundary_nodes_do_not_collide(orc):
    nx, ny = 14, 11
    p = params(orc, nx, ny, 0, 0.1)
    f = wl.random_populations(9, nx, ny, seed=73, amp=0.05)
    st, mask, _ = orc.step(p, f, 1, record=True)
    assert st.n_fluid == (nx - 2) * (ny - 2)
    edge = np.ones((ny, nx), dtype=bool)
    edge[1:-1, 1:-1] = False
    assert np.all((mask[edge] & 8) != 0) and np.all((mask[~edge] & 8) == 0)


def test_mass_changes_only_by_what_is_in_transit(orc):
    """Free flight carries what a wall node received from the fluid off the
    grid and back into the node's inward slots, which the wall rule then
    replaces by the same mass: M(t+1) - M(t) = A(t) - A(t-1), with A the mass
    that arrived at the non-corner boundary nodes from the fluid."""
    nx, ny = 16, 13
    p = params(orc, nx, ny, 1, 0.1, limiter=2, delta_median=1e-4)
    f = wl.random_populations(9, nx, ny, seed=74, amp=0.05)

    def arrived(g):
        return sum(g[i, y, x] for x, y, (mx, my), _ in boundary_nodes(nx, ny)
                   for i in range(9) if VX[i] * mx + VY[i] * my < 0)

    hist = [(f.sum(), arrived(f))]
    for _ in range(30):
        orc.step(p, f, 1)
        hist.append((f.sum(), arrived(f)))
    for t in range(1, len(hist) - 1):
        dm = hist[t + 1][0] - hist[t][0]
        da = hist[t][1] - hist[t - 1][1]
        assert dm == pytest.approx(da, abs=1e-13 * hist[0][0])


def test_steady_cavity_matches_bounce_back_cavity(orc):
    """Re = 100 on 41 x 41 nodes: the primary vortex of the diffusive cavity
    sits within one node of the bounce-back cavity's (both walls are no-slip
    to first order; they differ in how they reach it)."""
    n, u0, re = 41, 0.1, 100.0
    beta = wl.beta_from_nu(u0 * n / re)
    centres = {}
    for bc in (CAV, DIFF):
        p = orc.make_params(lattice=D2Q9, nx=n, ny=n, beta=beta, qe=1, bc=bc, lid_ux=u0, rho0=1.0)
        rho, u = wl.cavity_rest(n, n, rho0=1.0)
        f = orc.init_equilibrium(p, rho, u)
        orc.step(p, f, 6000)
        _, ux, _ = orc.moments(D2Q9, f)
        centres[bc] = vortex_centres(stream_function(ux))["primary"]
    (xa, ya), (xb, yb) = centres[CAV], centres[DIFF]
    assert abs(xa - xb) <= 1 and abs(ya - yb) <= 1, centres
    # the primary vortex sits in the upper half, right of the centre at Re = 100
    assert xb > n // 2 and yb > n // 2
