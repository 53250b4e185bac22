"""Pins of the oracle's median entropy filter step (Sec. 3.5; cavity stencils
of Sec. 4.4), independent of the oracle's own stencil and decision code: the
medians are recomputed with np.roll / np.median from the recorded Delta S'
(itself recomputed from the input state), the FLOOR and GATE decisions are
taken again, and every filtered node is checked to land on its target on the
populations that came out of the step.  `median_pins` holds the checks."""
import pytest

import median_pins as mp


@pytest.mark.parametrize("delta", [0.0, 3e-4, 2e-3])
@pytest.mark.parametrize("mode", [mp.FLOOR, mp.GATE])
@pytest.mark.parametrize("form", [mp.QUAD, mp.EXACT])
def test_periodic_median_step(orc, form, mode, delta):
    mp.check_periodic_2d(orc, form, mode, delta, homothety=1 if form == mp.EXACT else 0)


@pytest.mark.parametrize("mode", [mp.FLOOR, mp.GATE])
def test_periodic_median_step_entropic_sqrt_homothety(orc, mode):
    """Entropic f*, exact Delta S, the homothety factor sqrt(t / Delta S')."""
    mp.check_periodic_2d(orc, mp.EXACT, mode, 1e-4, qe=mp.ENTROPIC, homothety=0, seed=29)


@pytest.mark.parametrize("delta", [0.0, 3e-4])
@pytest.mark.parametrize("mode", [mp.FLOOR, mp.GATE])
@pytest.mark.parametrize("form", [mp.QUAD, mp.EXACT])
def test_cavity_near_wall_stencils(orc, form, mode, delta):
    mp.check_cavity(orc, form, mode, delta)


@pytest.mark.parametrize("mode", [mp.FLOOR, mp.GATE])
@pytest.mark.parametrize("bc", [mp.PERIODIC, mp.TUBE])
def test_d1q3_three_point_median(orc, bc, mode):
    mp.check_d1q3(orc, bc, mp.QUAD, mode, 2e-4)
    mp.check_d1q3(orc, bc, mp.EXACT, mode, 2e-4, qe=mp.ENTROPIC)


@pytest.mark.parametrize("shift", [(5, -7), (1, 23), (-1, 0), (0, 1), (19, 12)])
@pytest.mark.parametrize("mode", [mp.FLOOR, mp.GATE])
@pytest.mark.parametrize("form", [mp.QUAD, mp.EXACT])
def test_translation_across_the_seams(orc, form, mode, shift):
    mp.check_translation(orc, form, mode, shift)
