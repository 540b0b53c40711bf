"""The radial reference's own pins: still water stays still (the hoop
source balances the ring-face pressure differences), and the volume on the
rings is conserved while the wave stays inside the outer edge."""
import numpy as np

from radial_reference import radial_dambreak, ring_mass


def test_still_water_stays_still():
    rc, h, q = radial_dambreak(0.7, 0.7, 2.5, 20.0, 400, 1.0)
    assert np.abs(h - 0.7).max() <= 1e-12
    assert np.abs(q).max() <= 1e-12


def test_volume_is_conserved_before_the_edge():
    n, r_max = 800, 30.0
    dr = r_max / n
    rc, h0, _ = radial_dambreak(2.5, 0.5, 2.5, r_max, n, 0.0)
    rc, h, q = radial_dambreak(2.5, 0.5, 2.5, r_max, n, 1.5)
    assert abs(ring_mass(rc, h, dr) - ring_mass(rc, h0, dr)) <= 1e-10 * ring_mass(rc, h0, dr)
    # the front has moved out but not reached the edge
    assert h[rc > 20.0].max() == 0.5 and h[rc < 2.0].max() < 2.5
