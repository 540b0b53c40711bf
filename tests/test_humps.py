"""Oracle: the lake at rest over the three hump profiles of the Section 3.1
well-balancedness case (70 m x 30 m closed basin, L = 8, eps = 1e-3; hump
shapes chosen to meet Table 3's wetting conditions).  The update balances
the fluxes against the bed-slope terms, so still water stays still: after
the first step (which replaces finest depths under a coarse leaf by the leaf
average) discharges stay at round-off and depths do not move."""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("profile", ["smooth", "steeper", "rectangular"])
def test_humps_lake_at_rest_stays_at_rest(profile):
    w = W.humps_lake_at_rest(profile)
    rows, eta = w.meta["basin_rows"], w.meta["eta"]
    basin_h, basin_z = w.h[:rows], w.z[:rows]
    # Table 3's wetting conditions: dry cells around the highest hump, the
    # free surface at eta wherever it is wet
    assert (basin_h == 0.0).any() and (basin_h > 0.0).mean() > 0.9
    assert np.abs((basin_h + basin_z)[basin_h > 0] - eta).max() <= 1e-12
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    o.step()
    h1, _, _ = o.fine()
    o.run(299)
    h, qx, qy = o.fine()
    assert o.scalars()["step"] == 300
    assert max(np.abs(qx).max(), np.abs(qy).max()) <= 1e-12
    assert np.abs(h - h1).max() <= 1e-12
    # the coarse leaves are wet leaves at the lake level or dry ground
    assert 0 < o.scalars()["n_leaves"] < 4 ** w.L
