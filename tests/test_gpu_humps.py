"""GPU: the lake at rest over the three hump profiles of the Section 3.1
well-balancedness case on the padded 70 m x 30 m basin: 200 steps against
the oracle (fields within 1e-10, identical leaf lists), then the whole
100 s on the GPU with the largest discharge at round-off throughout (the
paper's check of its Fig. 9)."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2206_05761_amd as hw
    return hw


@pytest.mark.parametrize("profile", ["smooth", "steeper", "rectangular"])
def test_humps_lake_at_rest_on_the_gpu(hw, profile):
    w = W.humps_lake_at_rest(profile)
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    st = sim.run(200)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    n = o.run(200)
    assert st["steps"] == n == 200
    err = max(float(np.abs(a - b).max()) for a, b in zip(sim.export(), o.fine()))
    assert err <= 1e-10
    assert np.array_equal(sim.buffers.leaf_list(), o.leaves())
    hist = []
    while sim.scalars()["t"] < w.params["t_end"]:
        sim.run(500)
        h, qx, qy = sim.export()
        hist.append(max(float(np.abs(qx).max()), float(np.abs(qy).max())))
    s = sim.scalars()
    print(f"  {profile}: {s['step']} steps to t={s['t']}, max |q| per 500 steps "
          f"{['%.1e' % v for v in hist]}, {s['n_leaves']} leaves", flush=True)
    sys.stdout.flush()
    assert s["t"] == w.params["t_end"] and s["nonfinite"] == 0
    assert max(hist) <= 1e-10
    sim.close()
