"""GPU: the circular dam break (Section 3.2's verification) against the
one-dimensional radial reference (tests/radial_reference.py, 6000 rings
over 30 m).  At t = 1.5 s, before the front meets a wall, the mean absolute
depth difference within 15 m of the dam centre is bounded (bounds a little
above the oracle's 0.0135 m at L = 8 and 0.0073 m at L = 9) and falls by at
least 1.5 per level, the first-order convergence of FV1."""
import sys

import numpy as np
import pytest

import workloads as W
from radial_reference import radial_dambreak

pytestmark = pytest.mark.gpu

BOUND = {8: 0.015, 9: 0.008, 10: 0.0045}


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2206_05761_amd as hw
    return hw


def test_circular_dambreak_converges_to_the_radial_solution(hw):
    rc, hr, _ = radial_dambreak(2.5, 0.5, 2.5, 30.0, 6000, 1.5)
    means = {}
    for L in (8, 9, 10):
        w = W.circular_dambreak_flat(L, 1e-3, t_end=1.5)
        sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
        st = sim.run(100_000)
        assert st["t"] == 1.5
        h = sim.export()[0]
        sim.close()
        c = (np.arange(1 << L) + 0.5) * w.params["dx"]
        x, y = np.meshgrid(c, c)
        r = np.hypot(x - 21.3, y - 20.7)
        inside = r < 15.0
        d = np.abs(h - np.interp(r, rc, hr))[inside]
        means[L] = float(d.mean())
        print(f"  L={L}: {st['steps']} steps, {st['n_leaves']} leaves, mean |h - h_radial| "
              f"{means[L]:.4e} m, max {float(d.max()):.3f} m", flush=True)
        sys.stdout.flush()
        assert means[L] <= BOUND[L]
    assert means[8] / means[9] >= 1.5 and means[9] / means[10] >= 1.5
