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
from parity_utils import compare_leaf_lists, oracle_tie_band

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
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


def _oracle_uniform_to_end(w):
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    while o.scalars()["t"] < w.params["t_end"]:
        o.uniform_fv1_step()
    return o


@pytest.mark.parametrize("t_end", [6.0, 12.0])
def test_humps_dambreak_against_uniform_fv1(hw, t_end):
    """Section 3.1's frictional dam break over the smooth humps: HWFV1
    (L = 8, eps = 1e-3) against the oracle, and its mean absolute depth
    difference from uniform FV1 over the basin at 6 and 12 s, which the
    GPU and the oracle must give alike."""
    w = W.humps_dambreak(t_end=t_end)
    rows = w.meta["basin_rows"]
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    st = sim.run(100_000)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    n = o.run(100_000)
    assert st["steps"] == n and st["t"] == t_end
    hg = sim.export()
    assert max(float(np.abs(a - b).max()) for a, b in zip(hg, o.fine())) <= 1e-10
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    u = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    plan = hw.Plan([u.problem], [u.buffers], uniform=True)
    hw.hwfv1_run(u.problem, u.buffers, 100_000, plan=plan)
    plan.close()
    hu = u.export()[0]
    ou = _oracle_uniform_to_end(w)
    l1_gpu = float(np.abs(hg[0][:rows] - hu[:rows]).mean())
    l1_oracle = float(np.abs(o.fine()[0][:rows] - ou.fine()[0][:rows]).mean())
    print(f"  humps dam break t={t_end}: {n} steps, {st['n_leaves']} leaves, "
          f"L1 depth difference HWFV1 - uniform FV1 {l1_gpu:.3e} m "
          f"(oracle {l1_oracle:.3e})", flush=True)
    sys.stdout.flush()
    assert abs(l1_gpu - l1_oracle) <= 1e-10
    assert l1_gpu <= 5e-3
    sim.close()
    u.close()
