"""GPU: the phase timing entry point (hw_plan_profile) on HWFV1, uniform
and batched plans.  It runs real steps without the graph, so the state it
leaves is the graphed run's bit for bit; its times are finite and
non-negative, and each single-launch figure (first encoding pass, heavy FV1
kernel) lies within the phase that contains it."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2206_05761_amd as hw
    return hw


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_times(hw, prof, uniform=False):
    keys = hw.PHASES + hw.PROF_KERNELS
    assert set(prof) == set(keys)
    for k in keys:
        assert np.isfinite(prof[k]) and prof[k] >= 0.0, (k, prof[k])
    assert prof["encode_first_pass"] <= prof["encode"] + 1e-3
    assert prof["fv1_heavy"] <= prof["fv1"] + 1e-3
    assert prof["fv1"] > 0.0
    if uniform:
        assert prof["encode"] < 0.05 and prof["traverse"] < 0.05
    else:
        assert prof["encode_first_pass"] > 0.0


def _exported(hw, sim):
    return [t.cpu().numpy() for t in hw.hw_export(sim.problem, sim.buffers)]


@pytest.mark.parametrize("uniform", [False, True])
def test_profile_steps_equal_graphed_steps(hw, uniform):
    w = W.circular_dambreak_flat(8)
    log(f"[profile] circular L=8 uniform={uniform}")
    out = []
    for mode in ("graph", "profile"):
        sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp64")
        plan = hw.Plan([sim.problem], [sim.buffers], uniform=uniform)
        hw.hwfv1_run(sim.problem, sim.buffers, 5, plan=plan)
        if mode == "graph":
            hw.hwfv1_run(sim.problem, sim.buffers, 4, plan=plan)
        else:
            _check_times(hw, hw.hw_plan_profile(plan, 4), uniform)
        out.append((_exported(hw, sim), sim.scalars()))
        plan.close()
        sim.close()
    (fa, sa), (fb, sb) = out
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    assert sa["t"] == sb["t"] and sa["step"] == sb["step"]


def test_profile_batched_plan(hw):
    ws = [W.circular_dambreak_flat(7), W.circular_dambreak_flat(8)]
    log("[profile] batch of two")
    sims = [hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp32_bulk") for w in ws]
    plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims])
    hw.hwfv1_run_batch(plan, 3, stats=False)
    _check_times(hw, hw.hw_plan_profile(plan, 3))
    for s in sims:
        assert s.scalars()["step"] == 6
    plan.close()
    for s in sims:
        s.close()
