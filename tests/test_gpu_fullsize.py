"""GPU parity at full size on the paths that carry the work, through the C
ABI and the captured step graph, against the CPU oracle on the same seeded
inputs (FP64 bar: h, qx, qy within 1e-10 max-abs, leaf lists identical
outside the tie band, t, dt, mass to round-off):

  - every cell wet at L = 12 (16.8 M leaves, each through the full FV1
    update: no leaf is finished by the dry pass);
  - the circular dam break at L = 12 with the tree-sparse finest set of the
    plans (leaves on many levels, span skips of the encoder and copy-down);
  - a wet window of the L = 12 hydrograph (pond, moving front, inflow near
    its peak, dry pass and full update in the same steps);
  - the circular dam break on fractal terrain at L = 10 for all 500 steps.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_utils import check_leaf_list, compare_leaf_lists, oracle_tie_band

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def _max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def _compare(hw, w, sim, o, steps):
    st, so = sim.scalars(), o.scalars()
    assert st["step"] == so["step"] == steps
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    err = (_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    log(f"  {w.name}: {steps} steps, max abs h {err[0]:.3e} qx {err[1]:.3e} "
        f"qy {err[2]:.3e}, leaves {int(so['n_leaves'])} of {4 ** w.L}")
    assert max(err) <= TOL
    leaves = sim.buffers.leaf_list()
    compare_leaf_lists(w.L, leaves, o.leaves(), oracle_tie_band(o), log)
    assert st["t"] == pytest.approx(so["t"], rel=1e-13)
    assert st["dt"] == pytest.approx(so["dt"], rel=1e-10)
    # The oracle adds the leaves' masses one after the other: with N nearly
    # equal terms that sum's rounding error can reach N 2^-53 of the total
    # (the bound of recursive summation); the GPU sums per block.
    assert st["mass"] == pytest.approx(so["mass"], rel=max(1e-12, 4.0 ** w.L * 2.0 ** -53))
    return st, so, leaves


def test_flooded_basin_l12_every_leaf_takes_the_full_update(hw):
    w = W.flooded_basin_l12()
    steps = 5
    log("flooded basin L = 12:", steps, "steps")
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    run = sim.run(steps)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    assert o.run(steps) == steps
    st, so, _ = _compare(hw, w, sim, o, steps)
    # all leaves finest, and none finished by the dry pass
    assert run["leaf_updates"] == steps * 4 ** w.L
    assert run["dry_stored"] == 0 and run["dry_skipped"] == 0
    sim.close()


def test_circular_dambreak_l12_tree_sparse_plan(hw):
    w = W.circular_dambreak_flat(12)
    steps = 40
    log("circular dam break L = 12, tree-sparse plan:", steps, "steps")
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    sim.run(steps)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    assert o.run(steps) == steps
    st, so, leaves = _compare(hw, w, sim, o, steps)
    n = len(leaves)
    assert 0 < n < 4 ** w.L // 16   # coarse leaves cover most of the domain
    sig = O.regularise_flags(w.L, sim.buffers.raw[: hw.n_coarse(w.L)].cpu().numpy())
    check_leaf_list(w.L, leaves, sig)
    sim.close()


def test_hydrograph_l12_wet_window(hw):
    import torch
    w = W.hydrograph_wet_window()
    steps = w.n_steps
    t0 = w.meta["t0"]
    log("hydrograph wet window L = 12 from t =", t0, ":", steps, "steps")
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    sc = hw.HwScalars.from_buffer_copy(sim.buffers.scal.cpu().numpy().tobytes())
    sc.t = t0
    sim.buffers.scal.copy_(torch.frombuffer(bytearray(bytes(sc)), dtype=torch.uint8))
    hw.hw_forget(sim.problem, sim.buffers)
    run = sim.run(steps)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    so0 = o.scalars()
    o.set_time(t0, so0["dt"], 0)
    assert o.run(steps) == steps
    _compare(hw, w, sim, o, steps)
    # both kinds of leaf update took part
    full = run["leaf_updates"] - run["dry_stored"] - run["dry_skipped"]
    log("  full updates", full, "dry pass", run["dry_stored"] + run["dry_skipped"])
    assert full > 0 and run["dry_stored"] + run["dry_skipped"] > 0
    sim.close()


def test_circular_dambreak_l10_all_500_steps(hw):
    w = W.circular_dambreak_l10()
    steps = w.n_steps
    log("circular dam break on fractal terrain L = 10:", steps, "steps")
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    sim.run(steps)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    assert o.run(steps) == steps
    _compare(hw, w, sim, o, steps)
    sim.close()


def test_sheetflow_l13_prefix(hw):
    """The precision-stress workload at its full size (L = 13, 67 M finest
    cells, eps = 1e-4, thin sheet over 500 m of relief, rain, Manning
    0.05): the first 2 steps in FP64 against the oracle, and the FP32-bulk
    form's error against the same oracle state (reported, loosely bounded)."""
    w = W.sheetflow_l13()
    steps = 2
    log("sheet flow L = 13:", steps, "steps")
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    assert o.run(steps) == steps
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    sim.run(steps)
    _compare(hw, w, sim, o, steps)
    sim.close()
    del sim
    s32 = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp32_bulk")
    s32.run(steps)
    f32 = s32.export()
    fo = o.fine()
    l1 = [float(np.mean(np.abs(a - b))) for a, b in zip(f32, fo)]
    linf = [_max_abs(a, b) for a, b in zip(f32, fo)]
    lo, lg = o.leaves(), s32.buffers.leaf_list()
    sym = len(np.setxor1d(lo, lg))
    log(f"  FP32 bulk vs FP64 oracle: L1 h/qx/qy {l1}, Linf {linf}, "
        f"leaf symmetric difference {sym} of {len(lo)}")
    assert l1[0] <= 1e-6 and linf[0] <= 1e-4
    s32.close()
