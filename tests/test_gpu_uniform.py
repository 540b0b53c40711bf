"""GPU: the uniform FV1 plan (every finest cell updated each step, the
comparison of the paper's speed-up figures) against the oracle's
uniform-grid FV1 step, which the oracle suite pins to HWFV1 at eps = 0.

Bar (FP64): h, qx, qy within 1e-10 max-abs after the run (the GPU takes one
reciprocal where the update divides several times, and device square and
cube roots may differ in the last bit), t within 1e-13 relative, mass
within 1e-12 relative.  Sizes from L = 1 (one cell, a partial wave) to
L = 9 (many super-chunks), walls, open edges, inflow, rain and friction."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_utils import compare_leaf_lists, oracle_tie_band

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


def _uniform_run(hw, w, steps, precision="fp64"):
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    plan = hw.Plan([sim.problem], [sim.buffers], uniform=True)
    st = hw.hwfv1_run(sim.problem, sim.buffers, steps, plan=plan)
    plan.close()
    return sim, st


def _oracle_uniform(w, steps):
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    n = 0
    while n < steps and o.scalars()["t"] < w.params["t_end"]:
        o.uniform_fv1_step()
        n += 1
    return o, n


def _cases():
    out = []
    for L in (1, 2, 3, 4):
        out.append((f"bumps_l{L}", lambda L=L: W.dambreak_bumps_l6(L=L), 25))
    out.append(("bumps_l6", lambda: W.dambreak_bumps_l6(), 40))
    out.append(("circular_l8", lambda: W.circular_dambreak_l10(L=8), 30))
    out.append(("hydrograph_l8", lambda: W.hydrograph_l12(L=8), 40))
    out.append(("sheetflow_l7", lambda: W.sheetflow_l13(L=7), 30))
    out.append(("dry_patches_l9", lambda: W.dry_patches(9, 3, inlet=True), 20))
    return out


@pytest.mark.parametrize("name,make,steps", _cases(), ids=[c[0] for c in _cases()])
def test_uniform_plan_matches_oracle(hw, name, make, steps):
    w = make()
    if name.startswith("dry_patches"):
        w.params = dict(w.params, t_end=math.inf)
    log("uniform", name, "L", w.L, "steps", steps)
    sim, st = _uniform_run(hw, w, steps)
    o, n = _oracle_uniform(w, steps)
    so = o.scalars()
    assert st["steps"] == n == so["step"]
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    err = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    log("  max abs", err, "t", st["t"], so["t"])
    assert err <= TOL
    assert st["t"] == pytest.approx(so["t"], rel=1e-13)
    assert st["mass"] == pytest.approx(so["mass"], rel=1e-12, abs=1e-300)
    s = sim.scalars()
    assert s["n_leaves"] == 4 ** w.L
    assert s["leaf_updates"] == n * 4 ** w.L
    sim.close()


def test_uniform_plan_equals_hwfv1_at_eps_zero(hw):
    """With eps = 0 every detail is significant and HWFV1 updates every
    finest cell: the two GPU forms give the same fields bit for bit (the
    mass sum may be ordered differently)."""
    w = W.circular_dambreak_l10(L=9)
    w.params = dict(w.params, eps=0.0)
    a, sa = _uniform_run(hw, w, 30)
    b = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    sb = b.run(30)
    assert sa["steps"] == sb["steps"] == 30 and sa["t"] == sb["t"]
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)
    assert b.scalars()["n_leaves"] == 4 ** w.L
    a.close()
    b.close()


def test_uniform_batch_equals_single_runs(hw):
    ws = [W.dambreak_bumps_l6(L=5), W.hydrograph_l12(L=7), W.sheetflow_l13(L=6),
          W.dry_patches(6, 4)]
    ws[3].params = dict(ws[3].params, t_end=math.inf)
    sims = [hw.Simulation(w.params, w.h, w.qx, w.qy, w.z) for w in ws]
    plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims], uniform=True)
    hw.hwfv1_run_batch(plan, 25)
    plan.close()
    for w, s in zip(ws, sims):
        ref, _ = _uniform_run(hw, w, 25)
        log("  batch", w.name, "t", s.scalars()["t"])
        for x, y in zip(s.export(), ref.export()):
            assert np.array_equal(x, y)
        assert s.scalars()["t"] == ref.scalars()["t"]
        ref.close()
        s.close()


def test_uniform_fp32_bulk_error_against_fp64_oracle(hw):
    w = W.dambreak_bumps_l6()
    sim, st = _uniform_run(hw, w, 40, precision="fp32_bulk")
    o, n = _oracle_uniform(w, 40)
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    err = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    log("  fp32 uniform max abs", err)
    assert st["steps"] == n
    assert err <= 1e-4


def test_circular_dambreak_flat_full_run_matches_oracle(hw):
    """The speed-up workload (flat circular dam break, leaves on many levels)
    over its whole 3.5 s at L = 7: HWFV1 against the oracle's HWFV1 (fields,
    leaf list, time) and the uniform plan against the oracle's uniform FV1."""
    w = W.circular_dambreak_flat(7)
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    st = sim.run(100_000)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    n = o.run(100_000)
    so = o.scalars()
    log("  hwfv1 steps", st["steps"], n, "leaves", so["n_leaves"], "of", 4 ** w.L)
    assert st["steps"] == n and st["t"] == so["t"] == 3.5
    assert 0 < so["n_leaves"] < 4 ** w.L
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    assert max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo)) <= TOL
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    sim.close()
    u, su = _uniform_run(hw, w, 100_000)
    ou, nu = _oracle_uniform(w, 100_000)
    assert su["steps"] == nu and su["t"] == pytest.approx(ou.scalars()["t"], rel=1e-13)
    h, qx, qy = u.export()
    ho, qxo, qyo = ou.fine()
    assert max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo)) <= TOL
    u.close()


def test_pseudo2d_dambreak_matches_oracle(hw):
    """The pseudo-2D dam break of the transient speed-up series to 2.5 s at
    L = 7: HWFV1 and the uniform plan against the oracle."""
    w = W.pseudo2d_dambreak(7, t_end=2.5)
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
    st = sim.run(100_000)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    n = o.run(100_000)
    so = o.scalars()
    log("  pseudo-2D steps", st["steps"], n, "leaves", so["n_leaves"], "of", 4 ** w.L)
    assert st["steps"] == n and st["t"] == so["t"] == 2.5
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    assert max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo)) <= TOL
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    sim.close()
    u, su = _uniform_run(hw, w, 100_000)
    ou, nu = _oracle_uniform(w, 100_000)
    assert su["steps"] == nu
    h, qx, qy = u.export()
    ho, qxo, qyo = ou.fine()
    assert max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo)) <= TOL
    u.close()
