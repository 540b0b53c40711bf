"""GPU: the tree-sparse finest set of plans (encode_skip, fill_skip).

Below a leaf of the previous step's tree every finest cell holds that leaf's
value (the copy-down of the FV1 update), so a wave of the first encoding
pass whose span of 64 * cells finest cells lies inside one leaf loads the
span's first `cells` cells on every lane (encode_skip).  With fill_skip the
copy-down then writes, in each span of 1024 cells below one leaf of level
<= L-5, only the cells that encoding reads; the traversal completes a span
the next tree refines, and every run call ends by completing the current
set.  Checks:

* runs with the skips on and off give the same fields, scalars and leaf
  lists bit for bit (mixed trees, FP64 and FP32 bulk, both encoding tiles,
  a batch), and the same complete current set after a run call and after
  phase profiling; the standalone encoder then agrees too;
* the skips fire and nothing reads a cell they leave out: before a step,
  the cells of spans below one leaf of the previous tree that the next
  encoding does not read are overwritten with different values (with
  encode_skip alone: only spans the next tree covers too, since the FV1
  update reads finest values of its finest leaves).  With both skips the
  coarse values of levels L-4 .. L-2 of those spans are poisoned as well
  (the first encoding pass stores only level L-5 of a tile one leaf
  covers).  The run still equals an untouched one bit for bit, and with
  both skips off it does not.  In the fill_skip case the poisoned spans
  that the next tree refines must be completed by the traversal, and some
  are.
"""
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


MODES = {"both": (1, 1), "encode": (1, 0), "off": (0, 0)}


def _make(hw, w, precision, mode, cells):
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    es, fs = MODES[mode]
    plan = hw.Plan([sim.problem], [sim.buffers],
                   tuning=dict(encode_skip=es, fill_skip=fs, encode_cells_per_thread=cells))
    return sim, plan


def _current(sim):
    import torch
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in sim.buffers.fine[sim.scalars()["cur"]]]


def _same(a, b):
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)
    sa, sb = a.scalars(), b.scalars()
    assert sa == sb
    assert np.array_equal(a.buffers.leaf_list(), b.buffers.leaf_list())


CASES = [("circular_l9", lambda: W.circular_dambreak_flat(9), 60),
         ("pseudo2d_l9", lambda: W.pseudo2d_dambreak(9), 60),
         ("channel_l8", lambda: W.pseudo2d_channel(8), 60),
         ("hydrograph_l8", lambda: W.hydrograph_l12(L=8), 40),
         ("bumps_l6", lambda: W.dambreak_bumps_l6(), 40),
         # flat bed, dry outside the dam: about 9 in 10 cells below dry coarse
         # leaves of level <= L-5 (dry shortcut inside covered spans) ...
         ("circular_dry_l9", lambda: _circular_dry(0.0), 60),
         # ... and the same with rain falling on it (no dry shortcut)
         ("circular_dry_rain_l9", lambda: _circular_dry(1.4e-5), 60),
         # rough beds: every leaf finest, the skips never fire (controls)
         ("sheetflow_l8", lambda: W.sheetflow_l13(L=8), 30),
         ("dry_patches_l9_inlet", lambda: _patches(), 30)]


def _circular_dry(rain):
    w = W.circular_dambreak_flat(9)
    w.h = np.where(w.h > 1.0, w.h, 0.0)
    w.params = dict(w.params, rain_rate=rain)
    return w


def _patches():
    w = W.dry_patches(9, 5, inlet=True, rain=0.0)
    w.params = dict(w.params, t_end=float("inf"))
    return w


@pytest.mark.parametrize("mode", ["both", "encode"])
@pytest.mark.parametrize("cells", [4, 16])
@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("name,make,steps", CASES, ids=[c[0] for c in CASES])
def test_skip_on_equals_skip_off(hw, name, make, steps, precision, cells, mode):
    w = make()
    log("skip", mode, name, precision, "cells", cells, "steps", steps)
    on, pon = _make(hw, w, precision, mode, cells)
    off, poff = _make(hw, w, precision, "off", cells)
    a = hw.hwfv1_run(on.problem, on.buffers, steps, plan=pon)
    b = hw.hwfv1_run(off.problem, off.buffers, steps, plan=poff)
    assert a["steps"] == b["steps"]
    _same(on, off)
    for x, y in zip(_current(on), _current(off)):
        assert np.array_equal(x, y)
    log("  leaves", on.scalars()["n_leaves"], "of", 4 ** w.L)
    for x in (pon, poff):
        x.close()
    on.close()
    off.close()


def test_skip_in_a_batch(hw):
    ws = [W.circular_dambreak_flat(8), W.pseudo2d_dambreak(9), W.hydrograph_l12(L=7),
          W.dambreak_bumps_l6()]
    runs = []
    for skip in (1, 0):
        sims = [hw.Simulation(w.params, w.h, w.qx, w.qy, w.z) for w in ws]
        plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims],
                       tuning=dict(encode_skip=skip, fill_skip=skip, encode_cells_per_thread=4))
        hw.hwfv1_run_batch(plan, 50)
        plan.close()
        runs.append(sims)
    for a, b in zip(*runs):
        _same(a, b)
        for x, y in zip(_current(a), _current(b)):
            assert np.array_equal(x, y)
    for s in runs[0] + runs[1]:
        s.close()


def test_profiling_and_standalone_encoder_after_a_run(hw):
    """Phase profiling ends with a complete current set, and the standalone
    encoder (which reads every finest cell) then gives what it gives after
    a run without the skips."""
    import torch
    w = W.circular_dambreak_flat(9)
    sims = []
    for mode in ("both", "off"):
        sim, plan = _make(hw, w, "fp64", mode, 4)
        hw.hwfv1_run(sim.problem, sim.buffers, 30, plan=plan)
        hw.hw_plan_profile(plan, 7)
        plan.close()
        sims.append(sim)
    a, b = sims
    for x, y in zip(_current(a), _current(b)):
        assert np.array_equal(x, y)
    for s in sims:
        hw.mra_encode(s.problem, s.buffers)
    torch.cuda.synchronize()
    for x, y in zip(a.buffers.coarse, b.buffers.coarse):
        assert torch.equal(x, y)
    _same(a, b)
    for s in sims:
        s.close()


def _spans(leaves, L, span_log4):
    """Spans of 4^span_log4 finest cells that lie inside one leaf."""
    leaves = np.asarray(leaves, dtype=np.int64)
    n = np.floor(np.log2(3 * leaves + 1) / 2).astype(np.int64)
    # guard the float log against a level off by one
    n = np.where((4 ** (n + 1) - 1) // 3 <= leaves, n + 1, n)
    n = np.where((4 ** n - 1) // 3 > leaves, n - 1, n)
    code = leaves - (4 ** n - 1) // 3
    sel = n <= L - span_log4
    S = 4 ** span_log4
    spans = [np.arange((int(c) << (2 * (L - int(m)))) // S,
                       ((int(c) + 1) << (2 * (L - int(m)))) // S)
             for m, c in zip(n[sel], code[sel])]
    return np.concatenate(spans) if spans else np.zeros(0, dtype=np.int64)


def _poison(sim, spans, span_log4, offsets):
    """Overwrite the cells at the given offsets of each span."""
    import torch
    S = 4 ** span_log4
    idx = (spans[:, None] * S + offsets[None, :]).ravel()
    torch.cuda.synchronize()
    if idx.size:
        t = torch.from_numpy(idx).to(sim.buffers.fine[0][0].device)
        cur = sim.buffers.fine[sim.scalars()["cur"]]
        cur[0][t] += 1.0
        cur[1][t] += 0.5
        cur[2][t] -= 0.25
    torch.cuda.synchronize()
    return int(idx.size)


def _poison_coarse(sim, spans, L):
    """Overwrite the coarse values of levels L-4 .. L-2 below each span of
    1024 finest cells (a level L-5 cell)."""
    import torch
    idx = []
    for j in (1, 2, 3):
        n = L - 5 + j
        idx.append(((4 ** n - 1) // 3 + spans[:, None] * 4 ** j
                    + np.arange(4 ** j)[None, :]).ravel())
    idx = np.concatenate(idx)
    torch.cuda.synchronize()
    if idx.size:
        t = torch.from_numpy(idx).to(sim.buffers.coarse[0].device)
        for v, d in enumerate((2.0, -1.0, 0.75)):
            sim.buffers.coarse[v][t] += d
    torch.cuda.synchronize()
    return int(idx.size)


@pytest.mark.parametrize("dry", [False, True])
@pytest.mark.parametrize("mode", ["encode", "both"])
@pytest.mark.parametrize("cells", [4, 16])
def test_skipped_cells_are_read_by_nobody(hw, cells, mode, dry):
    w = _circular_dry(0.0) if dry else W.circular_dambreak_flat(9)
    L = w.L
    if mode == "both":
        # spans of 1024 cells below a leaf of level <= L-5; the encoder reads
        # the first `cells` cells of each run of 64 * cells
        k = 5
        off = np.arange(1024)
        offsets = off[(off % (64 * cells)) >= cells]
    else:
        k = 4 if cells == 4 else 5
        offsets = np.arange(cells, 4 ** k)
    ref, pref = _make(hw, w, "fp64", "off", cells)
    on, pon = _make(hw, w, "fp64", mode, cells)
    off_, poff = _make(hw, w, "fp64", "off", cells)
    poisoned = refined = 0
    for step in range(60):
        hw.hwfv1_run(ref.problem, ref.buffers, 1, plan=pref)
        if step >= 2:
            prev = _spans(on.buffers.leaf_list(), L, k)
            nxt = _spans(ref.buffers.leaf_list(), L, k)
            sp = prev if mode == "both" else np.intersect1d(prev, nxt)
            refined += int(np.setdiff1d(prev, nxt).size)
            poisoned += _poison(on, sp, k, offsets)
            _poison(off_, sp, k, offsets)
            if mode == "both":
                poisoned += _poison_coarse(on, sp, L)
                _poison_coarse(off_, sp, L)
        for sim, plan in ((on, pon), (off_, poff)):
            hw.hwfv1_run(sim.problem, sim.buffers, 1, plan=plan)
    log("  poisoned cells", poisoned, "spans refined by the next tree", refined,
        "cells/thread", cells, mode)
    assert poisoned > 0
    if mode == "both":
        assert refined > 0
    _same(on, ref)
    assert any(not np.array_equal(x, y) for x, y in zip(off_.export(), ref.export()))
    for x in (pref, pon, poff):
        x.close()
    for s in (ref, on, off_):
        s.close()


def test_skips_at_full_size_l12(hw):
    """The circular dam break of the speed-up series at L = 12 (16.8 M
    finest cells, most of them below coarse leaves), in the plan shape the
    benchmark times: 400 steps with the skips on and off, bit for bit."""
    w = W.circular_dambreak_flat(12)
    on, pon = _make(hw, w, "fp64", "both", 4)
    off, poff = _make(hw, w, "fp64", "off", 4)
    a = hw.hwfv1_run(on.problem, on.buffers, 400, plan=pon)
    b = hw.hwfv1_run(off.problem, off.buffers, 400, plan=poff)
    assert a["steps"] == b["steps"] == 400
    log("  L=12:", on.scalars()["n_leaves"], "leaves of", 4 ** 12)
    assert 0 < on.scalars()["n_leaves"] < 4 ** 12 // 4
    _same(on, off)
    for x in (pon, poff):
        x.close()
    on.close()
    off.close()
