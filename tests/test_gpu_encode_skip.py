"""GPU: the encoder's span skip (plans with encode_skip = 1).

Below a leaf of the previous step's tree every finest cell holds that leaf's
value (the copy-down of the FV1 update), so a wave of the first encoding
pass whose span of 64 * cells finest cells lies inside one leaf loads the
span's first `cells` cells on every lane.  Two checks:

* runs with the skip on and off give the same fields, scalars and leaf
  lists bit for bit (mixed trees, FP64 and FP32 bulk, both encoding tiles,
  a batch);
* the skip fires and the encoder reads nothing but the span's first cells:
  before a step, every later cell of each span that lies inside one leaf of
  the previous tree and inside one leaf of the tree the step will use (an
  untouched run gives it) is overwritten with different values.  Those
  cells are then read by nobody but the encoder (the FV1 update reads
  finest values only for leaves on the two finest levels, and replaces
  speculative neighbour loads below a coarser leaf by the leaf's value), so
  with the skip on the run still equals the untouched one bit for bit, and
  with the skip off it does not."""
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


def _make(hw, w, precision, skip, cells):
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    plan = hw.Plan([sim.problem], [sim.buffers],
                   tuning=dict(encode_skip=skip, encode_cells_per_thread=cells))
    return sim, plan


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
         ("bumps_l6", lambda: W.dambreak_bumps_l6(), 40)]


@pytest.mark.parametrize("cells", [4, 16])
@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("name,make,steps", CASES, ids=[c[0] for c in CASES])
def test_skip_on_equals_skip_off(hw, name, make, steps, precision, cells):
    w = make()
    log("encode skip", name, precision, "cells", cells, "steps", steps)
    on, pon = _make(hw, w, precision, 1, cells)
    off, poff = _make(hw, w, precision, 0, cells)
    a = hw.hwfv1_run(on.problem, on.buffers, steps, plan=pon)
    b = hw.hwfv1_run(off.problem, off.buffers, steps, plan=poff)
    assert a["steps"] == b["steps"]
    _same(on, off)
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
                       tuning=dict(encode_skip=skip, encode_cells_per_thread=4))
        hw.hwfv1_run_batch(plan, 50)
        plan.close()
        runs.append(sims)
    for a, b in zip(*runs):
        _same(a, b)
    for s in runs[0] + runs[1]:
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


def _poison(sim, spans, span_log4, cells):
    import torch
    S = 4 ** span_log4
    idx = (spans[:, None] * S + np.arange(cells, S)[None, :]).ravel()
    torch.cuda.synchronize()
    if idx.size:
        t = torch.from_numpy(idx).to(sim.buffers.fine[0][0].device)
        cur = sim.buffers.fine[sim.scalars()["cur"]]
        cur[0][t] += 1.0
        cur[1][t] += 0.5
        cur[2][t] -= 0.25
    torch.cuda.synchronize()
    return int(idx.size)


@pytest.mark.parametrize("cells", [4, 16])
def test_skip_reads_only_the_span_first_cells(hw, cells):
    w = W.circular_dambreak_flat(9)
    L = w.L
    k = 4 if cells == 4 else 5
    ref, pref = _make(hw, w, "fp64", 1, cells)
    on, pon = _make(hw, w, "fp64", 1, cells)
    off, poff = _make(hw, w, "fp64", 0, cells)
    poisoned = 0
    for step in range(25):
        hw.hwfv1_run(ref.problem, ref.buffers, 1, plan=pref)
        if step >= 2:
            sp = np.intersect1d(_spans(on.buffers.leaf_list(), L, k),
                                _spans(ref.buffers.leaf_list(), L, k))
            poisoned += _poison(on, sp, k, cells)
            _poison(off, sp, k, cells)
        for sim, plan in ((on, pon), (off, poff)):
            hw.hwfv1_run(sim.problem, sim.buffers, 1, plan=plan)
    log("  poisoned cells over the run", poisoned, "cells/thread", cells)
    assert poisoned > 0
    _same(on, ref)
    assert any(not np.array_equal(x, y) for x, y in zip(off.export(), ref.export()))
    for x in (pref, pon, poff):
        x.close()
    for s in (ref, on, off):
        s.close()
