"""GPU: the block-first leaf list of plans.

A plan's traversal lists the leaves of every aligned 8 x 8 block of finest
leaves first (block by block, ascending Morton order), then the other
leaves in depth-first order, so that the FV1 kernels update a whole block
per wave through the staged block update (with coarser face neighbours
taken from the leaf-level map): hw_tuning.block_list = 2 whenever there is
such a block, the default 1 from 2^19 leaves in them.  The entry points keep the depth-first list
and update every leaf on its own.  Checks, step by step on mixed trees:

* the stored list has exactly that layout: its head holds every whole
  finest block of the depth-first list and nothing else, and the rest is
  the depth-first list without those cells, in order;
* a plan step and the entry-point step (encode, flag, traverse, FV1) give
  the same leaves, fields and scalars bit for bit (FP64 and FP32 bulk; flat
  and bumpy beds; wet, partly dry and with a wet-dry front; with and
  without friction; the dry write history on; the mass, a sum over partial
  records, to 1e-12).
"""
import sys

import numpy as np
import pytest

import workloads as W
from parity_utils import check_block_first

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


def _partly_dry():
    w = W.circular_dambreak_flat(9)
    w.h = np.where(w.h > 1.0, w.h, 0.0)
    return w


CASES = {
    "circular_l9": lambda: W.circular_dambreak_flat(9),
    "circular_dry_l9": _partly_dry,
    # Gaussian bumps, walls
    "bumps_l8": lambda: W.dambreak_bumps_l6(L=8),
    # smooth humps, friction, walls, a wet-dry front
    "humps_dambreak_l8": lambda: W.humps_dambreak(8),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_plan_steps_equal_entry_point_steps(hw, name, precision):
    w = CASES[name]()
    L = w.L
    log(f"[block list] {name} {precision}")
    a = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    b = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    plan = hw.Plan([a.problem], [a.buffers], tuning=dict(fv1_write_skip=1, block_list=2))
    blocks = mixed = 0
    for k in range(40):
        hw.hwfv1_run(a.problem, a.buffers, 1, plan=plan)
        hw.mra_encode(b.problem, b.buffers)
        hw.mra_flag(b.problem, b.buffers)
        hw.mra_traverse_leaves(b.problem, b.buffers)
        hw.fv1_step(b.problem, b.buffers)
        sa, sb = a.scalars(), b.scalars()
        canon = a.buffers.leaf_list()
        stored_b = b.buffers.leaf_list_stored()
        assert np.array_equal(canon, stored_b), k
        if sa["n_leaves"] < 4 ** L:
            mixed += 1
            blocks += check_block_first(L, a.buffers.leaf_list_stored(), canon)
        for x, y in zip(a.export(), b.export()):
            assert np.array_equal(x, y), k
        for key in ("t", "dt", "step", "n_leaves", "maxspeed", "clips"):
            assert sa[key] == sb[key], (k, key)
        # a sum over partial records (the launch shapes may differ)
        assert sa["mass"] == pytest.approx(sb["mass"], rel=1e-12)
    log(f"  mixed steps {mixed}, whole blocks listed {blocks}")
    assert mixed > 0 and blocks > 0
    plan.close()
    a.close()
    b.close()



@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_block_list_modes_agree(hw, precision):
    """hw_tuning.block_list = 2 lists the whole blocks first whenever there
    is one; 1 (the default) only when they hold at least 2^19 leaves, so
    these small problems keep the depth-first list (the emit pass then
    places the counted whole blocks in depth-first order); 0 never counts
    them.  All three plans give the same leaves, fields and scalars bit for
    bit (a batch of two problems, so the interleaved chunk order of the FV1
    kernels covers more than one problem)."""
    ws = [W.circular_dambreak_flat(9), W.dambreak_bumps_l6(L=8)]
    log(f"[block list] modes {precision}")
    runs = []
    for mode in (2, 1, 0):
        sims = [hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision) for w in ws]
        plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims],
                       tuning=dict(block_list=mode))
        hw.hwfv1_run_batch(plan, 30, stats=False)
        for s, w in zip(sims, ws):
            stored = s.buffers.leaf_list_stored()
            canon = s.buffers.leaf_list()
            if mode == 2:
                assert check_block_first(w.L, stored, canon) > 0
            else:
                assert np.array_equal(stored, canon)
        runs.append([(s.export(), s.scalars(), s.buffers.leaf_list()) for s in sims])
        plan.close()
        for s in sims:
            s.close()
    for other in runs[1:]:
        for (ea, sa, la), (eb, sb, lb) in zip(runs[0], other):
            for x, y in zip(ea, eb):
                assert np.array_equal(x, y)
            assert np.array_equal(la, lb)
            for key in ("t", "dt", "step", "n_leaves", "maxspeed", "clips"):
                assert sa[key] == sb[key], key
