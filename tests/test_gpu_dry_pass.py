"""GPU: the dry pass of the FV1 step against a census of the input state.

A leaf may skip the full update when its depth and the depths of its four
in-domain face neighbours are at most h_tol and neither rain nor inflow
reaches it: every flux then vanishes, h stays and the discharges are zero
(Section 2.1.1 with the wet/dry treatment of the FV1 scheme).  When every
leaf is finest, the dry pass finishes an aligned Morton group of 64 cells
(all N cells when N < 64) when all of its cells qualify, and counts those
leaf updates in hw_scalars.dry_stored / dry_skipped.  The census below
recomputes the number of such groups from the seeded input alone, so the
test pins the pass's decision (the encoder's block flags, the edge bits
of the neighbour blocks, the inflow and rain cases) exactly, and the store
history's sequence: with the history on, a group dry at three steps in a
row skips its stores from the third on."""
import sys

import numpy as np
import pytest

import workloads as W
from parity_utils import morton_to_rowmajor

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


def inflow_rate(p, t):
    """Triangular hydrograph of the workload parameters."""
    if not p["q_peak"] > 0.0:
        return 0.0
    if t <= p["t_peak"]:
        return p["q_peak"] * t / p["t_peak"]
    if t <= p["t_base"]:
        return p["q_peak"] * (p["t_base"] - t) / (p["t_base"] - p["t_peak"])
    return 0.0


def dry_census(w, t):
    """Leaf updates the dry pass takes in one step from the input state at
    time t (every leaf finest)."""
    p = w.params
    L = w.L
    n = 1 << L
    if p["rain_rate"] != 0.0:
        return 0
    wet = w.h > p["h_tol"]
    bad = wet.copy()
    bad[:, 1:] |= wet[:, :-1]
    bad[:, :-1] |= wet[:, 1:]
    bad[1:, :] |= wet[:-1, :]
    bad[:-1, :] |= wet[1:, :]
    if inflow_rate(p, t) != 0.0:
        dy = p["dy"]
        for j in range(n):
            lo = max(j * dy, p["inlet_y0"])
            hi = min(j * dy + dy, p["inlet_y1"])
            if hi - lo > 0.0:
                bad[j, 0] = True
    m = bad.ravel()[morton_to_rowmajor(L)]
    g = min(64, n * n)
    return int((~m.reshape(-1, g).any(axis=1)).sum()) * g


def _set_time(hw, sim, t):
    import torch
    torch.cuda.synchronize()
    sc = hw.HwScalars.from_buffer_copy(sim.buffers.scal.cpu().numpy().tobytes())
    sc.t = t
    sim.buffers.scal.copy_(torch.frombuffer(bytearray(bytes(sc)), dtype=torch.uint8))
    torch.cuda.synchronize()


def _dry(s):
    return s["dry_stored"] + s["dry_skipped"]


# L, seed, inlet, rain, wet rectangles, single wet cells
CASES = [(2, 1, False, 0.0, 0, 0), (3, 2, False, 0.0, 0, 1), (4, 3, True, 0.0, 0, 2),
         (5, 4, False, 0.0, 2, 6), (6, 5, True, 0.0, 4, 12), (6, 6, False, 1e-4, 4, 12),
         (8, 7, True, 0.0, 4, 12), (9, 8, False, 0.0, 6, 40)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("L,seed,inlet,rain,nr,ns", CASES)
def test_dry_pass_matches_census(hw, precision, L, seed, inlet, rain, nr, ns):
    w = W.dry_patches(L, seed, n_rect=nr, n_single=ns, inlet=inlet, rain=rain)
    t = 0.5
    expect = dry_census(w, t)
    log("dry pass", w.name, precision, "seed", seed, "inlet", inlet, "rain", rain,
        "expect", expect)
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    _set_time(hw, sim, t)
    sim.run(1)
    s = sim.scalars()
    assert s["n_leaves"] == 4 ** L, "the rough bed must make every leaf finest"
    assert s["dry_skipped"] == 0          # no history before the first step
    assert _dry(s) == expect
    assert expect < 4 ** L or rain == 0.0
    sim.close()


def test_dry_pass_census_in_a_batch(hw):
    """Several problems in one launch: each one's count is its own census."""
    ws = [W.dry_patches(6, 11, inlet=True), W.dry_patches(8, 12), W.dry_patches(5, 13),
          W.dry_patches(4, 14, inlet=True)]
    sims = [hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp64") for w in ws]
    for s in sims:
        _set_time(hw, s, 0.5)
    plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims])
    hw.hwfv1_run_batch(plan, 1)
    for w, s in zip(ws, sims):
        st = s.scalars()
        log("  batch", w.name, "dry", _dry(st), "census", dry_census(w, 0.5))
        assert st["n_leaves"] == 4 ** w.L
        assert _dry(st) == dry_census(w, 0.5)
    plan.close()
    for s in sims:
        s.close()


@pytest.mark.parametrize("L", [4, 7])
@pytest.mark.parametrize("skip", [1, 0])
def test_dry_pass_store_history_sequence(hw, L, skip):
    """An all-dry field: every step is all dry pass; with the history on,
    the first two steps store and the later ones skip (the set being
    written already holds the state), with it off every step stores."""
    w = W.dry_patches(L, 21, n_rect=0, n_single=0)
    w.h[:] = 0.0
    N = 4 ** L
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp64")
    plan = hw.Plan([sim.problem], [sim.buffers], tuning=dict(fv1_write_skip=skip))
    prev = sim.scalars()
    seen = []
    for k in range(4):
        hw.hwfv1_run(sim.problem, sim.buffers, 1, plan=plan)
        s = sim.scalars()
        seen.append((s["dry_stored"] - prev["dry_stored"], s["dry_skipped"] - prev["dry_skipped"]))
        prev = s
    log("  history", L, "skip", skip, seen)
    if skip:
        assert seen == [(N, 0), (N, 0), (0, N), (0, N)]
    else:
        assert seen == [(N, 0)] * 4
    h, qx, qy = sim.export()
    assert not h.any() and not qx.any() and not qy.any()
    plan.close()
    sim.close()
