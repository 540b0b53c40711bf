"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle
on the same seeded inputs.

Bar (FP64): bit-identical bed hierarchy, encoding, details, flags and leaf
lists (the encoding uses only sums and exact scalings by 1/4); finest h, qx,
qy within 1e-10 max-abs after the run (device and host square root and
cube root may differ in the last bit).  Cells within 1e-12 of the
significance threshold would be reported as ties; none is expected."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_utils import (check_leaf_list, compare_leaf_lists, morton_to_rowmajor,
                          oracle_tie_band)

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


def _to_np(t):
    return t.detach().cpu().numpy()


def _sim(hw, w, precision="fp64", params=None):
    return hw.Simulation(params or w.params, w.h, w.qx, w.qy, w.z, precision=precision)


def _max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


# ----------------------------------------------------------------------------
# ingest: Morton permutation, bed hierarchy, bed flags, first timestep
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("L", [1, 2, 3, 6])
def test_ingest_matches_oracle(hw, L):
    w = W.dambreak_bumps_l6(L=L) if L > 1 else W.lake_at_rest(1, 0.8, 3, 1e-3)
    log("ingest", w.name)
    sim = _sim(hw, w)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    h, qx, qy = sim.export()
    assert np.array_equal(h, w.h) and np.array_equal(qx, w.qx) and np.array_equal(qy, w.qy)
    r = morton_to_rowmajor(L)
    assert np.array_equal(_to_np(sim.buffers.fine[0][0])[: 4 ** L], w.h.ravel()[r])
    assert np.array_equal(_to_np(sim.buffers.zhier), o.hierarchy("z"))
    assert np.array_equal(_to_np(sim.buffers.zsig)[: len(o.flags("zraw"))], o.flags("zraw"))
    s, so = sim.scalars(), o.scalars()
    assert s["dt"] == so["dt"]
    assert s["smax"][3] == so["smax_z"]
    assert s["mass0"] == pytest.approx(so["mass"], rel=1e-13)
    assert s["cur"] == 0 and s["step"] == 0 and s["done"] == 0


# ----------------------------------------------------------------------------
# phase by phase against the oracle's phases
# ----------------------------------------------------------------------------
def _load_oracle_state(hw, sim, o, z):
    """Put the oracle's current state (fields, t, dt, step) into the GPU
    buffers, so that the next phases start from identical inputs."""
    import torch
    ho, qxo, qyo = o.fine()
    dev = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")
           for a in (ho, qxo, qyo, z)]
    hw.hw_ingest(sim.problem, sim.buffers, *dev)
    torch.cuda.synchronize()
    so = o.scalars()
    sc = hw.HwScalars.from_buffer_copy(sim.buffers.scal.cpu().numpy().tobytes())
    sc.t, sc.dt, sc.step = so["t"], so["dt"], int(so["step"])
    sim.buffers.scal.copy_(torch.frombuffer(bytearray(bytes(sc)), dtype=torch.uint8))
    torch.cuda.synchronize()


def _phase_case(hw, w, steps):
    """Each step starts both sides from the oracle's state: encoding, flags,
    regularisation and the leaf list must then agree exactly, the FV1 update
    within the FP64 bar (the GPU takes one reciprocal where the definition
    divides several times)."""
    import torch
    sim = _sim(hw, w)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    p, b = sim.problem, sim.buffers
    L = w.L
    nc = hw.n_coarse(L)
    det = torch.zeros(9 * max(nc, 1), dtype=torch.float64, device="cuda")
    for k in range(steps):
        log(w.name, "phase step", k)
        if k > 0:
            _load_oracle_state(hw, sim, o, w.z)
        hw.mra_encode(p, b, det)
        o.phase_encode()
        torch.cuda.synchronize()
        for v, name in enumerate(("h", "qx", "qy")):
            assert np.array_equal(_to_np(b.coarse[v])[:nc], o.hierarchy(name)[:nc]), name
            dg = _to_np(det)[v * 3 * nc:(v + 1) * 3 * nc].reshape(3, nc)
            assert np.array_equal(dg, o.details(name)), name
        raw_enc = _to_np(b.raw)[:nc].copy()
        assert np.array_equal(raw_enc, o.flags("raw"))
        hw.mra_flag(p, b)
        o.phase_regularise()
        torch.cuda.synchronize()
        assert np.array_equal(_to_np(b.raw)[:nc], raw_enc)
        sig = _to_np(b.sig)[:nc]
        assert np.array_equal(sig, o.flags("sig"))
        hw.mra_traverse_leaves(p, b)
        o.phase_traverse()
        leaves = b.leaf_list()
        compare_leaf_lists(L, leaves, o.leaves(), oracle_tie_band(o), log)
        check_leaf_list(L, leaves, sig)
        hw.fv1_step(p, b)
        o.phase_fv1()
        h, qx, qy = sim.export()
        ho, qxo, qyo = o.fine()
        err = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
        log("  max abs", err, "bitwise", np.array_equal(h, ho) and np.array_equal(qx, qxo))
        assert err <= TOL
        s, so = sim.scalars(), o.scalars()
        assert s["step"] == so["step"] and s["n_leaves"] == so["n_leaves"]
        assert s["t"] == pytest.approx(so["t"], rel=1e-14)
        assert s["dt"] == pytest.approx(so["dt"], rel=1e-12)
        assert s["mass"] == pytest.approx(so["mass"], rel=1e-12)


def test_phases_dambreak_bumps_l6(hw):
    _phase_case(hw, W.dambreak_bumps_l6(), 6)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 7])
def test_phases_small_and_ragged_levels(hw, L):
    """Levels below one encoding tile / traversal workgroup, leaf counts that
    are not multiples of a workgroup, coarse leaves above the traversal
    groups (copy-down by the fill kernel)."""
    w = W.dambreak_bumps_l6(L=L, seed=L + 10)
    p = dict(w.params, eps=5e-3, t_end=math.inf)
    w.params = p
    _phase_case(hw, w, 4)


# ----------------------------------------------------------------------------
# whole runs through hwfv1_run (captured graph)
# ----------------------------------------------------------------------------
def _run_case(hw, w, steps, precision="fp64"):
    log("run", w.name, "steps", steps, precision)
    sim = _sim(hw, w, precision)
    st = sim.run(steps)
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    n = o.run(steps)
    return sim, st, o, n


def test_run_dambreak_bumps_l6_to_t_end(hw):
    w = W.dambreak_bumps_l6()
    sim, st, o, n = _run_case(hw, w, 10_000)
    so = o.scalars()
    assert st["steps"] == n == so["step"]
    assert st["t"] == so["t"] == 0.05
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    err = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    log("  max abs", err)
    assert err <= TOL
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    assert st["mass"] == pytest.approx(so["mass"], rel=1e-12)


def test_run_circular_dambreak_l10(hw):
    w = W.circular_dambreak_l10()
    sim, st, o, n = _run_case(hw, w, 20)
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    err = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    log("  max abs", err)
    assert err <= TOL
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    assert st["t"] == pytest.approx(o.scalars()["t"], rel=1e-13)


def test_run_hydrograph_l12_prefix(hw):
    """Full-size hydrograph workload (L = 12, the benchmark configuration):
    the first 3 steps element by element (inflow starts on step 2)."""
    w = W.hydrograph_l12()
    sim, st, o, n = _run_case(hw, w, 3)
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    err = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    log("  max abs", err, "mass", st["mass"], o.scalars()["mass"])
    assert err <= TOL
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)
    assert st["mass"] == pytest.approx(o.scalars()["mass"], rel=1e-12)


def test_run_hydrograph_l12_full_length_properties(hw):
    """All 2000 steps of the benchmark run: properties that hold at any
    size (finite, non-negative depth, valid leaf list, stored volume no more
    than the hydrograph volume delivered so far)."""
    w = W.hydrograph_l12()
    sim = _sim(hw, w)
    st = sim.run(w.n_steps)
    assert st["steps"] == w.n_steps
    s = sim.scalars()
    assert s["nonfinite"] == 0
    h, qx, qy = (_to_np(t) for t in sim.buffers.current_fine())
    assert np.all(np.isfinite(h)) and np.all(h >= 0.0)
    assert np.all(np.isfinite(qx)) and np.all(np.isfinite(qy))
    # the step's raw flags regularised by the oracle (not the kernel's sig)
    sig = O.regularise_flags(w.L, _to_np(sim.buffers.raw))
    check_leaf_list(w.L, sim.buffers.leaf_list(), sig)
    t = s["t"]
    qp, tp = w.params["q_peak"], w.params["t_peak"]
    delivered = 0.5 * qp * t * t / tp if t <= tp else None
    log("  t", t, "mass", s["mass"], "delivered", delivered, "leaves", s["n_leaves"])
    if delivered is not None:
        assert s["mass"] <= delivered * (1.0 + 1e-6) + 1e-9


def test_run_sheetflow_rain_small(hw):
    """Rain, Manning friction and open boundaries over steep terrain (the
    thin-sheet workload at L = 7)."""
    w = W.sheetflow_l13(L=7)
    sim, st, o, n = _run_case(hw, w, 50)
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    err = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    log("  max abs", err)
    assert err <= TOL
    compare_leaf_lists(w.L, sim.buffers.leaf_list(), o.leaves(), oracle_tie_band(o), log)


def test_nonfinite_input_is_reported(hw):
    w = W.dambreak_bumps_l6(L=4)
    h = w.h.copy()
    h[3, 3] = np.nan
    sim = hw.Simulation(w.params, h, w.qx, w.qy, w.z)
    assert sim.scalars()["nonfinite"] == 2
    with pytest.raises(hw.HwError) as e:
        sim.run(2)
    assert e.value.code == hw.HW_ENONFINITE


# ----------------------------------------------------------------------------
# FP32-bulk and batched forms
# ----------------------------------------------------------------------------
def test_fp32_bulk_error_against_fp64_oracle(hw):
    w = W.dambreak_bumps_l6()
    sim, st, o, n = _run_case(hw, w, 10_000, precision="fp32_bulk")
    h, qx, qy = sim.export()
    ho, qxo, qyo = o.fine()
    l1 = np.mean(np.abs(h - ho))
    linf = max(_max_abs(h, ho), _max_abs(qx, qxo), _max_abs(qy, qyo))
    lo, lg = set(o.leaves().tolist()), set(sim.buffers.leaf_list().tolist())
    log("  fp32 L1(h)", l1, "Linf", linf, "leaf symdiff", len(lo ^ lg),
        "mass rel", (st["mass"] - o.scalars()["mass"]) / o.scalars()["mass"])
    assert l1 <= 1e-4 and linf <= 1e-2


def test_batch_equals_individual_runs(hw):
    """Problems of different L and eps in one plan evolve exactly as when
    each runs alone."""
    ws = [W.dambreak_bumps_l6(L=5, seed=21), W.dambreak_bumps_l6(L=4, seed=23),
          W.circular_dambreak_l10(L=7), W.dambreak_bumps_l6(L=3, seed=22),
          W.sheetflow_l13(L=6)]
    ws[0].params = dict(ws[0].params, t_end=math.inf, eps=1e-2)
    ws[1].params = dict(ws[1].params, t_end=0.01)   # finishes after a few steps
    ws[3].params = dict(ws[3].params, t_end=math.inf, eps=1e-4)
    steps = 25
    sims = [_sim(hw, w) for w in ws]
    plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims])
    stats = hw.hwfv1_run_batch(plan, steps)
    for i, (w, s, st) in enumerate(zip(ws, sims, stats)):
        ref = _sim(hw, w)
        ref.run(steps)
        a, b = s.export(), ref.export()
        log("  batch", w.name, "steps", st["steps"], "leaves", s.scalars()["n_leaves"],
            "of", 4 ** w.L)
        if i == 1:
            # reached t_end early; the other problems kept stepping
            assert 0 < st["steps"] < steps and abs(s.scalars()["t"] - 0.01) <= 1e-15
            assert st["steps"] == ref.scalars()["step"]
        else:
            assert st["steps"] == steps
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert np.array_equal(s.buffers.leaf_list(), ref.buffers.leaf_list())
        assert s.scalars()["t"] == ref.scalars()["t"]
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_launch_shapes_do_not_change_results(hw, precision):
    """Every encode tile size, FV1 grid and the FV1 store skip give the
    same state, bit for bit (the launch shape only reorders independent
    work; the mass sum may differ in the last bits)."""
    w = W.circular_dambreak_l10(L=9)
    ref = None
    for tu in ({}, dict(encode_cells_per_thread=16, fv1_grid=8),
               dict(encode_cells_per_thread=4, fv1_grid=4096, fv1_write_skip=0),
               dict(encode_cells_per_thread=16, fv1_grid=512),
               # the FP32 first pass with 1, 2 and 4 tiles per workgroup
               dict(encode_skip=0, fill_skip=0, encode_tiles=1),
               dict(encode_skip=0, fill_skip=0, encode_tiles=2),
               dict(encode_skip=0, fill_skip=0, encode_tiles=4)):
        sim = _sim(hw, w, precision)
        plan = hw.Plan([sim.problem], [sim.buffers], tuning=tu)
        hw.hwfv1_run(sim.problem, sim.buffers, 30, plan=plan)
        out = sim.export() + (sim.buffers.leaf_list(),)
        log("  tuning", tu, "leaves", len(out[3]))
        if ref is None:
            ref = out
        else:
            for x, y in zip(ref, out):
                assert np.array_equal(x, y)
        plan.close()


def _flood_with_recession(L=8):
    """Hydrograph case at small L whose inflow stops early: cells get wet,
    and blocks stay dry, turn wet and settle while the run goes on."""
    w = W.hydrograph_l12(L=L)
    w.params = dict(w.params, t_peak=300.0, t_base=600.0, t_end=math.inf)
    return w


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_write_history_does_not_change_results(hw, precision):
    """The FV1 step skips the stores of blocks that stayed dry; forgetting
    the history before every step (so that nothing is skipped) must give
    the same states, bit for bit."""
    w = _flood_with_recession()
    a, b = _sim(hw, w, precision), _sim(hw, w, precision)
    steps = 240
    a.run(steps)
    for _ in range(steps):
        hw.hw_forget(b.problem, b.buffers, stream=b.stream)
        b.run(1)
    sa, sb = a.scalars(), b.scalars()
    log("  history", precision, "t", sa["t"], "leaves", sa["n_leaves"],
        "wet cells", int((a.export()[0] > w.params["h_tol"]).sum()))
    assert sa["step"] == sb["step"] == steps and sa["t"] == sb["t"]
    assert sa["mass"] == sb["mass"]
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.buffers.leaf_list(), b.buffers.leaf_list())


def test_forget_after_restoring_a_state(hw):
    """A saved state written back into the buffers, followed by hw_forget,
    continues exactly as the first time."""
    w = _flood_with_recession()
    sim = _sim(hw, w)
    sim.run(60)
    snap = ([t.clone() for t in sim.buffers.fine[0]], [t.clone() for t in sim.buffers.fine[1]],
            sim.buffers.scal.clone())
    sim.run(40)
    ref = sim.export()
    for dst, src in zip(sim.buffers.fine[0], snap[0]):
        dst.copy_(src)
    for dst, src in zip(sim.buffers.fine[1], snap[1]):
        dst.copy_(src)
    sim.buffers.scal.copy_(snap[2])
    hw.hw_forget(sim.problem, sim.buffers, stream=sim.stream)
    sim.run(40)
    for x, y in zip(ref, sim.export()):
        assert np.array_equal(x, y)


def test_autotune_restores_state_and_picks_a_candidate(hw):
    from paper_2206_05761_amd.autotune import CANDIDATES, autotune
    w = W.circular_dambreak_l10(L=8)
    sim = _sim(hw, w)
    sim.run(5)
    before = sim.export() + (sim.scalars()["t"], sim.scalars()["step"])
    best, table = autotune([sim.problem], [sim.buffers], steps=3, warmup=1,
                           cache_path=None)
    after = sim.export() + (sim.scalars()["t"], sim.scalars()["step"])
    # a launch shape of the list, with the tree-sparse finest set on (the
    # default) or both of its skips off; one more timing for that choice
    shape = {k: v for k, v in best.items() if k not in ("encode_skip", "fill_skip")}
    assert shape in CANDIDATES and len(table) == len(CANDIDATES) + 1
    assert best == shape or (best["encode_skip"], best["fill_skip"]) == (0, 0)
    for x, y in zip(before[:3], after[:3]):
        assert np.array_equal(x, y)
    assert before[3:] == after[3:]


@pytest.mark.parametrize("precision", ["fp32_bulk", "fp64"])
def test_64_member_ensemble_equals_individual_runs(hw, precision):
    """The benchmark's ensemble shape at smaller levels: 64 members (the
    plan maximum) with their own L, eps, relief, friction and forcing
    (dam breaks with open edges, hydrographs through a west inlet), one
    launch per phase; every member's fields, leaf list, t and step count
    equal its own single run bit for bit."""
    ws = W.ensemble_64(n=64, n_steps=15, levels=(4, 5, 6, 7))
    steps = 15
    sims = [_sim(hw, w, precision) for w in ws]
    plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims])
    stats = hw.hwfv1_run_batch(plan, steps)
    log(f"  ensemble of {len(ws)} ({precision}): levels",
        sorted({w.L for w in ws}), "steps", [st["steps"] for st in stats][:8], "...")
    for w, s, st in zip(ws, sims, stats):
        ref = _sim(hw, w, precision)
        ref.run(steps)
        assert st["steps"] == ref.scalars()["step"], w.name
        for x, y in zip(s.export(), ref.export()):
            assert np.array_equal(x, y), w.name
        assert np.array_equal(s.buffers.leaf_list(), ref.buffers.leaf_list()), w.name
        assert s.scalars()["t"] == ref.scalars()["t"], w.name
        ref.close()
    plan.close()
    for s in sims:
        s.close()
