"""GPU: mra_traverse_leaves_noalloc (no workspace, scratch in the library's
per-GPU array) gives the leaf list and count of mra_traverse_leaves, bit for
bit, on two calls in a row, the second with a smaller problem; both match
the oracle's depth-first walk of the same flags.  Called through the C ABI."""
import sys

import numpy as np
import pytest

import oracle as O
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


def _flags_case(hw, w, eps):
    """Buffers of a workload after encoding and flagging (sig on device)."""
    import torch
    params = dict(w.params, eps=eps)
    sim = hw.Simulation(params, w.h, w.qx, w.qy, w.z)
    hw.mra_encode(sim.problem, sim.buffers)
    hw.mra_flag(sim.problem, sim.buffers)
    torch.cuda.synchronize()
    return sim


def _leaves(hw, sim):
    import torch
    torch.cuda.synchronize()
    n = int(sim.buffers.scalars()["n_leaves"])
    return sim.buffers.leaves[:n].cpu().numpy().view(np.uint32).copy(), n


def test_noalloc_traversal_equals_workspace_traversal(hw):
    import torch
    cases = [(W.circular_dambreak_flat(11), 1e-3),   # the largest level held
             (W.dambreak_bumps_l6(L=6), 5e-3)]       # then a smaller one
    for w, eps in cases:
        L = w.L
        log("no-alloc traversal", w.name, "L", L, "eps", eps)
        sim = _flags_case(hw, w, eps)
        p, b = sim.problem, sim.buffers
        hw.mra_traverse_leaves(p, b)
        ref, nref = _leaves(hw, sim)
        # poison the outputs, then the variant without a workspace
        b.leaves.fill_(-1)
        sc = hw.HwScalars.from_buffer_copy(b.scal.cpu().numpy().tobytes())
        sc.n_leaves = 0
        b.scal.copy_(torch.frombuffer(bytearray(bytes(sc)), dtype=torch.uint8))
        c = hw.HwBuffers.from_buffer_copy(bytes(b.c))
        c.work = None
        c.work_bytes = 0
        hw.mra_traverse_leaves_noalloc(p, c)
        got, n = _leaves(hw, sim)
        log("  leaves", n, "of", 4 ** L)
        assert n == nref and 1 < n < 4 ** L
        assert np.array_equal(got, ref)
        sig = b.sig[: hw.n_coarse(L)].cpu().numpy()
        assert np.array_equal(got, O.dft_from_flags(L, sig))
        sim.close()


def test_noalloc_traversal_rejects_levels_beyond_its_scratch(hw):
    p = hw.make_problem(W.base_params(12, 1.0, 1e-3))
    c = hw.HwBuffers()
    with pytest.raises(hw.HwError) as e:
        hw.mra_traverse_leaves_noalloc(p, c)
    assert e.value.code == hw.HW_ECAPACITY
    assert hw.noalloc_scratch_bytes() < 8 << 20
