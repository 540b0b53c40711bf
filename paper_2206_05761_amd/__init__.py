"""Python binding of the MI355X HWFV1 library (libhwfv1.so, C ABI in
include/hwfv1.h).

Argument marshalling only: every step of the timestep runs in the library's
HIP kernels.  PyTorch provides device memory (tensors) and streams.  The
library must be built (``python -m paper_2206_05761_amd.build`` or
``__graft_entry__.build()``); importing the entry points without it raises.
"""
import ctypes as C
import math
import os
from pathlib import Path

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libhwfv1.so"

HW_OK, HW_EINVAL, HW_EINPUT, HW_ECAPACITY, HW_EHIP, HW_ENONFINITE = range(6)
HW_FP64, HW_FP32_BULK = 0, 1
HW_BC_WALL, HW_BC_OPEN = 0, 1
PRECISION = {"fp64": HW_FP64, "f64": HW_FP64, "fp32_bulk": HW_FP32_BULK,
             "fp32": HW_FP32_BULK, HW_FP64: HW_FP64, HW_FP32_BULK: HW_FP32_BULK}
_BC = {"wall": HW_BC_WALL, "open": HW_BC_OPEN}


class HwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"HWFV1 error {code}: {msg}")
        self.code = code


class HwProblem(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("precision", C.c_int32), ("bc", C.c_int32 * 4),
        ("eps", C.c_double), ("g", C.c_double), ("cfl", C.c_double),
        ("h_tol", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
        ("dt_max", C.c_double), ("manning_n", C.c_double),
        ("rain_rate", C.c_double), ("inlet_y0", C.c_double),
        ("inlet_y1", C.c_double), ("q_peak", C.c_double),
        ("t_peak", C.c_double), ("t_base", C.c_double), ("t_end", C.c_double),
        ("zsmax", C.c_double),
    ]


class HwScalars(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("dt", C.c_double), ("mass", C.c_double),
        ("mass0", C.c_double), ("smax", C.c_double * 4),
        ("maxspeed", C.c_double), ("acc", C.c_double * 6),
        ("step", C.c_uint64), ("n_leaves", C.c_uint64),
        ("leaf_updates", C.c_uint64), ("clips", C.c_uint64),
        ("dry_stored", C.c_uint64), ("dry_skipped", C.c_uint64),
        ("cur", C.c_uint32), ("done", C.c_uint32), ("nonfinite", C.c_uint32),
        ("map_step", C.c_uint32),
    ]


class HwBuffers(C.Structure):
    _fields_ = [
        ("fine", (C.c_void_p * 3) * 2), ("coarse", C.c_void_p * 3),
        ("zhier", C.c_void_p), ("zsig", C.c_void_p), ("raw", C.c_void_p),
        ("sig", C.c_void_p), ("leaves", C.c_void_p), ("scal", C.c_void_p),
        ("work", C.c_void_p), ("work_bytes", C.c_size_t),
    ]


class HwTuning(C.Structure):
    _fields_ = [("encode_cells_per_thread", C.c_int32),
                ("fv1_block", C.c_int32), ("fv1_grid", C.c_int32),
                ("fv1_write_skip", C.c_int32), ("encode_skip", C.c_int32),
                ("fill_skip", C.c_int32), ("encode_tiles", C.c_int32),
                ("block_list", C.c_int32)]


class HwStats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("t", C.c_double), ("dt", C.c_double),
        ("mass0", C.c_double), ("mass", C.c_double),
        ("n_leaves", C.c_uint64), ("leaf_updates", C.c_uint64),
        ("clips", C.c_uint64), ("dry_stored", C.c_uint64),
        ("dry_skipped", C.c_uint64), ("wall_s", C.c_double),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "python -m paper_2206_05761_amd.build")
        L = C.CDLL(str(LIB_PATH))
        vp, P = C.c_void_p, C.POINTER
        L.hw_last_error.restype = C.c_char_p
        L.hw_validate.argtypes = [P(HwProblem)]
        for f in ("hw_n_fine", "hw_n_coarse", "hw_n_hier"):
            getattr(L, f).argtypes = [C.c_int32]
            getattr(L, f).restype = C.c_uint64
        L.hw_workspace_bytes.argtypes = [P(HwProblem)]
        L.hw_workspace_bytes.restype = C.c_size_t
        L.hw_default_tuning.argtypes = [P(HwProblem), P(HwTuning)]
        L.hw_default_tuning.restype = None
        L.hw_ingest.argtypes = [P(HwProblem), P(HwBuffers), vp, vp, vp, vp, vp]
        L.mra_encode.argtypes = [P(HwProblem), P(HwBuffers), vp, vp]
        L.mra_flag.argtypes = [P(HwProblem), P(HwBuffers), vp]
        L.mra_traverse_leaves.argtypes = [P(HwProblem), P(HwBuffers), vp]
        L.mra_traverse_leaves_noalloc.argtypes = [P(HwProblem), P(HwBuffers), vp]
        L.hw_noalloc_scratch_bytes.argtypes = []
        L.hw_noalloc_scratch_bytes.restype = C.c_size_t
        L.fv1_step.argtypes = [P(HwProblem), P(HwBuffers), vp]
        L.hwfv1_run.argtypes = [P(HwProblem), P(HwBuffers), vp, C.c_int64,
                                P(HwStats), vp]
        L.hw_plan_create.argtypes = [P(vp), P(HwProblem), P(HwBuffers),
                                     C.c_int32, P(HwTuning)]
        L.hw_plan_create_uniform.argtypes = [P(vp), P(HwProblem), P(HwBuffers),
                                             C.c_int32, P(HwTuning)]
        L.hw_plan_destroy.argtypes = [vp]
        L.hwfv1_run_batch.argtypes = [vp, C.c_int64, P(HwStats), vp]
        L.hw_export.argtypes = [P(HwProblem), P(HwBuffers), vp, vp, vp, vp]
        L.hw_forget.argtypes = [P(HwProblem), P(HwBuffers), vp]
        L.hw_plan_profile.argtypes = [vp, C.c_int64, P(C.c_double), vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != HW_OK:
        raise HwError(rc, lib().hw_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_problem(params: dict, precision="fp64") -> HwProblem:
    """Problem struct from the shared parameter dictionary."""
    p = HwProblem()
    p.L = int(params["L"])
    p.precision = PRECISION[precision]
    bc = params.get("bc", ("wall",) * 4)
    for k in range(4):
        p.bc[k] = _BC[bc[k]] if isinstance(bc[k], str) else int(bc[k])
    p.eps = float(params["eps"])
    p.g = float(params.get("g", 9.80665))
    p.cfl = float(params.get("cfl", 0.5))
    p.h_tol = float(params.get("h_tol", 1e-6))
    p.dx = float(params["dx"])
    p.dy = float(params.get("dy", params["dx"]))
    p.dt_max = float(params.get("dt_max", 1.0))
    p.manning_n = float(params.get("manning_n", 0.0))
    p.rain_rate = float(params.get("rain_rate", 0.0))
    p.inlet_y0 = float(params.get("inlet_y0", 0.0))
    p.inlet_y1 = float(params.get("inlet_y1", 0.0))
    p.q_peak = float(params.get("q_peak", 0.0))
    p.t_peak = float(params.get("t_peak", 1.0))
    p.t_base = float(params.get("t_base", 2.0))
    p.t_end = float(params.get("t_end", math.inf))
    p.zsmax = float(params.get("zsmax", 0.0))
    return p


def validate(problem: HwProblem) -> None:
    _check(lib().hw_validate(C.byref(problem)))


def n_fine(L):
    return int(lib().hw_n_fine(L))


def n_coarse(L):
    return int(lib().hw_n_coarse(L))


def n_hier(L):
    return int(lib().hw_n_hier(L))


def first_descendant(leaves, L):
    """Morton index of the first finest descendant of each hierarchy index
    (the depth-first sort key of a leaf list)."""
    idx = np.asarray(leaves, dtype=np.int64)
    offs = (4 ** np.arange(L + 2, dtype=np.int64) - 1) // 3
    n = np.searchsorted(offs, idx, side="right") - 1
    return (idx - offs[n]) << (2 * (L - n))


def workspace_bytes(problem: HwProblem) -> int:
    n = int(lib().hw_workspace_bytes(C.byref(problem)))
    if n == 0:
        validate(problem)
    return n


class Buffers:
    """Device buffers of one problem (torch tensors) and their C view."""

    def __init__(self, problem: HwProblem, device="cuda"):
        L = problem.L
        flow = torch.float64 if problem.precision == HW_FP64 else torch.float32
        N, Nc, Nh = n_fine(L), n_coarse(L), n_hier(L)
        e = lambda n, dt: torch.empty(max(n, 1), dtype=dt, device=device)
        self.fine = [[e(N, flow) for _ in range(3)] for _ in range(2)]
        self.coarse = [e(Nc, flow) for _ in range(3)]
        self.zhier = e(Nh, torch.float64)
        self.zsig = e(Nc, torch.uint8)
        self.raw = e(Nc, torch.uint8)
        self.sig = e(Nc, torch.uint8)
        self.leaves = e(N, torch.int32)
        self.scal = torch.zeros(C.sizeof(HwScalars), dtype=torch.uint8, device=device)
        wb = workspace_bytes(problem)
        self.work = torch.empty(wb, dtype=torch.uint8, device=device)
        c = HwBuffers()
        for s in range(2):
            for v in range(3):
                c.fine[s][v] = self.fine[s][v].data_ptr()
        for v in range(3):
            c.coarse[v] = self.coarse[v].data_ptr()
        c.zhier = self.zhier.data_ptr()
        c.zsig = self.zsig.data_ptr()
        c.raw = self.raw.data_ptr()
        c.sig = self.sig.data_ptr()
        c.leaves = self.leaves.data_ptr()
        c.scal = self.scal.data_ptr()
        c.work = self.work.data_ptr()
        c.work_bytes = wb
        self.c = c
        self.L = L
        self.problem = problem

    def scalars(self) -> dict:
        raw = self.scal.cpu().numpy().tobytes()
        s = HwScalars.from_buffer_copy(raw)
        out = {k: getattr(s, k) for k, _ in HwScalars._fields_ if k not in ("smax", "acc", "map_step")}
        out["smax"] = list(s.smax)
        return out

    def current_fine(self):
        cur = self.scalars()["cur"]
        return self.fine[cur]

    def leaf_list_stored(self):
        """The current leaf list as stored.  When every finest cell is a
        leaf the time loop does not write the list (it is the finest level in
        order).  After a plan step the whole 8 x 8 blocks of finest leaves
        come first (block-first list); the entry points store depth-first
        order."""
        n = int(self.scalars()["n_leaves"])
        if n == n_fine(self.problem.L):
            return (np.arange(n, dtype=np.uint64) + n_coarse(self.problem.L)).astype(np.uint32)
        return self.leaves[:n].cpu().numpy().view(np.uint32)

    def leaf_list(self):
        """The current leaves in depth-first order (Algorithm 2: ascending
        first finest descendant), whichever order they are stored in."""
        raw = self.leaf_list_stored()
        key = first_descendant(raw, self.problem.L)
        if raw.size < 2 or bool(np.all(key[1:] > key[:-1])):
            return raw
        return raw[np.argsort(key, kind="stable")]


# ---- entry points (same names as the C ABI) ---------------------------------
def hw_ingest(problem, buffers, h, qx, qy, z, stream=None):
    """h, qx, qy, z: row-major float64 CUDA tensors of 4^L entries."""
    arrs = []
    for a in (h, qx, qy, z):
        if not (a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()):
            raise ValueError("ingest inputs must be contiguous float64 CUDA tensors")
        if a.numel() != n_fine(problem.L):
            raise ValueError("ingest input size does not match 4^L")
        arrs.append(C.c_void_p(a.data_ptr()))
    _check(lib().hw_ingest(C.byref(problem), C.byref(buffers.c), *arrs, _stream(stream)))


def mra_encode(problem, buffers, details=None, stream=None):
    dp = None
    if details is not None:
        if details.dtype != torch.float64 or details.numel() < 9 * n_coarse(problem.L):
            raise ValueError("details needs 9 (4^L-1)/3 float64 entries")
        dp = C.c_void_p(details.data_ptr())
    _check(lib().mra_encode(C.byref(problem), C.byref(buffers.c), dp, _stream(stream)))


def mra_flag(problem, buffers, stream=None):
    _check(lib().mra_flag(C.byref(problem), C.byref(buffers.c), _stream(stream)))


def mra_traverse_leaves(problem, buffers, stream=None):
    _check(lib().mra_traverse_leaves(C.byref(problem), C.byref(buffers.c), _stream(stream)))


def mra_traverse_leaves_noalloc(problem, buffers, stream=None):
    """Traversal without a workspace (scratch in a per-GPU library array,
    levels up to 11); buffers may be a Buffers object or an HwBuffers."""
    c = buffers.c if hasattr(buffers, "c") else buffers
    _check(lib().mra_traverse_leaves_noalloc(C.byref(problem), C.byref(c), _stream(stream)))


def noalloc_scratch_bytes():
    return int(lib().hw_noalloc_scratch_bytes())


def fv1_step(problem, buffers, stream=None):
    _check(lib().fv1_step(C.byref(problem), C.byref(buffers.c), _stream(stream)))


def hw_forget(problem, buffers, stream=None):
    """Forget the FV1 write history (after writing fine sets or scal directly)."""
    _check(lib().hw_forget(C.byref(problem), C.byref(buffers.c), _stream(stream)))


def hw_export(problem, buffers, stream=None):
    """Current finest h, qx, qy as row-major float64 CUDA tensors [2^L, 2^L]."""
    n = 1 << problem.L
    out = [torch.empty((n, n), dtype=torch.float64, device=buffers.zhier.device)
           for _ in range(3)]
    _check(lib().hw_export(C.byref(problem), C.byref(buffers.c),
                           *[C.c_void_p(o.data_ptr()) for o in out], _stream(stream)))
    return tuple(out)


def _stats_dict(st: HwStats) -> dict:
    return {k: getattr(st, k) for k, _ in HwStats._fields_}


def hwfv1_run(problem, buffers, max_steps, plan=None, stats=True, stream=None):
    """Run up to max_steps steps (or to t_end); returns the stats dict when
    stats is true (this synchronises the stream)."""
    st = HwStats() if stats else None
    _check(lib().hwfv1_run(C.byref(problem), C.byref(buffers.c),
                           plan.handle if plan is not None else None,
                           int(max_steps), C.byref(st) if st is not None else None,
                           _stream(stream)))
    return _stats_dict(st) if st is not None else None


class Plan:
    """Descriptors, launch shapes and the captured step graph of 1..64
    problems.  uniform=True makes a uniform FV1 plan (every finest cell
    updated each step, no multiresolution phases)."""

    def __init__(self, problems, buffers, tuning=None, uniform=False):
        n = len(problems)
        self._probs = (HwProblem * n)(*problems)
        self._bufs = (HwBuffers * n)(*[b.c for b in buffers])
        self._keep = list(buffers)
        self.n = n
        tu = None
        if tuning is not None:
            tu = HwTuning(int(tuning.get("encode_cells_per_thread", 0)),
                          int(tuning.get("fv1_block", 0)),
                          int(tuning.get("fv1_grid", 0)),
                          int(tuning.get("fv1_write_skip", 1)),
                          int(tuning.get("encode_skip", 1)),
                          int(tuning.get("fill_skip", 1)),
                          int(tuning.get("encode_tiles", 0)),
                          int(tuning.get("block_list", 1)))
        h = C.c_void_p()
        create = lib().hw_plan_create_uniform if uniform else lib().hw_plan_create
        _check(create(C.byref(h), self._probs, self._bufs, n,
                      C.byref(tu) if tu is not None else None))
        self.handle = h
        self.uniform = bool(uniform)

    def close(self):
        if self.handle:
            lib().hw_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PHASES = ("encode", "regularise", "traverse", "fv1", "fill", "finalize")
# single launches inside those phases (HW_PROF_ENCODE_FIRST, HW_PROF_FV1_HEAVY)
PROF_KERNELS = ("encode_first_pass", "fv1_heavy")


def hw_plan_profile(plan, steps, stream=None) -> dict:
    """Total milliseconds per phase over `steps` un-graphed steps, and of
    the first encoding pass and the heavy FV1 kernel alone."""
    keys = PHASES + PROF_KERNELS
    out = (C.c_double * len(keys))()
    _check(lib().hw_plan_profile(plan.handle, int(steps), out, _stream(stream)))
    return dict(zip(keys, list(out)))


def hwfv1_run_batch(plan, max_steps, stats=True, stream=None):
    arr = (HwStats * plan.n)() if stats else None
    _check(lib().hwfv1_run_batch(plan.handle, int(max_steps), arr, _stream(stream)))
    return [_stats_dict(s) for s in arr] if arr is not None else None


# ---- convenience -------------------------------------------------------------
class Simulation:
    """One problem on the GPU: buffers, ingest from host arrays, runs."""

    def __init__(self, params: dict, h, qx, qy, z, precision="fp64",
                 device="cuda", stream=None):
        self.params = dict(params)
        self.problem = make_problem(params, precision)
        validate(self.problem)
        self.buffers = Buffers(self.problem, device)
        self.stream = stream
        dev = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1),
                               device=device) for a in (h, qx, qy, z)]
        hw_ingest(self.problem, self.buffers, *dev, stream=stream)
        self.plan = None

    def run(self, max_steps, stats=True):
        if self.plan is None:
            self.plan = Plan([self.problem], [self.buffers])
        return hwfv1_run(self.problem, self.buffers, max_steps, plan=self.plan,
                         stats=stats, stream=self.stream)

    def export(self):
        return tuple(t.cpu().numpy() for t in hw_export(self.problem, self.buffers,
                                                         stream=self.stream))

    def scalars(self):
        torch.cuda.synchronize()
        return self.buffers.scalars()

    def close(self):
        if self.plan is not None:
            self.plan.close()
            self.plan = None
