"""ctypes wrapper of the HWFV1 CPU oracle.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package.  The HIP product path never does.

Arrays cross the boundary as float64 / uint8 / uint32 numpy arrays.  Finest
fields are row-major [j, i] (j = row / y, i = column / x).  Hierarchy data are
in the Z-order index layout (Morton code within a level, levels concatenated
from the coarsest).
"""
import ctypes as C
import math

import numpy as np

from .build import ensure_built

_lib = None

VAR = {"h": 0, "qx": 1, "qy": 2, "z": 3}
BC = {"wall": 0, "open": 1}
SCALARS = ["t", "dt", "step", "n_leaves", "mass", "clips", "maxspeed",
           "leaf_updates", "smax_h", "smax_qx", "smax_qy", "smax_z"]


class OracleProblem(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("bc", C.c_int32 * 4),
        ("eps", C.c_double), ("g", C.c_double), ("cfl", C.c_double),
        ("h_tol", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
        ("dt_max", C.c_double), ("manning_n", C.c_double),
        ("rain_rate", C.c_double), ("inlet_y0", C.c_double),
        ("inlet_y1", C.c_double), ("q_peak", C.c_double),
        ("t_peak", C.c_double), ("t_base", C.c_double), ("t_end", C.c_double),
        ("zsmax", C.c_double),
    ]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _u32(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def lib():
    global _lib
    if _lib is None:
        path = ensure_built()
        L = C.CDLL(str(path))
        vp = C.c_void_p
        pd = C.POINTER(C.c_double)
        pu8 = C.POINTER(C.c_uint8)
        pu32 = C.POINTER(C.c_uint32)
        L.oracle_create.restype = vp
        L.oracle_create.argtypes = [C.POINTER(OracleProblem), pd, pd, pd, pd]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_set_time.argtypes = [vp, C.c_double, C.c_double, C.c_int64]
        for name in ("oracle_phase_encode", "oracle_phase_regularise",
                     "oracle_phase_traverse", "oracle_phase_fv1",
                     "oracle_uniform_fv1_step"):
            getattr(L, name).argtypes = [vp]
        L.oracle_step.argtypes = [vp]
        L.oracle_step.restype = C.c_int
        L.oracle_run.argtypes = [vp, C.c_int64]
        L.oracle_run.restype = C.c_int64
        L.oracle_get_fine.argtypes = [vp, pd, pd, pd]
        L.oracle_get_hierarchy.argtypes = [vp, C.c_int, pd]
        L.oracle_get_details.argtypes = [vp, C.c_int, pd]
        L.oracle_get_flags.argtypes = [vp, C.c_int, pu8]
        L.oracle_get_leaves.argtypes = [vp, pu32]
        L.oracle_get_leaves.restype = C.c_int64
        L.oracle_get_scalars.argtypes = [vp, pd]
        L.oracle_morton.argtypes = [C.c_uint32, C.c_uint32]
        L.oracle_morton.restype = C.c_uint32
        L.oracle_zindex.argtypes = [C.c_int, C.c_uint32, C.c_uint32]
        L.oracle_zindex.restype = C.c_uint64
        L.oracle_haar_encode.argtypes = [pd, pd]
        L.oracle_haar_decode.argtypes = [pd, pd]
        L.oracle_roundtrip.argtypes = [C.c_int, pd, pd]
        L.oracle_face_flux.argtypes = [C.POINTER(OracleProblem), pd, pd, pd,
                                       pd]
        L.oracle_dft_from_flags.argtypes = [C.c_int, pu8, pu32]
        L.oracle_dft_from_flags.restype = C.c_int64
        L.oracle_regularise_flags.argtypes = [C.c_int, pu8, pu8]
        _lib = L
    return _lib


def make_problem(params: dict) -> OracleProblem:
    """Problem struct from the shared parameter dictionary."""
    p = OracleProblem()
    p.L = int(params["L"])
    bc = params.get("bc", ("wall",) * 4)
    for k in range(4):
        p.bc[k] = BC[bc[k]] if isinstance(bc[k], str) else int(bc[k])
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


def n_coarse(L: int) -> int:
    return ((1 << (2 * L)) - 1) // 3


def n_hier(L: int) -> int:
    return ((1 << (2 * (L + 1))) - 1) // 3


class Oracle:
    """One HWFV1 run on the CPU oracle."""

    def __init__(self, params: dict, h, qx, qy, z):
        self.params = dict(params)
        self.L = int(params["L"])
        self.side = 1 << self.L
        self._prob = make_problem(params)
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
                for a in (h, qx, qy, z)]
        for a in arrs:
            if a.size != self.side * self.side:
                raise ValueError("input size does not match 4^L")
        self._h = lib().oracle_create(C.byref(self._prob), *[_dp(a) for a in arrs])
        if not self._h:
            raise ValueError("oracle_create rejected the problem")

    def close(self):
        if self._h:
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # time loop -----------------------------------------------------------
    def step(self) -> bool:
        return bool(lib().oracle_step(self._h))

    def run(self, max_steps: int) -> int:
        return int(lib().oracle_run(self._h, int(max_steps)))

    def set_time(self, t, dt, step):
        lib().oracle_set_time(self._h, float(t), float(dt), int(step))

    def phase_encode(self):
        lib().oracle_phase_encode(self._h)

    def phase_regularise(self):
        lib().oracle_phase_regularise(self._h)

    def phase_traverse(self):
        lib().oracle_phase_traverse(self._h)

    def phase_fv1(self):
        lib().oracle_phase_fv1(self._h)

    def uniform_fv1_step(self):
        lib().oracle_uniform_fv1_step(self._h)

    # getters ----------------------------------------------------------------
    def fine(self):
        n = self.side
        out = [np.empty((n, n)) for _ in range(3)]
        lib().oracle_get_fine(self._h, *[_dp(a) for a in out])
        return tuple(out)

    def hierarchy(self, var):
        out = np.empty(n_hier(self.L))
        lib().oracle_get_hierarchy(self._h, VAR.get(var, var), _dp(out))
        return out

    def details(self, var):
        out = np.empty(3 * n_coarse(self.L))
        lib().oracle_get_details(self._h, VAR.get(var, var), _dp(out))
        return out.reshape(3, -1)

    def flags(self, which):
        code = {"raw": 0, "sig": 1, "zraw": 2}.get(which, which)
        out = np.empty(n_coarse(self.L), dtype=np.uint8)
        lib().oracle_get_flags(self._h, code, _u8(out))
        return out

    def leaves(self):
        n = int(lib().oracle_get_leaves(self._h, None))
        out = np.empty(max(n, 1), dtype=np.uint32)
        lib().oracle_get_leaves(self._h, _u32(out))
        return out[:n]

    def scalars(self) -> dict:
        out = np.empty(len(SCALARS))
        lib().oracle_get_scalars(self._h, _dp(out))
        return dict(zip(SCALARS, out.tolist()))


# building blocks -------------------------------------------------------------
def morton(i: int, j: int) -> int:
    return int(lib().oracle_morton(i, j))


def zindex(n: int, i: int, j: int) -> int:
    return int(lib().oracle_zindex(n, i, j))


def haar_encode(children):
    s = np.ascontiguousarray(children, dtype=np.float64)
    out = np.empty(4)
    lib().oracle_haar_encode(_dp(s), _dp(out))
    return out


def haar_decode(coeffs):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    out = np.empty(4)
    lib().oracle_haar_decode(_dp(c), _dp(out))
    return out


def roundtrip(L: int, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    lib().oracle_roundtrip(int(L), _dp(f), _dp(out))
    return out


def face_flux(params: dict, left, right):
    p = make_problem(params)
    l = np.ascontiguousarray(left, dtype=np.float64)
    r = np.ascontiguousarray(right, dtype=np.float64)
    F = np.empty(3)
    hs = np.empty(2)
    lib().oracle_face_flux(C.byref(p), _dp(l), _dp(r), _dp(F), _dp(hs))
    return F, hs


def dft_from_flags(L: int, sig):
    s = np.ascontiguousarray(sig, dtype=np.uint8)
    out = np.empty(1 << (2 * L), dtype=np.uint32)
    n = int(lib().oracle_dft_from_flags(int(L), _u8(s), _u32(out)))
    return out[:n]


def regularise_flags(L: int, raw):
    r = np.ascontiguousarray(raw, dtype=np.uint8)
    out = np.empty_like(r)
    lib().oracle_regularise_flags(int(L), _u8(r), _u8(out))
    return out
