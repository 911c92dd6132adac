"""ctypes binding of libflamefront.so (argument marshalling only).

The library is built in-tree by ``paper_0911_2889_amd.build``. Importing this
module without the built library raises: there is no fallback path.
"""

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libflamefront.so")

FLAME_OK = 0
FLAME_ERR_INVALID_ARG = -1
FLAME_ERR_WORKSPACE_TOO_SMALL = -2
FLAME_ERR_HIP = -3
FLAME_ERR_UNSUPPORTED_SIZE = -4
FLAME_ERR_NONFINITE = -5
FLAME_ERR_TIMEOUT = -6

# every symbol the C header declares
EXPORTS = (
    "flame_state_bytes", "flame_workspace_bytes", "flame_init", "flame_set_spectrum",
    "flame_get_spectrum", "flame_set_state", "flame_get_state", "flame_state_modified",
    "flame_step_index", "flame_step", "flame_diagnostics", "flame_adjoint_step", "flame_area_gradient",
    "flame_synthesize", "flame_timing_begin", "flame_timing_end", "flame_set_graph_steps",
    "flame_set_points_per_thread", "flame_get_points_per_thread", "flame_set_product_grid",
    "flame_get_product_grid", "flame_set_streaming_stores", "flame_get_streaming_stores", "flame_set_r0_table",
    "flame_set_forcing", "flame_autotune", "flame_destroy", "flame_step_noalloc",
    "flame_circle_state_bytes", "flame_circle_step", "flame_circle_diagnostics", "flame_diagnostics_host",
    "flame_set_persistent", "flame_get_persistent", "flame_last_error",
)


class FlameDesc(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int32),
        ("n2", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("theta_pi", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("axis_scale", ctypes.c_double * 2),
        ("r0_law", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
    ]


class CircleDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("seg", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
    ]


class FlameError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"flame error {code}: {message}")
        self.code = code


_lib = None


def load():
    """Load the shared library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0911_2889_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    desc_p = ctypes.POINTER(FlameDesc)
    sig = {
        "flame_state_bytes": [desc_p, ctypes.POINTER(sz)],
        "flame_workspace_bytes": [desc_p, i32, ctypes.POINTER(sz)],
        "flame_init": [desc_p, i32, ctypes.POINTER(P), P, sz, P, ctypes.POINTER(P)],
        "flame_set_spectrum": [P, i32, P, i64],
        "flame_get_spectrum": [P, i32, P],
        "flame_set_state": [P, i32, P, i64],
        "flame_get_state": [P, i32, P],
        "flame_state_modified": [P, i32, i64],
        "flame_step_index": [P, ctypes.POINTER(i64)],
        "flame_step": [P, i32],
        "flame_diagnostics": [P, i32, P, ctypes.c_void_p],
        "flame_diagnostics_host": [P, i32, ctypes.POINTER(ctypes.c_double)],
        "flame_adjoint_step": [P, i32, i64, P, P, P],
        "flame_area_gradient": [P, i32, i64, P, P],
        "flame_synthesize": [P, i32, P, P],
        "flame_set_graph_steps": [P, i32],
        "flame_set_persistent": [P, i32, i32, i32],
        "flame_get_persistent": [P, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "flame_set_points_per_thread": [P, i32, i32, i32, i32],
        "flame_get_points_per_thread": [P, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "flame_autotune": [P, i32, ctypes.POINTER(i32)],
        "flame_set_product_grid": [P, i32, i32, i32],
        "flame_set_r0_table": [P, i32, ctypes.c_void_p, ctypes.c_int64],
        "flame_set_forcing": [P, i32, ctypes.c_void_p],
        "flame_get_product_grid": [P, i32, i32, ctypes.POINTER(i32)],
        "flame_set_streaming_stores": [P, i32, i32, i32],
        "flame_get_streaming_stores": [P, i32, i32, ctypes.POINTER(i32)],
        "flame_timing_begin": [P],
        "flame_timing_end": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
        "flame_destroy": [P],
        "flame_step_noalloc": [desc_p, P, i64, i32, P],
        "flame_circle_state_bytes": [ctypes.POINTER(CircleDesc), ctypes.POINTER(sz)],
        "flame_circle_step": [ctypes.POINTER(CircleDesc), i32, P, i64, i32, P],
        "flame_circle_diagnostics": [ctypes.POINTER(CircleDesc), i32, P, i64, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.flame_last_error.argtypes = []
    lib.flame_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc):
    if rc != FLAME_OK:
        msg = load().flame_last_error().decode("utf-8", "replace")
        raise FlameError(rc, msg)
    return rc


def make_desc(n1, n2, gamma=0.8, theta_pi=1.0, t0=200.0, dt=0.25, axis_scale=None, r0_law=0, integrator=0):
    """integrator: 0 integrating-factor Euler, 1 integrating-factor Heun (or "euler" / "rk2")."""
    d = FlameDesc()
    d.n1, d.n2 = int(n1), int(n2)
    d.gamma, d.theta_pi, d.t0, d.dt = float(gamma), float(theta_pi), float(t0), float(dt)
    sc = (0.0, 0.0) if axis_scale is None else (float(axis_scale[0]), float(axis_scale[1]))
    d.axis_scale[0], d.axis_scale[1] = sc
    d.r0_law = int(r0_law)
    d.integrator = {"euler": 0, "rk2": 1}.get(integrator, integrator) if isinstance(integrator, str) else int(integrator)
    return d


def state_bytes(desc):
    out = ctypes.c_size_t()
    check(load().flame_state_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def workspace_bytes(descs):
    arr = (FlameDesc * len(descs))(*descs)
    out = ctypes.c_size_t()
    check(load().flame_workspace_bytes(arr, len(descs), ctypes.byref(out)))
    return out.value


def make_circle_desc(n, gamma=0.8, seg=1.0, t0=200.0, dt=0.25):
    d = CircleDesc()
    d.n = int(n)
    d.gamma, d.seg, d.t0, d.dt = float(gamma), float(seg), float(t0), float(dt)
    return d
