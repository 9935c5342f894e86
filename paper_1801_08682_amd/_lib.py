"""ctypes binding of libadg.so (argument marshalling only).

Every numerical step runs in the HIP kernels behind include/adg.h.  Loading
fails loudly when the library is missing: there is no CPU fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadg.so")
PEAKS_PATH = os.path.join(HERE, "libadg_peaks.so")
PEAKS_EXPORTS = ["adg_peak_fma", "adg_stream_copy", "adg_stream_triad"]

ADG_OK, ADG_ERR_INVALID_ARG, ADG_ERR_UNSUPPORTED, ADG_ERR_DEVICE, ADG_ERR_WORKSPACE = range(5)
STATUS_NAMES = {0: "ADG_OK", 1: "ADG_ERR_INVALID_ARG", 2: "ADG_ERR_UNSUPPORTED",
                3: "ADG_ERR_DEVICE", 4: "ADG_ERR_WORKSPACE"}

EXPORTS = ["adg_query", "adg_init", "adg_predict", "adg_correct", "adg_step",
           "adg_wave_speed", "adg_cfl_dt", "adg_step_adjoint", "adg_run_fused", "adg_fused_begin",
           "adg_fused_sweep", "adg_fused_end", "adg_step_noalloc", "adg_fv_project",
           "adg_fv_reconstruct", "adg_fv_step", "adg_destroy",
           "adg_last_error", "adg_version"]


class AdgConfig(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32),
                ("order", ctypes.c_int32),
                ("n_cells", ctypes.c_int32 * 3),
                ("length", ctypes.c_double * 3),
                ("pde", ctypes.c_int32),
                ("pde_param", ctypes.c_double * 4),
                ("picard_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32),
                ("adjoint", ctypes.c_int32),
                ("fused", ctypes.c_int32),
                ("spacetime_traces", ctypes.c_int32)]


class AdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load libadg.so once and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_1801_08682_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(path)
    vp, i64, dp, ip = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    cfgp = ctypes.POINTER(AdgConfig)
    sig = {
        "adg_query": [cfgp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "adg_init": [cfgp, vp, i64, vp, ctypes.POINTER(vp)],
        "adg_predict": [vp, dp, dp, dp],
        "adg_correct": [vp, dp, dp, dp, ip],
        "adg_step": [vp, dp, dp, dp, ip],
        "adg_wave_speed": [vp, dp, dp],
        "adg_cfl_dt": [vp, ctypes.c_double, dp, dp],
        "adg_step_adjoint": [vp, dp, dp, dp, dp, dp],
        "adg_run_fused": [vp, dp, dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                          ctypes.c_int32, dp, ip, ip],
        "adg_fused_begin": [vp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, dp,
                            ctypes.c_int32, ip, ip],
        "adg_fused_sweep": [vp],
        "adg_fused_end": [vp],
        "adg_step_noalloc": [vp, dp, dp, dp, ip, dp],
        "adg_fv_project": [vp, dp, dp],
        "adg_fv_reconstruct": [vp, dp, dp],
        "adg_fv_step": [vp, dp, dp, dp, dp, ip],
        "adg_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.adg_last_error.argtypes = [vp]
    L.adg_last_error.restype = ctypes.c_char_p
    L.adg_version.argtypes = []
    L.adg_version.restype = ctypes.c_int32
    _lib = L
    return L


_peaks = None


def load_peaks(path=PEAKS_PATH):
    """Load libadg_peaks.so (roofline measurement kernels) once."""
    global _peaks
    if _peaks is not None:
        return _peaks
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_1801_08682_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    for name, args in {"adg_peak_fma": [i32, i32, i32, vp, vp],
                       "adg_stream_copy": [vp, vp, i64, vp],
                       "adg_stream_triad": [vp, vp, vp, ctypes.c_double, i64, vp]}.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    _peaks = L
    return L


def check(status, ctx=None):
    if status != ADG_OK:
        L = load()
        msg = L.adg_last_error(ctx).decode()
        raise AdgError(status, msg)


def make_config(dim, order, n_cells, length, pde, pde_param=(), picard_iters=0, precision=0,
                adjoint=False, fused=False, spacetime=False):
    c = AdgConfig()
    c.dim = dim
    c.order = order
    nc = list(n_cells) + [1] * (3 - len(n_cells))
    ln = list(length) if hasattr(length, "__len__") else [length * nc[i] / nc[0] for i in range(3)]
    ln = ln + [1.0] * (3 - len(ln))
    for i in range(3):
        c.n_cells[i] = int(nc[i])
        c.length[i] = float(ln[i])
    c.pde = pde
    pp = list(pde_param) + [0.0] * (4 - len(pde_param))
    for i in range(4):
        c.pde_param[i] = float(pp[i])
    c.picard_iters = picard_iters
    c.precision = precision
    c.adjoint = 1 if adjoint else 0
    c.fused = 1 if fused else 0
    c.spacetime_traces = 1 if spacetime else 0
    return c


def query(cfg):
    """(dofs_per_cell, params_per_cell, workspace_bytes); host only."""
    L = load()
    a, b, w = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(L.adg_query(ctypes.byref(cfg), ctypes.byref(a), ctypes.byref(b), ctypes.byref(w)))
    return a.value, b.value, w.value
