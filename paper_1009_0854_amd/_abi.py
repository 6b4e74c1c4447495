"""ctypes mirror of include/mact.h and the loader of libmact.so.

The library is loaded from this package's directory.  There is no fallback:
if libmact.so is absent every call raises, naming the build command.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

# MACT_LIB_VARIANT=san loads the build with sanitized host code (build.py --sanitize)
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "libmact_san.so" if os.environ.get("MACT_LIB_VARIANT") == "san" else "libmact.so")

# status codes
OK, E_INVALID, E_NOCONV, E_DEVICE, E_NOMEM, E_UNSUPPORTED, E_BUSY, E_CANCELLED = 0, -1, -2, -3, -4, -5, -6, -7
# functions
FN_CBRT, FN_ATAN_SQRT3, FN_ASIN2, FN_ACOS, FN_ATAN, FN_ATANC, FN_SIN, FN_COS, FN_ENC709, FN_DEC709 = range(10)
# transforms, element types, layouts, transfer functions, LUT methods
LAB, HSI, SCT, LUV = 0, 1, 2, 3
U8, F16, F32, U16 = 0, 1, 2, 3
HWC, CHW = 0, 1
GAMMA_BT709, GAMMA_SRGB, GAMMA_NONE = 0, 1, 2
TRILINEAR, PRISM, PYRAMIDAL, TETRAHEDRAL = 0, 1, 2, 3

XFORMS = {"lab": LAB, "hsi": HSI, "sct": SCT, "luv": LUV}
GAMMAS = {"bt709": GAMMA_BT709, "srgb": GAMMA_SRGB, "none": GAMMA_NONE}
METHODS = {"trilinear": TRILINEAR, "prism": PRISM, "pyramidal": PYRAMIDAL, "tetrahedral": TETRAHEDRAL}


class Approx(ctypes.Structure):
    _fields_ = [("fn", c_int32), ("n", c_int32), ("m", c_int32), ("iters", c_int32),
                ("lo", c_double), ("hi", c_double), ("p", c_double * 8), ("q", c_double * 8),
                ("eps", c_double), ("alt", c_double * 18), ("n_alt", c_int32), ("converged", c_int32)]

    @property
    def p_list(self):
        return [self.p[k] for k in range(self.n + 1)]

    @property
    def q_list(self):
        return [self.q[k] for k in range(self.m + 1)] if self.m > 0 else [1.0]


class Image(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("dtype", c_int32), ("layout", c_int32), ("width", c_int64),
                ("height", c_int64), ("row_stride", c_int64), ("plane_stride", c_int64), ("batch", c_int64),
                ("batch_stride", c_int64), ("gamma", c_int32), ("reserved", c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("xform", c_int32), ("out_mode", c_int32), ("f", Approx * 4)]


class Tune(ctypes.Structure):
    _fields_ = [("block", c_int32), ("tile", c_int32), ("vec", c_int32), ("waves_per_cu", c_int32),
                ("one_launch", c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena_bytes", c_size_t), ("max_batch", c_int32), ("compute_streams", c_int32),
                ("max_queue", c_int32), ("fail_request", c_int32), ("params", Params * 4)]


class Request(ctypes.Structure):
    _fields_ = [("host_in", c_void_p), ("host_out", c_void_p), ("in_dtype", c_int32), ("out_dtype", c_int32),
                ("xform", c_int32), ("gamma", c_int32), ("width", c_int64), ("height", c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("rejected", c_int64), ("batches", c_int64),
                ("p50_ms", c_double), ("p99_ms", c_double), ("mean_ms", c_double), ("mean_batch", c_double),
                ("device_busy_ms", c_double), ("failed", c_int64), ("cancelled", c_int64)]


class ErrorStats(ctypes.Structure):
    _fields_ = [("count", c_int64), ("mean", c_double), ("max", c_double), ("max_abs", c_double * 3)]


# exported symbol -> (restype, argtypes); the list the ABI test checks against the header
SIGNATURES = {
    "mact_status_str": (c_char_p, [c_int32]),
    "mact_last_error": (c_char_p, []),
    "mact_version": (c_char_p, []),
    "mact_fit": (c_int32, [c_int32, c_int32, c_int32, c_double, c_double, POINTER(Approx)]),
    "mact_fit_ex": (c_int32, [c_int32, c_int32, c_int32, c_double, c_double, c_int32, POINTER(Approx)]),
    "mact_transform_exact": (c_int32, [c_int32, POINTER(Image), POINTER(Image), c_void_p]),
    "mact_fit_weighted": (c_int32, [c_int32, c_int32, c_int32, c_double, c_double, POINTER(c_double), c_int32,
                                    c_int32, POINTER(Approx)]),
    "mact_default_approx": (c_int32, [c_int32, POINTER(Approx)]),
    "mact_paper_approx": (c_int32, [c_int32, c_int32, c_int32, POINTER(Approx)]),
    "mact_params_default": (c_int32, [c_int32, POINTER(Params)]),
    "mact_transform": (c_int32, [POINTER(Params), POINTER(Image), POINTER(Image), c_void_p]),
    "mact_transform_backward": (c_int32, [POINTER(Params), POINTER(Image), POINTER(Image), POINTER(Image), c_void_p]),
    "lut_bytes": (c_size_t, [c_int32, c_int32]),
    "lut_build": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_size_t, c_void_p]),
    "lut_interp": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(Image), POINTER(Image), c_void_p]),
    "mact_inverse_params_default": (c_int32, [c_int32, POINTER(Params)]),
    "mact_inverse": (c_int32, [POINTER(Params), POINTER(Image), POINTER(Image), c_void_p]),
    "mact_error_stats": (c_int32, [POINTER(Params), POINTER(Image), POINTER(ErrorStats), c_void_p]),
    "mact_error_stats_noalloc": (c_int32, [POINTER(Params), POINTER(Image), POINTER(ErrorStats), c_void_p]),
    "lut_cells_bytes": (c_size_t, [c_int32, c_int32]),
    "lut_cells_build": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_size_t, c_void_p]),
    "lut_cells_interp": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(Image), POINTER(Image), c_void_p]),
    "lut_cache_bytes": (c_size_t, [c_int32, c_int32]),
    "lut_cache_build": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_size_t, c_void_p]),
    "lut_cache_interp": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(Image), POINTER(Image), c_void_p]),
    "mact_batch_plan_create": (c_int32, [POINTER(Params), POINTER(Image), POINTER(Image), c_int32, POINTER(Tune),
                                         c_void_p, POINTER(c_void_p)]),
    "mact_batch_plan_launch": (c_int32, [c_void_p, c_int32, c_void_p]),
    "mact_batch_plan_tune": (c_int32, [c_void_p, POINTER(Tune)]),
    "mact_batch_plan_destroy": (c_int32, [c_void_p]),
    "mact_batch_run": (c_int32, [POINTER(Params), POINTER(Image), POINTER(Image), c_int32, POINTER(Tune), c_void_p]),
    "mact_server_create": (c_int32, [POINTER(ServerConfig), POINTER(c_void_p)]),
    "mact_server_submit": (c_int32, [c_void_p, POINTER(Request), POINTER(c_int64)]),
    "mact_server_poll": (c_int32, [c_void_p, c_int64, POINTER(c_int32)]),
    "mact_server_wait": (c_int32, [c_void_p, c_int64, c_int32]),
    "mact_server_latency": (c_int32, [c_void_p, c_int64, POINTER(c_double)]),
    "mact_server_stats_get": (c_int32, [c_void_p, POINTER(ServerStats)]),
    "mact_server_cancel": (c_int32, [c_void_p, c_int64]),
    "mact_server_destroy": (c_int32, [c_void_p]),
    "mact_stream_u8_to_f32": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    "mact_copy": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
}

_lib = None


class MactError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__("libmact status %d: %s" % (status, detail))


def lib():
    """The loaded libmact.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmact.so is not built (%s); run: python -m paper_1009_0854_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:  # the ABI test reports missing exports
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, allow=()):
    if status == OK or status in allow:
        return status
    detail = lib().mact_last_error().decode(errors="replace")
    raise MactError(status, detail)
