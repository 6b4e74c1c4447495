"""MACT on MI355X: minimax-approximated colour-space transforms (Celebi,
Kingravi & Celiker, "Fast Color Space Transformations Using Minimax
Approximations") as hand-written HIP kernels for gfx950 behind a C ABI
(include/mact.h, libmact.so).

This module only marshals arguments: torch tensors supply device memory and
streams, and every step of a transform runs in libmact's kernels.  If the
library has not been built, every call raises.
"""
import ctypes

from . import _abi as A
from ._abi import (CHW, E_BUSY, E_NOCONV, F16, F32, FN_ACOS, FN_ASIN2, FN_ATAN, FN_ATAN_SQRT3, FN_ATANC, FN_CBRT,
                   GAMMA_BT709, GAMMA_NONE, GAMMA_SRGB, HSI, HWC, LAB, PRISM, PYRAMIDAL, SCT, TETRAHEDRAL, TRILINEAR,
                   U8, Approx, Image, MactError, Params, Request, ServerConfig, ServerStats, Tune, lib)

__all__ = ["fit", "dark_end_weight", "default_approx", "paper_approx", "default_params", "make_params", "image", "transform",
           "transform_exact",
           "transform_backward", "inverse_params", "inverse", "error_stats", "error_stats_noalloc", "lut_bytes", "lut_build",
           "lut_interp", "lut_cells_bytes", "lut_cells_build", "lut_cells_interp",
           "lut_cache_bytes", "lut_cache_build", "lut_cache_interp",
           "approx_to_dict", "approx_from_dict", "save_approx", "load_approx", "BatchPlan", "batch_run",
           "Server", "stream_u8_to_f32", "copy", "MactError", "MactLab"]


def _torch():
    import torch
    return torch


def _xf(x):
    return A.XFORMS[x] if isinstance(x, str) else int(x)


def _gm(g):
    return A.GAMMAS[g] if isinstance(g, str) else int(g)


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- approximations

def fit(fn, n, m, lo, hi, max_iter=100, allow_noconv=False, weight=None, n_weight=4097):
    """mact_fit: Remez fit of function `fn` (FN_*) by p/q, degrees (n, m), on [lo, hi].

    With `weight` (samples at equally spaced points of [lo, hi], or a callable
    sampled at `n_weight` such points) the fit is mact_fit_weighted's: it
    minimises max |w (f - p/q)| and eps is that weighted maximum."""
    out = Approx()
    if weight is None:
        st = lib().mact_fit_ex(int(fn), int(n), int(m), float(lo), float(hi), int(max_iter), ctypes.byref(out))
    else:
        if callable(weight):
            weight = [float(weight(lo + (hi - lo) * i / (n_weight - 1))) for i in range(n_weight)]
        w = (ctypes.c_double * len(weight))(*[float(v) for v in weight])
        st = lib().mact_fit_weighted(int(fn), int(n), int(m), float(lo), float(hi), w, len(weight), int(max_iter),
                                     ctypes.byref(out))
    A.check(st, allow=(E_NOCONV,) if allow_noconv else ())
    return out


def dark_end_weight(beta, delta, lo=0.008856, hi=1.0):
    """The weight ((t - lo + delta) / (hi - lo + delta))^beta for a CIELAB
    cube-root fit: it damps the criterion near the threshold (the darkest
    colours, few in number), so the error shrinks over the rest of the range.
    beta = 0 is the plain minimax fit."""
    return lambda t: ((t - lo + delta) / (hi - lo + delta)) ** beta


def default_approx(fn):
    out = Approx()
    A.check(lib().mact_default_approx(int(fn), ctypes.byref(out)))
    return out


def paper_approx(fn, n, m=0):
    out = Approx()
    A.check(lib().mact_paper_approx(int(fn), int(n), int(m), ctypes.byref(out)))
    return out


def default_params(xform, decode=False):
    """mact_params_default; with decode=True (CIELAB, CIELUV) float inputs decode
    BT.709 with the default minimax polynomial instead of the exact power."""
    p = Params()
    A.check(lib().mact_params_default(_xf(xform), ctypes.byref(p)))
    if decode:
        if p.xform not in (A.LAB, A.LUV):
            raise ValueError("decode applies to CIELAB and CIELUV only")
        p.f[1] = default_approx(A.FN_DEC709)
    return p


# ---------------------------------------------------------------- persisted coefficient sets

_FN_NAMES = {A.FN_CBRT: "cbrt", A.FN_ATAN_SQRT3: "atan_sqrt3", A.FN_ASIN2: "asin2", A.FN_ACOS: "acos",
             A.FN_ATAN: "atan", A.FN_ATANC: "atanc", A.FN_SIN: "sin", A.FN_COS: "cos", A.FN_ENC709: "enc709",
             A.FN_DEC709: "dec709"}


def approx_to_dict(a):
    """One approximation as plain JSON data: function, interval, degrees,
    numerator and denominator coefficients, error, alternation points and the
    fitter's iteration count and convergence flag."""
    return {"function": _FN_NAMES.get(a.fn, "fn%d" % a.fn), "fn": int(a.fn), "n": int(a.n), "m": int(a.m),
            "interval": [a.lo, a.hi], "p": [a.p[k] for k in range(a.n + 1)],
            "q": [a.q[k] for k in range(a.m + 1)], "eps": a.eps,
            "alternation": [a.alt[k] for k in range(a.n_alt)], "iters": int(a.iters), "converged": int(a.converged)}


def approx_from_dict(d):
    """The mact_approx that approx_to_dict described (every value exactly:
    JSON keeps a double's shortest round-trip form)."""
    a = Approx()
    a.fn, a.n, a.m = int(d["fn"]), int(d["n"]), int(d["m"])
    if not (0 <= a.n <= 7 and 0 <= a.m <= 7 and len(d["p"]) == a.n + 1 and len(d["q"]) == a.m + 1):
        raise ValueError("approx_from_dict: degrees and coefficient counts disagree")
    if len(d["alternation"]) > 18:
        raise ValueError("approx_from_dict: more than 18 alternation points")
    a.lo, a.hi = float(d["interval"][0]), float(d["interval"][1])
    for k, v in enumerate(d["p"]):
        a.p[k] = float(v)
    for k, v in enumerate(d["q"]):
        a.q[k] = float(v)
    a.eps = float(d["eps"])
    for k, v in enumerate(d["alternation"]):
        a.alt[k] = float(v)
    a.n_alt = len(d["alternation"])
    a.iters, a.converged = int(d["iters"]), int(d["converged"])
    return a


def save_approx(path, approxes):
    """Writes a named set of approximations ({name: mact_approx}) to a JSON file."""
    import json
    with open(path, "w") as f:
        json.dump({k: approx_to_dict(v) for k, v in approxes.items()}, f, indent=1, sort_keys=True)


def load_approx(path):
    """Reads a set written by save_approx: {name: mact_approx}."""
    import json
    with open(path) as f:
        return {k: approx_from_dict(v) for k, v in json.load(f).items()}


def make_params(xform, approxes, out_mode=0):
    """Params for `xform` with the given approximations (LAB: [cbrt]; HSI:
    [atan_sqrt3]; SCT: [asin2, acos, atan, atanc])."""
    p = Params()
    p.xform = _xf(xform)
    p.out_mode = int(out_mode)
    for i, a in enumerate(approxes):
        p.f[i] = a
    return p


# ---------------------------------------------------------------- images

def _dtype_code(t):
    torch = _torch()
    m = {torch.uint8: U8, torch.float16: F16, torch.float32: F32, torch.uint16: A.U16}
    if t.dtype not in m:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return m[t.dtype]


def image(t, layout="hwc", gamma="bt709"):
    """Describe a CUDA tensor as an mact_image: HWC (H, W, 3) or (N, H, W, 3);
    CHW (3, H, W) or (N, 3, H, W).  Strides are taken from the tensor."""
    if not t.is_cuda:
        raise ValueError("image(): tensor must be on the GPU")
    if t.numel() == 0:
        # the C ABI reads batch 0 as one image: an empty tensor has no description
        raise ValueError("image(): empty tensor %s" % (tuple(t.shape),))
    if any(st == 0 and n > 1 for st, n in zip(t.stride(), t.shape)):
        # the C ABI reads a stride of 0 as "packed": a broadcast view would be read past its storage
        raise ValueError("image(): broadcast (zero-stride) tensor; call .contiguous() first")
    im = Image()
    im.data = t.data_ptr()
    im.dtype = _dtype_code(t)
    im.gamma = _gm(gamma)
    lay = HWC if layout in ("hwc", HWC) else CHW
    im.layout = lay
    s = t.stride()
    if lay == HWC:
        if t.dim() not in (3, 4) or t.shape[-1] != 3:
            raise ValueError("HWC tensor must be (H, W, 3) or (N, H, W, 3), got %s" % (tuple(t.shape),))
        if s[-1] != 1 or s[-2] != 3:
            raise ValueError("HWC tensor needs channel stride 1 and pixel stride 3")
        im.height, im.width = t.shape[-3], t.shape[-2]
        im.row_stride = s[-3]
        im.plane_stride = 0
        im.batch = t.shape[0] if t.dim() == 4 else 1
        im.batch_stride = s[0] if t.dim() == 4 else 0
    else:
        if t.dim() not in (3, 4) or t.shape[-3] != 3:
            raise ValueError("CHW tensor must be (3, H, W) or (N, 3, H, W), got %s" % (tuple(t.shape),))
        if s[-1] != 1:
            raise ValueError("CHW tensor needs unit stride along W")
        im.height, im.width = t.shape[-2], t.shape[-1]
        im.row_stride = s[-2]
        im.plane_stride = s[-3]
        im.batch = t.shape[0] if t.dim() == 4 else 1
        im.batch_stride = s[0] if t.dim() == 4 else 0
    return im


def _out_like(x, layout, out_layout, out_dtype):
    """An output tensor for x (in `layout`) in `out_layout`."""
    torch = _torch()
    shape = tuple(x.shape)
    lay = "hwc" if layout in ("hwc", HWC) else "chw"
    olay = "hwc" if out_layout in ("hwc", HWC) else "chw"
    if lay != olay:
        lead = shape[:-3]
        if lay == "hwc":  # (..., H, W, 3) -> (..., 3, H, W)
            shape = lead + (3, shape[-3], shape[-2])
        else:  # (..., 3, H, W) -> (..., H, W, 3)
            shape = lead + (shape[-2], shape[-1], 3)
    return torch.empty(shape, dtype=out_dtype, device=x.device)


def transform(x, xform="lab", params=None, layout="hwc", gamma="bt709", out=None, out_layout=None,
              out_dtype=None, stream=None):
    """mact_transform of tensor x; returns the output tensor (same shape)."""
    torch = _torch()
    p = params if params is not None else default_params(xform)
    out_layout = layout if out_layout is None else out_layout
    if out is None:
        out = _out_like(x, layout, out_layout, out_dtype or torch.float32)
    if x.numel() == 0:  # nothing to transform
        return out
    A.check(lib().mact_transform(ctypes.byref(p), ctypes.byref(image(x, layout, gamma)),
                                 ctypes.byref(image(out, out_layout)), _stream(stream)))
    return out


def transform_exact(x, xform="lab", gamma="bt709", out=None, out_dtype=None, stream=None):
    """mact_transform_exact: the exact transform in float32 with the device's
    elementary functions (the baseline MACT replaces), packed 8-bit HWC in."""
    torch = _torch()
    if out is None:
        out = _out_like(x, "hwc", "hwc", out_dtype or torch.float32)
    if x.numel() == 0:
        return out
    A.check(lib().mact_transform_exact(_xf(xform), ctypes.byref(image(x, "hwc", gamma)),
                                       ctypes.byref(image(out, "hwc")), _stream(stream)))
    return out


def transform_backward(x, grad_out, params=None, layout="chw", grad_in=None, stream=None):
    """mact_transform_backward: d(sum <grad_out, Lab(x)>)/dx for linear float32 x."""
    torch = _torch()
    p = params if params is not None else default_params("lab")
    if grad_in is None:
        grad_in = torch.empty_like(x)
    if x.numel() == 0:
        return grad_in
    A.check(lib().mact_transform_backward(ctypes.byref(p), ctypes.byref(image(x, layout, "none")),
                                          ctypes.byref(image(grad_out, layout)),
                                          ctypes.byref(image(grad_in, layout)), _stream(stream)))
    return grad_in


# ---------------------------------------------------------------- inverses, error statistics

def inverse_params(xform="lab"):
    """mact_inverse_params_default: the default approximations of the inverse."""
    p = Params()
    A.check(lib().mact_inverse_params_default(_xf(xform), ctypes.byref(p)))
    return p


def inverse(x, xform="lab", params=None, layout="hwc", gamma="bt709", out=None, out_layout=None, out_dtype=None,
            stream=None):
    """mact_inverse of float tensor x (L*a*b*, HSI, SCT or L*u*v* triples) to
    R'G'B' on the [0, 1] scale; `gamma` is the encoding of the CIELAB and
    CIELUV inverses' output ('bt709' or 'none')."""
    torch = _torch()
    p = params if params is not None else inverse_params(xform)
    out_layout = layout if out_layout is None else out_layout
    if out is None:
        out = _out_like(x, layout, out_layout, out_dtype or torch.float32)
    if x.numel() == 0:  # nothing to transform
        return out
    A.check(lib().mact_inverse(ctypes.byref(p), ctypes.byref(image(x, layout, "none")),
                               ctypes.byref(image(out, out_layout, gamma)), _stream(stream)))
    return out


def error_stats(x, xform="lab", params=None, layout="hwc", gamma="bt709", stream=None):
    """mact_error_stats: accuracy of the MACT transform of RGB tensor x against
    the exact transform, computed on the device.  Returns a dict with count,
    mean, max and max_abs (per channel)."""
    p = params if params is not None else default_params(xform)
    e = A.ErrorStats()
    if x.numel() == 0:
        return {"count": 0, "mean": 0.0, "max": 0.0, "max_abs": [0.0, 0.0, 0.0]}
    A.check(lib().mact_error_stats(ctypes.byref(p), ctypes.byref(image(x, layout, gamma)), ctypes.byref(e),
                                   _stream(stream)))
    return {"count": e.count, "mean": e.mean, "max": e.max, "max_abs": [e.max_abs[c] for c in range(3)]}


def error_stats_noalloc(x, xform="lab", params=None, layout="hwc", gamma="bt709", stream=None):
    """mact_error_stats_noalloc: error_stats without any device allocation in
    the library (the accumulator is a fixed per-GPU device array; calls that
    overlap on one GPU race)."""
    p = params if params is not None else default_params(xform)
    e = A.ErrorStats()
    if x.numel() == 0:
        return {"count": 0, "mean": 0.0, "max": 0.0, "max_abs": [0.0, 0.0, 0.0]}
    A.check(lib().mact_error_stats_noalloc(ctypes.byref(p), ctypes.byref(image(x, layout, gamma)), ctypes.byref(e),
                                           _stream(stream)))
    return {"count": e.count, "mean": e.mean, "max": e.max, "max_abs": [e.max_abs[c] for c in range(3)]}


# ---------------------------------------------------------------- LUTs

def lut_bytes(xform, n):
    return int(lib().lut_bytes(_xf(xform), int(n)))


def lut_build(xform, n, gamma="bt709", device="cuda", stream=None):
    """Packed N^3 LUT as a float32 device tensor (lut_build)."""
    torch = _torch()
    nbytes = lut_bytes(xform, n)
    if nbytes == 0:
        raise MactError(A.E_INVALID, "lut_bytes: invalid xform/n")
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device=device)
    A.check(lib().lut_build(_xf(xform), int(n), _gm(gamma), ctypes.c_void_p(buf.data_ptr()), nbytes, _stream(stream)))
    return buf


def lut_interp(lut, n, xform, method, x, layout="hwc", out=None, out_layout=None, out_dtype=None, stream=None):
    torch = _torch()
    out_layout = layout if out_layout is None else out_layout
    if out is None:
        out = _out_like(x, layout, out_layout, out_dtype or torch.float32)
    m = A.METHODS[method] if isinstance(method, str) else int(method)
    if x.numel() == 0:  # nothing to transform
        return out
    A.check(lib().lut_interp(ctypes.c_void_p(lut.data_ptr()), int(n), _xf(xform), m,
                             ctypes.byref(image(x, layout, "none")), ctypes.byref(image(out, out_layout)),
                             _stream(stream)))
    return out


def lut_cells_bytes(xform, n):
    return int(lib().lut_cells_bytes(_xf(xform), int(n)))


def lut_cells_build(lut, n, xform, stream=None):
    """Cell-major form (lut_cells_build) of a packed LUT from lut_build, as a
    float32 device tensor on the LUT's device."""
    torch = _torch()
    nbytes = lut_cells_bytes(xform, n)
    if nbytes == 0:
        raise MactError(A.E_INVALID, "lut_cells_bytes: invalid xform/n")
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device=lut.device)
    A.check(lib().lut_cells_build(ctypes.c_void_p(lut.data_ptr()), int(n), _xf(xform),
                                  ctypes.c_void_p(buf.data_ptr()), nbytes, _stream(stream)))
    return buf


def lut_cells_interp(cells, n, xform, method, x, layout="hwc", out=None, out_layout=None, out_dtype=None,
                     stream=None):
    torch = _torch()
    out_layout = layout if out_layout is None else out_layout
    if out is None:
        out = _out_like(x, layout, out_layout, out_dtype or torch.float32)
    m = A.METHODS[method] if isinstance(method, str) else int(method)
    if x.numel() == 0:  # nothing to transform
        return out
    A.check(lib().lut_cells_interp(ctypes.c_void_p(cells.data_ptr()), int(n), _xf(xform), m,
                                   ctypes.byref(image(x, layout, "none")), ctypes.byref(image(out, out_layout)),
                                   _stream(stream)))
    return out


def lut_cache_bytes(xform, n):
    return int(lib().lut_cache_bytes(_xf(xform), int(n)))


def lut_cache_build(xform, n, gamma="bt709", device="cuda", stream=None):
    """Caching form (lut_cache_build): per-cell records of the node value and
    the 12 edge differences, as a float32 device tensor."""
    torch = _torch()
    nbytes = lut_cache_bytes(xform, n)
    if nbytes == 0:
        raise MactError(A.E_INVALID, "lut_cache_bytes: invalid xform/n")
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device=device)
    A.check(lib().lut_cache_build(_xf(xform), int(n), _gm(gamma), ctypes.c_void_p(buf.data_ptr()), nbytes,
                                  _stream(stream)))
    return buf


def lut_cache_interp(cache, n, xform, method, x, layout="hwc", out=None, out_layout=None, out_dtype=None,
                     stream=None):
    torch = _torch()
    out_layout = layout if out_layout is None else out_layout
    if out is None:
        out = _out_like(x, layout, out_layout, out_dtype or torch.float32)
    m = A.METHODS[method] if isinstance(method, str) else int(method)
    if x.numel() == 0:  # nothing to transform
        return out
    A.check(lib().lut_cache_interp(ctypes.c_void_p(cache.data_ptr()), int(n), _xf(xform), m,
                                   ctypes.byref(image(x, layout, "none")), ctypes.byref(image(out, out_layout)),
                                   _stream(stream)))
    return out


# ---------------------------------------------------------------- batched form

def _arrays(params, ins, outs, layouts=None, gammas=None, out_layouts=None):
    n = len(ins)
    P = (Params * n)(*params)
    layouts = layouts or ["hwc"] * n
    out_layouts = out_layouts or layouts
    gammas = gammas or ["bt709"] * n
    I = (Image * n)(*[image(t, l, g) for t, l, g in zip(ins, layouts, gammas)])
    O = (Image * n)(*[image(t, l) for t, l in zip(outs, out_layouts)])
    return P, I, O


class BatchPlan:
    """A persistent, graph-captured batched transform of many images
    (mact_batch_plan_*).  Keeps references to the tensors it reads and writes."""

    def __init__(self, params, ins, outs, layouts=None, gammas=None, out_layouts=None, tune=None, stream=None):
        self._keep = (list(ins), list(outs))
        P, I, O = _arrays(params, ins, outs, layouts, gammas, out_layouts)
        h = ctypes.c_void_p()
        t = ctypes.byref(tune) if tune is not None else None
        A.check(lib().mact_batch_plan_create(P, I, O, len(ins), t, _stream(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, use_graph=True, stream=None):
        A.check(lib().mact_batch_plan_launch(self._h, 1 if use_graph else 0, _stream(stream)))

    @property
    def tune(self):
        t = Tune()
        A.check(lib().mact_batch_plan_tune(self._h, ctypes.byref(t)))
        return t

    def close(self):
        if self._h:
            lib().mact_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_run(params, ins, outs, layouts=None, gammas=None, out_layouts=None, tune=None, stream=None):
    P, I, O = _arrays(params, ins, outs, layouts, gammas, out_layouts)
    t = ctypes.byref(tune) if tune is not None else None
    A.check(lib().mact_batch_run(P, I, O, len(ins), t, _stream(stream)))


# ---------------------------------------------------------------- serving

def check_request_tensors(host_in, host_out):
    """The served form's buffers: contiguous (H, W, 3) host tensors of one
    shape (the engine copies H W 3 elements into and out of them); raises
    ValueError otherwise."""
    for name, t in (("host_in", host_in), ("host_out", host_out)):
        if t.is_cuda:
            raise ValueError("Server.submit: %s must be a host tensor" % name)
        if t.dim() != 3 or t.shape[-1] != 3:
            raise ValueError("Server.submit: %s must be (H, W, 3), got %s" % (name, tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("Server.submit: %s must be contiguous" % name)
    if tuple(host_out.shape) != tuple(host_in.shape):
        raise ValueError("Server.submit: host_out shape %s differs from host_in shape %s"
                         % (tuple(host_out.shape), tuple(host_in.shape)))


class Server:
    """Continuous-batching engine (mact_server_*)."""

    def __init__(self, arena_bytes=1 << 30, max_batch=64, compute_streams=2, max_queue=1 << 16, params=None,
                 fail_request=0):
        cfg = ServerConfig()
        cfg.arena_bytes = int(arena_bytes)
        cfg.max_batch = int(max_batch)
        cfg.compute_streams = int(compute_streams)
        cfg.max_queue = int(max_queue)
        cfg.fail_request = int(fail_request)  # fault injection for tests of the error path; 0 = off
        for i, x in enumerate(("lab", "hsi", "sct", "luv")):
            cfg.params[i] = (params or {}).get(x) or default_params(x)
        h = ctypes.c_void_p()
        A.check(lib().mact_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, host_in, host_out, xform="lab", gamma="bt709"):
        """Queue one packed HWC image held in pinned host tensors; returns its id.
        Both tensors must be contiguous (H, W, 3) host tensors of the same shape:
        the engine copies H W 3 elements in and out of them."""
        check_request_tensors(host_in, host_out)
        r = Request()
        r.host_in = host_in.data_ptr()
        r.host_out = host_out.data_ptr()
        r.in_dtype = _dtype_code(host_in)
        r.out_dtype = _dtype_code(host_out)
        r.xform = _xf(xform)
        r.gamma = _gm(gamma)
        r.height, r.width = host_in.shape[0], host_in.shape[1]
        i = ctypes.c_int64()
        A.check(lib().mact_server_submit(self._h, ctypes.byref(r), ctypes.byref(i)))
        self._keep[i.value] = (host_in, host_out)
        return i.value

    def poll(self, rid):
        d = ctypes.c_int32()
        A.check(lib().mact_server_poll(self._h, int(rid), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, rid, timeout_ms=60000):
        """Blocks until request `rid` completes; raises MactError with the
        request's status if it completed with an error (or on a time-out)."""
        st = lib().mact_server_wait(self._h, int(rid), int(timeout_ms))
        if st != E_BUSY:
            self._keep.pop(rid, None)
        A.check(st)

    def cancel(self, rid):
        """Withdraws request `rid` if it is still waiting for admission (True;
        it then completes with MACT_E_CANCELLED); False if it was already
        admitted and runs to completion."""
        st = lib().mact_server_cancel(self._h, int(rid))
        if st == E_BUSY:
            return False
        A.check(st)
        self._keep.pop(rid, None)
        return True

    def latency_ms(self, rid):
        v = ctypes.c_double()
        A.check(lib().mact_server_latency(self._h, int(rid), ctypes.byref(v)))
        return v.value

    def stats(self):
        s = ServerStats()
        A.check(lib().mact_server_stats_get(self._h, ctypes.byref(s)))
        return s

    def close(self):
        if self._h:
            A.check(lib().mact_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- reference kernels

def stream_u8_to_f32(src, dst, n_px, stream=None):
    A.check(lib().mact_stream_u8_to_f32(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                        int(n_px), _stream(stream)))


def copy(src, dst, nbytes, stream=None):
    A.check(lib().mact_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), int(nbytes),
                            _stream(stream)))


from .autograd import MactLab  # noqa: E402
