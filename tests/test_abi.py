"""The C ABI on the CPU: the library loads and exports every symbol the
header declares, struct layouts match, mact_fit agrees with the oracle's
independent Remez, the printed tables match, and invalid calls return the
documented status without touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mact.h")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    from paper_1009_0854_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1009_0854_amd import build
        build.build()
    M.lib()
    return M


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:mact_status|size_t|char\s*\*|const char\s*\*)\s*\**\s*(\w+)\s*\(", text, re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(M):
    from paper_1009_0854_amd import _abi
    names = declared_functions()
    assert len(names) >= 25, names
    L = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding knows every declared function, and nothing else
    assert sorted(_abi.SIGNATURES) == names


def test_struct_layouts_match_the_header(M, tmp_path):
    from paper_1009_0854_amd import _abi
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mact.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                   "sizeof(mact_approx), sizeof(mact_image), sizeof(mact_params), sizeof(mact_tune),"
                   "sizeof(mact_server_config), sizeof(mact_request), sizeof(mact_server_stats),"
                   "offsetof(mact_approx, eps), offsetof(mact_image, gamma), offsetof(mact_server_config, params),"
                   "sizeof(mact_error), offsetof(mact_error, max_abs), offsetof(mact_server_config, fail_request),"
                   "offsetof(mact_server_stats, failed));return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(_abi.Approx), ctypes.sizeof(_abi.Image), ctypes.sizeof(_abi.Params), ctypes.sizeof(_abi.Tune),
            ctypes.sizeof(_abi.ServerConfig), ctypes.sizeof(_abi.Request), ctypes.sizeof(_abi.ServerStats),
            _abi.Approx.eps.offset, _abi.Image.gamma.offset, _abi.ServerConfig.params.offset,
            ctypes.sizeof(_abi.ErrorStats), _abi.ErrorStats.max_abs.offset, _abi.ServerConfig.fail_request.offset,
            _abi.ServerStats.failed.offset]
    assert got == want


def test_status_strings(M):
    L = M.lib()
    for s in range(0, -8, -1):
        assert L.mact_status_str(s) != b"unknown status"
    assert L.mact_status_str(-7) == b"cancelled" and L.mact_status_str(-8) == b"unknown status"
    assert b"gfx950" in L.mact_version()


FITS = [
    (0, 4, 4, 0.008856, 1.0), (0, 2, 2, 0.008856, 1.0), (0, 3, 4, 0.008856, 1.0), (0, 5, 0, 0.0, 1.0),
    (1, 5, 0, 0.0, 1.0), (1, 3, 0, 0.0, 254 / 256), (2, 5, 0, 0.0, 1 / np.sqrt(2)), (3, 4, 0, 0.0, 0.5),
    (4, 5, 0, 0.0, 1.0), (5, 4, 0, 1 / 255, 1.0),
    # the inverses' functions: sine and cosine, the BT.709 encoding power
    (6, 7, 0, 0.0, np.pi / 2), (7, 7, 0, 0.0, np.pi / 2), (7, 7, 0, 0.0, 2 * np.pi / 3), (8, 4, 4, 0.018, 1.0),
    # the BT.709 decoding power, for float inputs
    (9, 7, 0, 0.081, 1.0),
]


@pytest.mark.parametrize("fn,n,m,lo,hi", FITS)
def test_mact_fit_agrees_with_oracle_remez(M, fn, n, m, lo, hi):
    from numpy.polynomial import polynomial as Pm
    from oracle import remez, tables as T
    f = [T.f_cbrt, T.f_atan_sqrt3, T.f_asin2, T.f_acos, T.f_atan, T.f_atanc, np.sin, np.cos,
         lambda x: 1.099 * np.power(x, 0.45) - 0.099, lambda x: np.power((x + 0.099) / 1.099, 1 / 0.45)][fn]
    a = M.fit(fn, n, m, lo, hi)
    o = remez.remez(f, n, m, lo, hi)
    assert a.converged == 1
    assert a.eps == pytest.approx(o.eps, rel=1e-6)
    x = np.linspace(lo, hi, 20001)
    r_lib = Pm.polyval(x, a.p_list) / Pm.polyval(x, a.q_list)
    assert np.max(np.abs(r_lib - o(x))) <= 1e-3 * o.eps
    # the library's own alternation set levels the error at eps with alternating signs
    alt = np.array(a.alt[:a.n_alt])
    assert a.n_alt == n + m + 2
    e = Pm.polyval(alt, a.p_list) / Pm.polyval(alt, a.q_list) - f(alt)
    assert np.all(np.sign(e[1:]) == -np.sign(e[:-1]))
    np.testing.assert_allclose(np.abs(e), a.eps, rtol=1e-5)


WEIGHTED = [
    # the dark-end damped weight of the CIELAB cube root, (beta, delta)
    (0, 4, 4, 0.008856, 1.0, "damped", (0.5, 0.02)), (0, 4, 4, 0.008856, 1.0, "damped", (0.25, 0.002)),
    (0, 3, 3, 0.008856, 1.0, "damped", (1.0, 0.1)),
    # a smooth polynomial weight on the arctangent
    (4, 5, 0, 0.0, 1.0, "poly", None),
]


@pytest.mark.parametrize("fn,n,m,lo,hi,kind,arg", WEIGHTED)
def test_mact_fit_weighted_agrees_with_oracle_remez(M, fn, n, m, lo, hi, kind, arg):
    # both sides fit under the same piecewise-linear weight (the library's samples, interpolated)
    from numpy.polynomial import polynomial as Pm
    from oracle import remez, tables as T
    f = [T.f_cbrt, None, None, None, T.f_atan][fn]
    if kind == "damped":
        g = M.dark_end_weight(*arg, lo=lo, hi=hi)
    else:
        g = lambda x: 1.0 + 4.0 * x * x
    knots = np.linspace(lo, hi, 4097)
    samples = g(knots)
    w = lambda x: np.interp(np.asarray(x, dtype=np.float64), knots, samples)
    a = M.fit(fn, n, m, lo, hi, weight=samples)
    o = remez.remez(f, n, m, lo, hi, w=w)
    assert a.converged == 1 and o.converged
    assert a.eps == pytest.approx(o.eps, rel=1e-6)
    x = np.linspace(lo, hi, 20001)
    r_lib = Pm.polyval(x, a.p_list) / Pm.polyval(x, a.q_list)
    assert np.max(np.abs(w(x) * (r_lib - o(x)))) <= 1e-3 * o.eps
    alt = np.array(a.alt[:a.n_alt])
    e = w(alt) * (Pm.polyval(alt, a.p_list) / Pm.polyval(alt, a.q_list) - f(alt))
    assert a.n_alt == n + m + 2
    assert np.all(np.sign(e[1:]) == -np.sign(e[:-1]))
    np.testing.assert_allclose(np.abs(e), a.eps, rtol=1e-5)
    # the callable form samples the same points (up to the rounding of the sample positions)
    b = M.fit(fn, n, m, lo, hi, weight=g, n_weight=4097)
    np.testing.assert_allclose(b.p_list, a.p_list, rtol=1e-8)
    assert b.eps == pytest.approx(a.eps, rel=1e-8)


def test_mact_fit_weighted_constant_weight_is_the_plain_fit(M):
    a = M.fit(0, 4, 4, 0.008856, 1.0)
    b = M.fit(0, 4, 4, 0.008856, 1.0, weight=[2.5, 2.5])
    np.testing.assert_allclose(b.p_list, a.p_list, rtol=1e-9)
    np.testing.assert_allclose(b.q_list, a.q_list, rtol=1e-9)
    assert b.eps == pytest.approx(2.5 * a.eps, rel=1e-9)


def test_mact_fit_weighted_invalid(M):
    from paper_1009_0854_amd import _abi
    L = M.lib()
    out = _abi.Approx()
    ok = (ctypes.c_double * 3)(1.0, 2.0, 1.0)
    assert L.mact_fit_weighted(0, 2, 2, 0.1, 1.0, None, 3, 100, ctypes.byref(out)) == _abi.E_INVALID
    assert L.mact_fit_weighted(0, 2, 2, 0.1, 1.0, ok, 1, 100, ctypes.byref(out)) == _abi.E_INVALID
    assert L.mact_fit_weighted(0, 2, 2, 0.1, 1.0, ok, 65537, 100, ctypes.byref(out)) == _abi.E_INVALID
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        w = (ctypes.c_double * 3)(1.0, bad, 1.0)
        assert L.mact_fit_weighted(0, 2, 2, 0.1, 1.0, w, 3, 100, ctypes.byref(out)) == _abi.E_INVALID, bad
        assert b"weight" in L.mact_last_error()
    assert L.mact_fit_weighted(0, 2, 2, 0.1, 1.0, ok, 3, 100, None) == _abi.E_INVALID
    assert L.mact_fit_weighted(0, 2, 2, 1.0, 0.5, ok, 3, 100, ctypes.byref(out)) == _abi.E_INVALID
    assert L.mact_fit_weighted(0, 2, 2, 0.1, 1.0, ok, 3, 100, ctypes.byref(out)) == _abi.OK


def test_mact_fit_nonconvergence_and_invalid(M):
    from paper_1009_0854_amd import _abi
    a = M.fit(0, 4, 4, 0.008856, 1.0, max_iter=1, allow_noconv=True)
    assert a.converged == 0 and a.eps > 0 and a.n == 4 and a.m == 4
    with pytest.raises(_abi.MactError) as e:
        M.fit(0, 4, 4, 0.008856, 1.0, max_iter=1)
    assert e.value.status == _abi.E_NOCONV
    L = M.lib()
    out = _abi.Approx()
    for args in [(0, 8, 0, 0.0, 1.0), (0, 2, 2, 1.0, 0.5), (3, 3, 0, -2.0, 0.5), (0, 2, 2, -1.0, 1.0), (_abi.FN_DEC709 + 1, 2, 0, 0.0, 1.0)]:
        assert L.mact_fit(*args, ctypes.byref(out)) == _abi.E_INVALID, args
    assert L.mact_fit(0, 2, 2, 0.1, 1.0, None) == _abi.E_INVALID
    assert L.mact_last_error()


def test_paper_tables_match_the_oracle_copy(M):
    # the library and the oracle each carry a transcription of Tables 1-7; they must agree
    from oracle import tables as T
    rows = [(0, n, 0, T.T1_CBRT_POLY[n][0], T.T1_CBRT_POLY[n][1], [1.0]) for n in T.T1_CBRT_POLY]
    rows += [(0, n, m, e, p, q) for (n, m), (e, p, q) in T.T2_CBRT_RAT.items()]
    for fn, tab in ((1, T.T3_ATAN_SQRT3), (2, T.T4_ASIN2), (3, T.T5_ACOS), (4, T.T6_ATAN), (5, T.T7_ATANC)):
        rows += [(fn, n, 0, e, c, [1.0]) for n, (e, c) in tab.items()]
    for fn, n, m, e, p, q in rows:
        a = M.paper_approx(fn, n, m)
        assert a.eps == e
        assert a.p_list == list(p)
        assert a.q_list == list(q)
    from paper_1009_0854_amd import _abi
    with pytest.raises(_abi.MactError):
        M.paper_approx(0, 5, 5)


def test_default_params(M):
    want = {0: [(0, 4, 4, 0.008856, 1.0)], 1: [(1, 5, 0, 0.0, 1.0)],
            2: [(2, 5, 0, 0.0, 1 / np.sqrt(2)), (3, 5, 0, 0.0, 0.5), (4, 5, 0, 0.0, 1.0), (5, 5, 0, 0.0, 1.0)]}
    for x, fs in want.items():
        p = M.default_params(x)
        assert p.xform == x and p.out_mode == 0
        for i, (fn, n, m, lo, hi) in enumerate(fs):
            a = p.f[i]
            assert (a.fn, a.n, a.m) == (fn, n, m)
            assert a.lo == pytest.approx(lo) and a.hi == pytest.approx(hi)
            assert a.converged == 1 and 0 < a.eps < 2e-4


def test_host_entry_points_are_reentrant(M):
    # fits, weighted fits and the default approximations called from 8 host threads at once
    # (ctypes drops the interpreter lock for the call) give the single-threaded results, and a
    # failing call's detail string stays on its own thread
    import threading
    from paper_1009_0854_amd import _abi
    jobs = [(0, 4, 4, 0.008856, 1.0, None), (4, 5, 0, 0.0, 1.0, None), (6, 7, 0, 0.0, np.pi / 2, None),
            (0, 3, 3, 0.008856, 1.0, (0.5, 0.01))]

    def run(job):
        fn, n, m, lo, hi, w = job
        a = M.fit(fn, n, m, lo, hi, weight=None if w is None else M.dark_end_weight(*w))
        return list(a.p_list), list(a.q_list), a.eps

    want = [run(j) for j in jobs]
    got, errs = {}, {}

    def worker(t):
        L = M.lib()
        for r in range(3):
            for i, j in enumerate(jobs):
                got[(t, r, i)] = run(j)
            assert M.default_params(t % 4).xform == t % 4
            st = L.mact_fit(0, 9, 0, 0.0, 1.0, None)  # invalid: this thread's own error text
            errs[(t, r)] = (st, L.mact_last_error())

    ts = [threading.Thread(target=worker, args=(t,)) for t in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert len(got) == 8 * 3 * len(jobs)
    for (t, r, i), v in got.items():
        assert v == want[i], (t, r, i)
    for st, msg in errs.values():
        assert st == _abi.E_INVALID and (b"out is NULL" in msg or b"degrees" in msg), msg


def _img(data=1, dtype=0, layout=0, w=4, h=3, **kw):
    from paper_1009_0854_amd import _abi
    im = _abi.Image()
    im.data, im.dtype, im.layout, im.width, im.height = data, dtype, layout, w, h
    for k, v in kw.items():
        setattr(im, k, v)
    return im


def test_transform_validation_without_gpu(M):
    from paper_1009_0854_amd import _abi as A
    L = M.lib()
    p = M.default_params(0)
    ok_in, ok_out = _img(0x1000, A.U8), _img(0x2000, A.F32)
    cases = [
        (None, ok_in, ok_out, A.E_INVALID),
        (p, _img(0, A.U8), ok_out, A.E_INVALID),                 # NULL data
        (p, _img(0x1000, A.U8, w=0), ok_out, A.E_INVALID),         # empty
        (p, _img(0x1000, 7), ok_out, A.E_INVALID),                 # dtype
        (p, _img(0x1000, A.U8, layout=3), ok_out, A.E_INVALID),    # layout
        (p, ok_in, _img(0x2000, A.U8), A.E_UNSUPPORTED),           # 8-bit output
        (p, ok_in, _img(0x2000, A.F32, w=5), A.E_INVALID),         # shape mismatch
        (p, _img(0x1000, A.U8, row_stride=5), ok_out, A.E_INVALID),  # stride < 3 W
        (p, _img(0x1000, A.U8, gamma=9), ok_out, A.E_INVALID),     # gamma
    ]
    for params, i, o, want in cases:
        pp = ctypes.byref(params) if params is not None else None
        assert L.mact_transform(pp, ctypes.byref(i), ctypes.byref(o), None) == want
        assert L.mact_last_error()
    bad = M.default_params(1)
    bad.out_mode = 1
    assert L.mact_transform(ctypes.byref(bad), ctypes.byref(ok_in), ctypes.byref(ok_out), None) == A.E_INVALID
    bad = M.default_params(1)
    bad.f[0].m = 2
    assert L.mact_transform(ctypes.byref(bad), ctypes.byref(ok_in), ctypes.byref(ok_out), None) == A.E_UNSUPPORTED
    bad = M.default_params(0)
    bad.f[0].n = 8
    assert L.mact_transform(ctypes.byref(bad), ctypes.byref(ok_in), ctypes.byref(ok_out), None) == A.E_INVALID
    bad = M.default_params(0)
    bad.xform = 5
    assert L.mact_transform(ctypes.byref(bad), ctypes.byref(ok_in), ctypes.byref(ok_out), None) == A.E_INVALID
    # backward: float32 linear only
    x = _img(0x1000, A.F32, gamma=A.GAMMA_NONE)
    assert L.mact_transform_backward(ctypes.byref(p), ctypes.byref(_img(0x1000, A.U8, gamma=A.GAMMA_NONE)),
                                     ctypes.byref(x), ctypes.byref(x), None) == A.E_UNSUPPORTED
    assert L.mact_transform_backward(ctypes.byref(p), ctypes.byref(_img(0x1000, A.F32)),
                                     ctypes.byref(x), ctypes.byref(x), None) == A.E_UNSUPPORTED
    hp = M.default_params(1)
    assert L.mact_transform_backward(ctypes.byref(hp), ctypes.byref(x), ctypes.byref(x), ctypes.byref(x), None) == A.E_UNSUPPORTED


def test_lut_validation_without_gpu(M):
    from paper_1009_0854_amd import _abi as A
    L = M.lib()
    assert L.lut_bytes(0, 17) == 17 ** 3 * 16
    assert L.lut_bytes(1, 33) == 33 ** 3 * 16
    assert L.lut_bytes(2, 17) == 17 ** 3 * 16 + (17 ** 3 + 3) // 4 * 16  # SCT: float4 angles + L plane
    assert L.lut_bytes(2, 9) == 9 ** 3 * 16 + (9 ** 3 + 3) // 4 * 16
    assert L.lut_bytes(0, 1) == 0 and L.lut_bytes(4, 17) == 0 and L.lut_bytes(0, 257) == 0
    assert L.lut_build(0, 1, 0, ctypes.c_void_p(0x1000), 1 << 20, None) == A.E_INVALID
    assert L.lut_build(0, 17, 0, None, 1 << 20, None) == A.E_INVALID
    assert L.lut_build(0, 17, 0, ctypes.c_void_p(0x1000), 100, None) == A.E_INVALID
    i, o = _img(0x1000, A.U8), _img(0x2000, A.F32)
    assert L.lut_interp(ctypes.c_void_p(0x1000), 17, 0, 7, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    assert L.lut_interp(ctypes.c_void_p(0x1004), 17, 0, 0, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    assert L.lut_interp(None, 17, 0, 0, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    # cell-major form: (N-1)^3 cells of 8 nodes
    assert L.lut_cells_bytes(0, 17) == 16 ** 3 * 8 * 16
    assert L.lut_cells_bytes(2, 33) == 32 ** 3 * 8 * 20
    assert L.lut_cells_bytes(0, 2) == 8 * 16
    assert L.lut_cells_bytes(0, 1) == 0 and L.lut_cells_bytes(4, 17) == 0 and L.lut_cells_bytes(1, 257) == 0
    need = L.lut_cells_bytes(0, 17)
    assert L.lut_cells_build(ctypes.c_void_p(0x1000), 17, 0, ctypes.c_void_p(0x2000), need - 1, None) == A.E_INVALID
    assert L.lut_cells_build(None, 17, 0, ctypes.c_void_p(0x2000), need, None) == A.E_INVALID
    assert L.lut_cells_build(ctypes.c_void_p(0x1000), 17, 0, ctypes.c_void_p(0x2008), need, None) == A.E_INVALID
    assert L.lut_cells_build(ctypes.c_void_p(0x1000), 300, 0, ctypes.c_void_p(0x2000), need, None) == A.E_INVALID
    assert L.lut_cells_interp(ctypes.c_void_p(0x1000), 17, 0, 9, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    assert L.lut_cells_interp(ctypes.c_void_p(0x1008), 17, 0, 0, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    assert L.lut_cells_interp(None, 17, 0, 0, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    # caching form: (N-1)^3 records of 13 entries of 3 (LAB, LUV), 4 (HSI) or 5 (SCT) floats; 33^3
    # LAB in float32 is 5.1 MB (the paper's 10.7 MB counts 33^3 nodes in FP64)
    assert L.lut_cache_bytes(0, 33) == 32 ** 3 * 13 * 3 * 4 == 5111808
    assert L.lut_cache_bytes(1, 17) == 16 ** 3 * 13 * 4 * 4
    assert L.lut_cache_bytes(2, 9) == 8 ** 3 * 13 * 5 * 4
    assert L.lut_cache_bytes(3, 2) == (13 * 3 * 4 + 15) // 16 * 16
    assert L.lut_cache_bytes(0, 1) == 0 and L.lut_cache_bytes(4, 17) == 0 and L.lut_cache_bytes(0, 257) == 0
    need = L.lut_cache_bytes(0, 17)
    assert L.lut_cache_build(0, 17, 0, None, need, None) == A.E_INVALID
    assert L.lut_cache_build(0, 17, 0, ctypes.c_void_p(0x2008), need, None) == A.E_INVALID
    assert L.lut_cache_build(0, 17, 0, ctypes.c_void_p(0x2000), need - 1, None) == A.E_INVALID
    assert L.lut_cache_build(0, 17, 5, ctypes.c_void_p(0x2000), need, None) == A.E_INVALID
    assert L.lut_cache_build(5, 17, 0, ctypes.c_void_p(0x2000), need, None) == A.E_INVALID
    assert L.lut_cache_interp(ctypes.c_void_p(0x1000), 17, 0, 9, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    assert L.lut_cache_interp(ctypes.c_void_p(0x1008), 17, 0, 0, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    assert L.lut_cache_interp(None, 17, 0, 0, ctypes.byref(i), ctypes.byref(o), None) == A.E_INVALID
    assert b"lut_cache_interp" in L.mact_last_error()


def test_batch_and_server_validation_without_gpu(M):
    from paper_1009_0854_amd import _abi as A
    L = M.lib()
    p = (A.Params * 1)(M.default_params(0))
    i = (A.Image * 1)(_img(0x1000, A.U8))
    o = (A.Image * 1)(_img(0x2000, A.F32))
    h = ctypes.c_void_p()
    assert L.mact_batch_plan_create(p, i, o, 0, None, None, ctypes.byref(h)) == A.E_INVALID
    t = A.Tune(100, 4096, 4, 32)
    assert L.mact_batch_plan_create(p, i, o, 1, ctypes.byref(t), None, ctypes.byref(h)) == A.E_INVALID
    t = A.Tune(256, 1000, 4, 32)
    assert L.mact_batch_plan_create(p, i, o, 1, ctypes.byref(t), None, ctypes.byref(h)) == A.E_INVALID
    t = A.Tune(256, 4096, 3, 32)
    assert L.mact_batch_plan_create(p, i, o, 1, ctypes.byref(t), None, ctypes.byref(h)) == A.E_INVALID
    for w in (-1, 65):
        t = A.Tune(256, 4096, 4, w)
        assert L.mact_batch_plan_create(p, i, o, 1, ctypes.byref(t), None, ctypes.byref(h)) == A.E_INVALID
    for one in (-1, 2):
        t = A.Tune(256, 4096, 4, 32, one)
        assert L.mact_batch_plan_create(p, i, o, 1, ctypes.byref(t), None, ctypes.byref(h)) == A.E_INVALID
        assert b"one_launch" in L.mact_last_error()
    cfg = A.ServerConfig()
    cfg.arena_bytes, cfg.max_batch, cfg.compute_streams, cfg.max_queue = 1 << 30, 64, 2, 100
    for x in range(3):
        cfg.params[x] = M.default_params(x)
    bad = A.ServerConfig.from_buffer_copy(cfg)
    bad.compute_streams = 9
    assert L.mact_server_create(ctypes.byref(bad), ctypes.byref(h)) == A.E_INVALID
    bad = A.ServerConfig.from_buffer_copy(cfg)
    bad.arena_bytes = 1000
    assert L.mact_server_create(ctypes.byref(bad), ctypes.byref(h)) == A.E_INVALID
    bad = A.ServerConfig.from_buffer_copy(cfg)
    bad.params[1] = M.default_params(0)
    assert L.mact_server_create(ctypes.byref(bad), ctypes.byref(h)) == A.E_INVALID
    bad = A.ServerConfig.from_buffer_copy(cfg)
    bad.fail_request = -1
    assert L.mact_server_create(ctypes.byref(bad), ctypes.byref(h)) == A.E_INVALID
    assert L.mact_server_cancel(None, 1) == A.E_INVALID


def test_server_submit_refuses_mismatched_host_tensors(M):
    # the engine copies H W 3 elements into and out of the two host tensors, so the binding
    # refuses anything but two contiguous (H, W, 3) host tensors of one shape
    torch = pytest.importorskip("torch")
    x = torch.zeros((4, 5, 3), dtype=torch.uint8)
    y = torch.zeros((4, 5, 3), dtype=torch.float32)
    M.check_request_tensors(x, y)
    bad = [
        (x, torch.zeros((4, 4, 3), dtype=torch.float32)),           # smaller output
        (x, torch.zeros((5, 4, 3), dtype=torch.float32)),           # same size, other shape
        (torch.zeros((3, 4, 5), dtype=torch.uint8), torch.zeros((3, 4, 5))),  # CHW
        (x.reshape(20, 3), y.reshape(20, 3)),                       # not (H, W, 3)
        (torch.zeros((4, 6, 3), dtype=torch.uint8)[:, :5], y),      # strided input
        (x, torch.zeros((4, 6, 3))[:, :5]),                         # strided output
        (x, torch.zeros((4, 5, 3, 1))[..., 0]),                     # a view that happens to be fine
    ]
    for k, (a, b) in enumerate(bad[:-1]):
        with pytest.raises(ValueError):
            M.check_request_tensors(a, b)
    M.check_request_tensors(*bad[-1])


def test_fast_division_method():
    # the round-up multiplier division the kernels use for pixel coordinates
    def make(d):
        l = 0
        while (1 << l) < d:
            l += 1
        return ((1 << 32) * ((1 << l) - d)) // d + 1, l

    g = np.random.default_rng(0)
    for d in [1, 2, 3, 5, 7, 255, 256, 1920, 1080 * 1920, 4096 * 4096, 2 ** 31 - 1]:
        m, s = make(d)
        n = np.concatenate([g.integers(0, 2 ** 32, 20000, dtype=np.uint64), np.arange(0, 5000, dtype=np.uint64),
                            np.array([2 ** 32 - 1, d, d - 1, 2 * d, 2 * d - 1], dtype=np.uint64)])
        n = n[n < 2 ** 32]
        q = (((n * np.uint64(m)) >> np.uint64(32)) + n) >> np.uint64(s)
        np.testing.assert_array_equal(q, n // np.uint64(d))


def test_exact_baseline_validation_without_gpu(M):
    from paper_1009_0854_amd import _abi as A
    L = M.lib()
    u8, f32, o32 = _img(0x1000, A.U8), _img(0x1000, A.F32), _img(0x2000, A.F32)
    assert L.mact_transform_exact(4, ctypes.byref(u8), ctypes.byref(o32), None) == A.E_INVALID
    assert L.mact_transform_exact(-1, ctypes.byref(u8), ctypes.byref(o32), None) == A.E_INVALID
    assert L.mact_transform_exact(0, ctypes.byref(f32), ctypes.byref(o32), None) == A.E_UNSUPPORTED
    chw = _img(0x1000, A.U8, layout=A.CHW)
    assert L.mact_transform_exact(0, ctypes.byref(chw), ctypes.byref(o32), None) == A.E_UNSUPPORTED
    assert L.mact_transform_exact(0, None, ctypes.byref(o32), None) == A.E_INVALID
    assert L.mact_transform_exact(0, ctypes.byref(u8), ctypes.byref(_img(0x2000, A.U8)), None) == A.E_UNSUPPORTED
    assert b"mact_transform_exact" in L.mact_last_error()


def test_inverse_and_error_stats_validation_without_gpu(M):
    # every case is rejected before any launch
    from paper_1009_0854_amd import _abi as A
    L = M.lib()
    i32, o32 = _img(0x1000, A.F32), _img(0x2000, A.F32)
    p = M.inverse_params("sct")
    assert p.f[0].fn == A.FN_SIN and p.f[1].fn == A.FN_COS and p.f[0].n == 7
    assert M.inverse_params("hsi").f[0].fn == A.FN_COS and M.inverse_params("hsi").f[0].hi == pytest.approx(2 * np.pi / 3)
    assert M.inverse_params("lab").f[0].fn == A.FN_ENC709 and M.inverse_params("lab").f[0].m == 4
    assert L.mact_inverse(None, ctypes.byref(i32), ctypes.byref(o32), None) == A.E_INVALID
    assert L.mact_inverse(ctypes.byref(p), ctypes.byref(_img(0x1000, A.U8)), ctypes.byref(o32), None) == A.E_UNSUPPORTED
    bad = M.inverse_params("sct")
    bad.f[0], bad.f[1] = bad.f[1], bad.f[0]  # cosine where the sine belongs
    assert L.mact_inverse(ctypes.byref(bad), ctypes.byref(i32), ctypes.byref(o32), None) == A.E_INVALID
    srgb = _img(0x2000, A.F32)
    srgb.gamma = A.GAMMA_SRGB
    assert L.mact_inverse(ctypes.byref(M.inverse_params("lab")), ctypes.byref(i32), ctypes.byref(srgb), None) == A.E_UNSUPPORTED
    assert L.mact_inverse(ctypes.byref(M.inverse_params("luv")), ctypes.byref(i32), ctypes.byref(srgb), None) == A.E_UNSUPPORTED
    luv = M.inverse_params("luv")
    assert luv.xform == A.LUV and luv.f[0].fn == A.FN_ENC709 and luv.f[0].m == 4
    luv.f[0] = M.inverse_params("hsi").f[0]  # cosine where the encoding belongs
    assert L.mact_inverse(ctypes.byref(luv), ctypes.byref(i32), ctypes.byref(o32), None) == A.E_INVALID
    assert L.mact_inverse_params_default(4, ctypes.byref(luv)) == A.E_INVALID
    e = A.ErrorStats()
    assert L.mact_error_stats(ctypes.byref(M.default_params(0)), ctypes.byref(i32), None, None) == A.E_INVALID
    assert L.mact_error_stats(None, ctypes.byref(i32), ctypes.byref(e), None) == A.E_INVALID
    dbg = M.default_params(0)
    dbg.out_mode = 1
    assert L.mact_error_stats(ctypes.byref(dbg), ctypes.byref(i32), ctypes.byref(e), None) == A.E_INVALID
    # the allocation-free form validates the same way, before it looks up its device record
    assert L.mact_error_stats_noalloc(ctypes.byref(M.default_params(0)), ctypes.byref(i32), None, None) == A.E_INVALID
    assert L.mact_error_stats_noalloc(None, ctypes.byref(i32), ctypes.byref(e), None) == A.E_INVALID
    assert L.mact_error_stats_noalloc(ctypes.byref(dbg), ctypes.byref(i32), ctypes.byref(e), None) == A.E_INVALID
    assert b"mact_error_stats_noalloc" in L.mact_last_error()
