"""The oracle reproduces the transformation errors the paper prints for all
2^24 8-bit colours (Tables 8, 9, 10 and 12).  CPU only; each test sweeps the
whole colour cube in a process pool."""
import numpy as np
import pytest

from oracle import colour, lut, mact, remez, tables as T
from tests.cubepool import cube_map, mean_max, sum_max


def _t8(v8):
    x = v8 / 255.0
    ex = colour.rgb_to_lab(x)
    out = {}
    for key, (_, p, q) in T.T2_CBRT_RAT.items():
        out[key] = sum_max(colour.delta_e(mact.mact_lab(x, p, q), ex))
    return out


def test_table8_cielab_errors_with_printed_rationals():
    parts = cube_map(_t8)
    for key, (avg, mx) in T.T8_CIELAB_ERR.items():
        got_avg, got_max = mean_max([p[key] for p in parts])
        # the printed rows agree to the 5th-6th digit (the printed coefficients have 7)
        assert got_avg == pytest.approx(avg, abs=6e-6), key
        assert got_max == pytest.approx(mx, abs=6e-6), key


def _t9(v8, fits):
    x = v8 / 255.0
    ex = colour.rgb_to_hsi(x)
    return {n: sum_max(colour.d_hsi(mact.mact_hsi(x, c), ex)) for n, c in fits.items()}


def test_table9_hsi_errors_with_fits_on_0_1():
    # the maxima of Table 9 are those of arctan(sqrt 3 x) fitted on [0, 1] (the argument reaches
    # -1 when two channels tie below the third); the means agree to a few percent
    fits = {n: remez.remez(T.f_atan_sqrt3, n, 0, 0.0, 1.0).p for n in (2, 3, 4, 5)}
    parts = cube_map(_t9, fits)
    for n, (avg, mx) in T.T9_HSI_ERR.items():
        got_avg, got_max = mean_max([p[n] for p in parts])
        assert got_max == pytest.approx(mx, abs=1.5e-6), n
        # the means are printed to 6 decimals (two digits for n = 5)
        assert abs(got_avg - avg) <= 0.03 * avg + 1e-6, (n, got_avg, avg)


def _t10(v8):
    x = v8 / 255.0
    ex = colour.rgb_to_sct(x)
    ex_lab = colour.rgb_to_lab(colour.sct_to_rgb(ex))
    out = {}
    for (n, m, r) in T.T10_SCT_ERR:
        s = mact.mact_sct(x, T.T4_ASIN2[n][1], T.T5_ACOS[m][1], T.T6_ATAN[r][1], T.T7_ATANC[r][1])
        out[(n, m, r)] = sum_max(colour.delta_e(colour.rgb_to_lab(colour.sct_to_rgb(s)), ex_lab))
    return out


def test_table10_sct_errors_with_printed_polynomials():
    parts = cube_map(_t10)
    for key, (avg, mx) in T.T10_SCT_ERR.items():
        got_avg, got_max = mean_max([p[key] for p in parts])
        assert got_avg == pytest.approx(avg, abs=4e-6), key
        assert got_max == pytest.approx(mx, rel=0.01), key


def _t12(v8, luts):
    ex = colour.rgb_to_lab(v8 / 255.0)
    out = {}
    for (method, N), L in luts.items():
        o, _ = lut.interp(L, "lab", method, v8=v8)
        out[(method, N)] = sum_max(colour.delta_e(o, ex))
    return out


def test_table12_lut_errors():
    # trilinear, prism and tetrahedral reproduce every printed digit; pyramidal is unpinned
    methods = ("trilinear", "prism", "tetrahedral")
    luts = {(m, N): lut.build("lab", N) for m in methods for N in (9, 17, 33)}
    parts = cube_map(_t12, luts)
    for key in luts:
        avg, mx = T.T12_LUT_ERR[key]
        got_avg, got_max = mean_max([p[key] for p in parts])
        assert got_avg == pytest.approx(avg, abs=1e-6), key
        assert got_max == pytest.approx(mx, abs=1e-6), key


def _t12_cache(v8, caches):
    ex = colour.rgb_to_lab(v8 / 255.0)
    out = {}
    for (method, N), C in caches.items():
        o, _ = lut.interp_cache(C, "lab", method, v8=v8)
        out[(method, N)] = sum_max(colour.delta_e(o, ex))
    return out


def test_table12_lut_errors_caching_form():
    # Table 12 prints one error per method for the standard and the caching versions: the
    # caching form reproduces the same digits
    caches = {(m, N): lut.build_cache("lab", N) for m in ("trilinear", "prism", "tetrahedral") for N in (9, 33)}
    parts = cube_map(_t12_cache, caches)
    for key in caches:
        avg, mx = T.T12_LUT_ERR[key]
        got_avg, got_max = mean_max([p[key] for p in parts])
        assert got_avg == pytest.approx(avg, abs=1e-6), key
        assert got_max == pytest.approx(mx, abs=1e-6), key
