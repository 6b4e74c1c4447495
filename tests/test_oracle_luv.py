"""Pins of the oracle's CIE 1976 L*u*v* (the extension the paper names in
Sec. 4) and of its minimax-approximated form.

L* is CIELAB's L* (pinned by Table 8); u', v' are pinned by the closed forms
from the BT.709 primaries' and D65's chromaticity coordinates, which the
RGB->XYZ matrix is built from."""
import numpy as np
import pytest

import synth
from oracle import colour as C, mact as OM, remez as R, tables as T


def _uv_prime(x, y):
    d = -2.0 * x + 12.0 * y + 3.0
    return 4.0 * x / d, 9.0 * y / d


def _uv_of(luv, un, vn):
    return luv[..., 1] / (13.0 * luv[..., 0]) + un, luv[..., 2] / (13.0 * luv[..., 0]) + vn


def test_white_black_and_grays():
    assert np.allclose(C.rgb_to_luv(np.array([1.0, 1.0, 1.0])), [100.0, 0.0, 0.0], atol=1e-12)
    assert np.array_equal(C.rgb_to_luv(np.array([0.0, 0.0, 0.0])), [0.0, 0.0, 0.0])
    g = np.repeat(np.linspace(0.001, 1.0, 50)[:, None], 3, axis=1)
    luv = C.rgb_to_luv(g)
    assert np.abs(luv[:, 1:]).max() < 1e-11


def test_lightness_is_cielab_lightness_for_every_colour():
    cube = synth.cube_u8().reshape(-1, 3)[::3] / 255.0
    assert np.array_equal(C.rgb_to_luv(cube)[:, 0], C.rgb_to_lab(cube)[:, 0])


def test_chromaticity_of_the_primaries_and_the_white():
    # BT.709 primaries and D65 chromaticities (x, y); the matrix is printed to 6 digits
    un, vn = _uv_prime(0.3127, 0.3290)
    Xn, Yn, Zn = C.WHITE_D65
    assert 4 * Xn / (Xn + 15 * Yn + 3 * Zn) == pytest.approx(un, abs=2e-5)
    assert 9 * Yn / (Xn + 15 * Yn + 3 * Zn) == pytest.approx(vn, abs=2e-5)
    Xn_, Yn_, Zn_ = C.WHITE_D65
    dn = Xn_ + 15 * Yn_ + 3 * Zn_
    un_lib, vn_lib = 4 * Xn_ / dn, 9 * Yn_ / dn
    for rgb, xy in (([1, 0, 0], (0.64, 0.33)), ([0, 1, 0], (0.30, 0.60)), ([0, 0, 1], (0.15, 0.06))):
        luv = C.rgb_to_luv(np.array(rgb, dtype=float), "none")
        u, v = _uv_of(luv, un_lib, vn_lib)
        want = _uv_prime(*xy)
        assert u == pytest.approx(want[0], abs=2e-5) and v == pytest.approx(want[1], abs=2e-5), rgb


def test_mact_luv_within_the_cube_root_error():
    # only L* is approximated; u*, v* scale with L*: |du*| <= 13 |dL*| |u' - u'n| with |u' - u'n| < 1
    cb = R.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL)
    cube = synth.cube_u8().reshape(-1, 3)[::5] / 255.0
    got = OM.mact_luv(cube, cb.p, cb.q)
    ex = C.rgb_to_luv(cube)
    dL = np.abs(got[:, 0] - ex[:, 0])
    assert dL.max() <= 116 * cb.eps * (1 + 1e-6)
    assert np.abs(got[:, 1:] - ex[:, 1:]).max() <= 13 * 116 * cb.eps
    assert dL.max() > 0.3 * 116 * cb.eps  # the approximation is in use
