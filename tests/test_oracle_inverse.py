"""Pins of the oracle's inverse transforms (the definitions of Sec. 3.2.1,
3.3.1 and 3.4.1 solved for R, G, B) and of their minimax-approximated forms.

The exact inverses are pinned by the forward transforms, which are themselves
pinned by the paper's tables: the round trip through every 24-bit colour must
come back to the colour.  The approximated inverses are pinned by the error
bound that follows from the approximation error of each elementary function."""
import numpy as np
import pytest

import synth
from oracle import colour as C, mact as OM, remez as R

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def cube():
    return synth.cube_u8().reshape(-1, 3) / 255.0


@pytest.mark.parametrize("gamma", ["bt709", "srgb", "none"])
def test_lab_round_trip_every_colour(cube, gamma):
    back = C.lab_to_rgb(C.rgb_to_lab(cube, gamma), gamma)
    assert np.abs(back - cube).max() < 1e-12


@pytest.mark.parametrize("gamma", ["bt709", "none"])
def test_luv_round_trip_every_colour(cube, gamma):
    back = C.luv_to_rgb(C.rgb_to_luv(cube, gamma), gamma)
    assert np.abs(back - cube).max() < 1e-12


def test_luv_inverse_special_values():
    # white, black, grays (u* = v* = 0 is the white's chromaticity at every lightness)
    assert np.allclose(C.luv_to_rgb(np.array([100.0, 0.0, 0.0])), 1.0, atol=1e-12)
    assert np.array_equal(C.luv_to_rgb(np.array([0.0, 0.0, 0.0])), [0.0, 0.0, 0.0])
    for L in (1.0, 8.0, 50.0, 99.0):
        rgb = C.luv_to_rgb(np.array([L, 0.0, 0.0]), "none")
        assert np.allclose(rgb, rgb[0], atol=1e-13)
    # Y of the definition: the luminance row of the matrix applied to linear RGB
    lin = synth.rng(3).random((1000, 3))
    xyz = C.luv_to_xyz(C.rgb_to_luv(lin, "none"))
    assert np.allclose(xyz[:, 1], lin @ C.M_RGB_XYZ[1], atol=1e-13)


def test_hsi_round_trip_every_colour(cube):
    back = C.hsi_to_rgb(C.rgb_to_hsi(cube))
    assert np.abs(back - cube).max() < 1e-12


def test_sct_round_trip_every_colour(cube):
    back = C.sct_to_rgb(C.rgb_to_sct(cube))
    assert np.abs(back - cube).max() < 1e-12


def test_inverse_special_values():
    # white, black and grays, the primaries
    assert np.allclose(C.lab_to_rgb(np.array([100.0, 0.0, 0.0])), 1.0, atol=1e-12)
    assert np.allclose(C.lab_to_rgb(np.array([0.0, 0.0, 0.0])), 0.0, atol=1e-15)
    for v in (0.0, 0.25, 1.0):
        assert np.allclose(C.hsi_to_rgb(np.array([0.0, 0.0, v])), v, atol=1e-15)
        assert np.allclose(C.hsi_to_rgb(np.array([4.0, 0.0, v])), v, atol=1e-15)  # hue irrelevant on gray
    third = 1.0 / 3.0
    assert np.allclose(C.hsi_to_rgb(np.array([0.0, 1.0, third])), [1, 0, 0], atol=1e-15)
    assert np.allclose(C.hsi_to_rgb(np.array([2 * np.pi / 3, 1.0, third])), [0, 1, 0], atol=1e-15)
    assert np.allclose(C.hsi_to_rgb(np.array([4 * np.pi / 3, 1.0, third])), [0, 0, 1], atol=1e-15)
    assert np.allclose(C.sct_to_rgb(np.array([1.0, 0.0, 0.0])), [0, 0, 1], atol=1e-15)
    assert np.allclose(C.sct_to_rgb(np.array([1.0, np.pi / 2, 0.0])), [1, 0, 0], atol=1e-15)


@pytest.mark.parametrize("kind", ["bt709", "srgb"])
def test_encode_inverts_decode_on_both_branches(kind):
    k = np.linspace(-0.05, 1.2, 20001)
    if kind == "bt709":
        # with the printed constants the decoding jumps down at 0.081: ((0.081 + 0.099) / 1.099)^(1/0.45)
        # = 0.0179866 < 0.081 / 4.5, so codes in [0.081, 0.0811876) decode below the encoding breakpoint
        # 0.018 and come back on the linear branch; no 8-bit code falls there (20/255 < 0.081 < 21/255)
        top = 1.099 * (0.081 / 4.5) ** 0.45 - 0.099
        band = (k >= 0.081) & (k < top)
        assert band.any() and not np.any((np.arange(256) / 255.0 >= 0.081) & (np.arange(256) / 255.0 < top))
        k = k[~band]
    assert np.abs(C.encode_gamma(C.inverse_gamma(k, kind), kind) - k).max() < 1e-13


def test_lab_f_inverse_and_the_gap_reading():
    t = np.concatenate([np.linspace(-0.01, 0.0088, 5001), np.linspace(0.0088, 0.0089, 5001),
                        np.linspace(0.0089, 2.0, 5001), [C.LAB_T0, np.nextafter(C.LAB_T0, 1.0)]])
    assert np.abs(C.lab_f_inv(C.lab_f(t)) - t).max() < 1e-13
    # f jumps up at the breakpoint (7.787 * 0.008856 + 16/116 < cbrt(0.008856)); f in the gap is
    # never produced and takes the linear branch
    lo, hi = C.LAB_K * C.LAB_T0 + C.LAB_C, np.cbrt(C.LAB_T0)
    assert lo < hi
    f = np.linspace(lo, hi, 11)[1:-1]
    assert np.array_equal(C.lab_f_inv(f), (f - C.LAB_C) / C.LAB_K)


@pytest.fixture(scope="module")
def fits():
    enc = R.remez(lambda x: 1.099 * x ** 0.45 - 0.099, 4, 4, 0.018, 1.0)
    sin = R.remez(np.sin, 7, 0, 0.0, np.pi / 2)
    cos = R.remez(np.cos, 7, 0, 0.0, np.pi / 2)
    cos_h = R.remez(np.cos, 7, 0, 0.0, 2 * np.pi / 3)
    return enc, sin, cos, cos_h


def test_mact_lab_inverse_within_the_encoding_error(cube, fits):
    enc = fits[0]
    lab = C.rgb_to_lab(cube)
    got = OM.mact_lab_inverse(lab, enc.p, enc.q)
    assert np.abs(got - cube).max() <= enc.eps * (1 + 1e-6) + 1e-12
    lin = OM.mact_lab_inverse(lab, enc.p, enc.q, gamma="none")
    assert np.abs(lin - C.inverse_gamma(cube)).max() < 1e-12


def test_mact_luv_inverse_within_the_encoding_error(cube, fits):
    enc = fits[0]
    luv = C.rgb_to_luv(cube)
    got = OM.mact_luv_inverse(luv, enc.p, enc.q)
    assert np.abs(got - cube).max() <= enc.eps * (1 + 1e-6) + 1e-12
    assert np.abs(got - cube).max() > 0.3 * enc.eps
    lin = OM.mact_luv_inverse(luv, enc.p, enc.q, gamma="none")
    assert np.abs(lin - C.inverse_gamma(cube)).max() < 1e-12


def test_mact_hsi_inverse_within_its_bound(cube, fits):
    # start = I (1 + S c1 / c2) with |c1 - cos|, |c2 - cos| <= eps and cos(pi/3 - h) >= 1/2:
    # the ratio is off by at most 6 eps (+ rounding), the third channel by twice that
    cos_h = fits[3]
    got = OM.mact_hsi_inverse(C.rgb_to_hsi(cube), cos_h.p)
    assert np.abs(got - cube).max() <= 12 * cos_h.eps * 1.01


def test_mact_sct_inverse_within_its_bound(cube, fits):
    sin, cos = fits[1], fits[2]
    eps = max(sin.eps, cos.eps)
    sct = C.rgb_to_sct(cube)
    got = OM.mact_sct_inverse(sct, sin.p, cos.p)
    bound = sct[:, 0] * (2 * eps + eps * eps) + 1e-12
    assert np.all(np.abs(got - cube).max(axis=1) <= bound)


def test_mact_inverse_approximations_are_not_exact(cube, fits):
    # the bound tests above would pass with the exact functions too; the approximated
    # inverses must actually use the polynomials (errors of the order of eps, not zero)
    enc, sin, cos, cos_h = fits
    assert np.abs(OM.mact_lab_inverse(C.rgb_to_lab(cube), enc.p, enc.q) - cube).max() > 0.3 * enc.eps
    assert np.abs(OM.mact_sct_inverse(C.rgb_to_sct(cube), sin.p, cos.p) - cube).max() > 0.3 * sin.eps


def test_mact_decode709_within_its_error(fits):
    # the decoding polynomial replaces the power above 0.081 only, within its eps there
    dec = R.remez(lambda x: ((x + 0.099) / 1.099) ** (1 / 0.45), 7, 0, 0.081, 1.0)
    k = np.linspace(0.0, 1.0, 100001)
    d = np.abs(OM.mact_decode709(k, dec.p) - C.inverse_gamma(k))
    assert d.max() <= dec.eps * (1 + 1e-6)
    assert np.all(d[k < 0.081] == 0.0)
    # CIELAB through the approximated decoding: L* moves by at most 116 * f'(t) * |dt|, f' <= 7.787,
    # |dt| <= eps (Y is a convex combination of the channels); checked on the cube against the bound
    cube = synth.cube_u8().reshape(-1, 3)[::5] / 255.0
    from oracle import tables as T
    cb = R.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL)
    a = OM.mact_lab(cube, cb.p, cb.q, decode=dec.p)
    b = OM.mact_lab(cube, cb.p, cb.q)
    assert np.abs(a[:, 0] - b[:, 0]).max() <= 116 * 7.787 * dec.eps * 1.01
    assert np.abs(a - b).max() > 0
