"""Pins of the oracle's exact transforms against what the paper and the
mathematics fix (CPU only)."""
import numpy as np
import pytest

from oracle import colour, tables
from tests.cubepool import cube_map


def test_d65_white_maps_to_l100():
    # the BT.709 matrix rows sum to the D65 white, so white has t = 1 and f = 1
    lab = colour.rgb_to_lab(np.array([1.0, 1.0, 1.0]))
    np.testing.assert_allclose(lab, [100.0, 0.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(colour.M_RGB_XYZ.sum(axis=1), colour.WHITE_D65, rtol=0, atol=1e-15)
    lab = colour.rgb_to_lab(np.array([1.0, 1.0, 1.0]), gamma="srgb")
    np.testing.assert_allclose(lab, [100.0, 0.0, 0.0], atol=1e-12)


def test_black_and_grays():
    np.testing.assert_allclose(colour.rgb_to_lab(np.zeros(3)), [0.0, 0.0, 0.0], atol=1e-12)
    # a gray has a* = b* = 0 because X/X0 = Y/Y0 = Z/Z0
    for v in (0.01, 0.2, 0.5, 0.9):
        lab = colour.rgb_to_lab(np.full(3, v))
        assert abs(lab[1]) < 1e-12 and abs(lab[2]) < 1e-12


def test_lab_f_is_continuous_at_breakpoint():
    t0 = colour.LAB_T0
    assert abs(np.cbrt(t0) - (colour.LAB_K * t0 + colour.LAB_C)) < 2e-6


def test_bt709_inverse_gamma_values():
    g = colour.inverse_gamma(np.array([0.0, 0.0405, 1.0]))
    np.testing.assert_allclose(g, [0.0, 0.009, 1.0], atol=1e-15)
    # the two branches nearly meet at 0.081
    lo = 0.081 / 4.5
    hi = ((0.081 + 0.099) / 1.099) ** (1 / 0.45)
    assert abs(lo - hi) < 1e-4


def test_srgb_transfer_function_values():
    # IEC 61966-2-1 (the sRGB option): decoding k/12.92 up to 0.04045, ((k + 0.055)/1.055)^2.4 above.
    # Pins that do not restate the formula:
    #  - the two decoding branches meet at the breakpoint 0.04045 (to 2.3e-9), and the two
    #    encoding branches at its image 0.0031308;
    #  - tabulated values of the standard's curve: code 0.5 decodes to 0.2140411, the 8-bit code 128
    #    to 0.2158605, and 18% linear grey encodes to 0.4613561;
    #  - 8-bit mid grey (128, 128, 128) has L* = 53.585 (Y = 0.2158605 relative to white).
    # A consistent wrong exponent pair (2.2 and 1/2.2) passes a round trip but none of these.
    lo = colour.inverse_gamma(np.array([0.04045 - 1e-12]), "srgb")[0]
    hi = colour.inverse_gamma(np.array([0.04045 + 1e-12]), "srgb")[0]
    assert abs(lo - hi) < 1e-8
    assert abs(lo - 0.0031308) < 1e-7
    elo = colour.encode_gamma(np.array([0.0031308 - 1e-12]), "srgb")[0]
    ehi = colour.encode_gamma(np.array([0.0031308 + 1e-12]), "srgb")[0]
    assert abs(elo - ehi) < 1e-7 and abs(elo - 0.04045) < 1e-6
    np.testing.assert_allclose(colour.inverse_gamma(np.array([0.5, 128 / 255.0, 1.0, 0.0]), "srgb"),
                               [0.2140411, 0.2158605, 1.0, 0.0], atol=1e-7)
    np.testing.assert_allclose(colour.encode_gamma(np.array([0.18, 0.2140411405]), "srgb"), [0.4613561, 0.5],
                               atol=1e-7)
    lab = colour.rgb_to_lab(np.full(3, 128 / 255.0), gamma="srgb")
    np.testing.assert_allclose(lab, [53.585, 0.0, 0.0], atol=1e-3)
    # the linear segment below the breakpoint: slope 1/12.92 through the origin
    np.testing.assert_allclose(colour.inverse_gamma(np.array([0.02, -0.01]), "srgb"),
                               [0.02 / 12.92, -0.01 / 12.92], rtol=1e-15)


def _cbrt_counts(v8):
    t = colour.lab_t(v8 / 255.0)
    return (t > colour.LAB_T0).sum(axis=0)


def test_cbrt_call_probabilities_over_all_colours():
    # Sec. 3.2.2: the probabilities of the cube-root branch over all 2^24 colours
    counts = sum(cube_map(_cbrt_counts))
    p = counts / float(1 << 24)
    np.testing.assert_allclose(p, tables.P_CBRT, atol=6e-7)


def test_hsi_primaries_secondaries_and_gray():
    cases = {
        (1, 0, 0): (0.0, 1.0, 1 / 3), (0, 1, 0): (2 * np.pi / 3, 1.0, 1 / 3), (0, 0, 1): (4 * np.pi / 3, 1.0, 1 / 3),
        (1, 1, 0): (np.pi / 3, 1.0, 2 / 3), (0, 1, 1): (np.pi, 1.0, 2 / 3), (1, 0, 1): (5 * np.pi / 3, 1.0, 2 / 3),
        (0.5, 0.5, 0.5): (0.0, 0.0, 0.5), (0, 0, 0): (0.0, 0.0, 0.0), (1, 1, 1): (0.0, 0.0, 1.0),
    }
    for rgb, want in cases.items():
        for fn in (colour.rgb_to_hsi, colour.rgb_to_hsi_kender):
            np.testing.assert_allclose(fn(np.array(rgb, dtype=float)), want, atol=1e-12, err_msg=str((fn, rgb)))


def _kender_vs_arccos(v8):
    x = v8 / 255.0
    a = colour.rgb_to_hsi(x)[..., 0]
    b = colour.rgb_to_hsi_kender(x)[..., 0]
    return float(colour.angle_diff(a, b).max())


def test_kender_equals_arccos_definition_over_all_colours():
    # Sec. 3.3.1: Kender's form gives the same hue as the arccos definition
    assert max(cube_map(_kender_vs_arccos)) < 1e-12


def _sct_stats(v8):
    x = v8 / 255.0
    s = colour.rgb_to_sct(x)
    back = colour.sct_to_rgb(s)
    rt = float(np.abs(back - x).max())
    R, G, B = v8[:, 0].astype(np.int64), v8[:, 1].astype(np.int64), v8[:, 2].astype(np.int64)
    upper = int(((3 * B * B >= R * R + G * G) & ((R + G + B) > 0)).sum())
    atan_calls = int((~((R == 0) & (G == 0))).sum())
    # the arctan form of angle B equals the arccos form where L sin A > 0; the
    # arccos form is ill-conditioned near angle 0, so compare the cosines
    ok = (R > 0) | (G > 0)
    d = np.cos(colour.rgb_to_sct_arccos(x[ok])[..., 2]) - np.cos(s[ok][..., 2])
    return rt, upper, atan_calls, float(np.abs(d).max())


def test_sct_round_trip_probabilities_and_arctan_form():
    parts = cube_map(_sct_stats)
    assert max(p[0] for p in parts) < 1e-13
    n = float(1 << 24)
    # Sec. 3.4.3: P(B/L >= 0.5) and P(arctan called); black (L = 0) is excluded from the former
    assert abs(sum(p[1] for p in parts) / n - tables.P_ARCSIN) < 6e-7
    assert abs(sum(p[2] for p in parts) / n - tables.P_ARCTAN) < 6e-7
    assert abs(sum(p[2] for p in parts) / n - (1 - 256.0 / 256 ** 3)) < 1e-15
    assert max(p[3] for p in parts) < 1e-10


def test_sct_special_points():
    s = colour.rgb_to_sct(np.array([[0, 0, 1.0], [1.0, 0, 0], [0, 1.0, 0], [1, 1, 1.0], [0, 0, 0.0], [0, 0.5, 0.5]]))
    np.testing.assert_allclose(s[0], [1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(s[1], [1, np.pi / 2, 0], atol=1e-15)
    np.testing.assert_allclose(s[2], [1, np.pi / 2, np.pi / 2], atol=1e-15)
    np.testing.assert_allclose(s[3], [np.sqrt(3), np.arccos(1 / np.sqrt(3)), np.pi / 4], atol=1e-15)
    np.testing.assert_allclose(s[4], [0, 0, 0], atol=0)
    np.testing.assert_allclose(s[5], [np.sqrt(0.5), np.pi / 4, np.pi / 2], atol=1e-15)


def test_metrics():
    assert colour.delta_e(np.array([0, 0, 0.0]), np.array([3, 4, 0.0])) == 5.0
    # hue difference wraps through 0
    a = np.array([0.1, 0.5, 0.4])
    b = np.array([2 * np.pi - 0.1, 0.5, 0.4])
    assert colour.d_hsi(a, b) == pytest.approx(2 * 0.5 * np.sin(0.1), rel=1e-12)
    # opposite hues at equal saturation: distance 2s
    a = np.array([0.0, 0.3, 0.2])
    b = np.array([np.pi, 0.3, 0.2])
    assert colour.d_hsi(a, b) == pytest.approx(0.6, rel=1e-12)
    # the SCT metric of identical triples is zero; of a pure L change it is the CIELAB change
    s = colour.rgb_to_sct(np.array([0.3, 0.4, 0.5]))
    assert colour.sct_delta_e(s, s) == 0.0
    s2 = s.copy()
    s2[0] *= 0.5
    want = colour.delta_e(colour.rgb_to_lab(np.array([0.15, 0.2, 0.25])), colour.rgb_to_lab(np.array([0.3, 0.4, 0.5])))
    assert colour.sct_delta_e(s, s2) == pytest.approx(want, rel=1e-12)
