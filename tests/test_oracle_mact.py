"""The oracle's MACT transforms differ from the exact transforms exactly by
the approximation error of the elementary functions (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import colour, mact, remez, tables as T


@pytest.fixture(scope="module")
def fits():
    return {
        "cbrt": remez.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL),
        "atan_sqrt3": remez.remez(T.f_atan_sqrt3, 5, 0, 0.0, 1.0),
        "asin2": remez.remez(T.f_asin2, 5, 0, *T.T4_INTERVAL),
        "acos": remez.remez(T.f_acos, 5, 0, *T.T5_INTERVAL),
        "atan": remez.remez(T.f_atan, 5, 0, 0.0, 1.0),
        "atanc": remez.remez(T.f_atanc, 5, 0, 0.0, 1.0),
    }


def _inputs():
    g = synth.rng(11)
    x = g.random((200000, 3))
    v8 = synth.cube_slice(int(g.integers(0, (1 << 24) - 200000)), 200000)
    edge = np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.5, 0.5, 0.5],
                     [1, 1, 0], [0, 1, 1], [1, 0, 1], [0, 0.5, 0.5], [0.25, 0.25, 1.0]], dtype=float)
    return np.concatenate([x, v8 / 255.0, edge])


def test_lab_f_error_is_the_fit_error(fits):
    fc = fits["cbrt"]
    t = np.concatenate([np.linspace(0, 1, 200001), [colour.LAB_T0, np.nextafter(colour.LAB_T0, 1)]])
    d = np.abs(mact.mact_lab_f(t, fc.p, fc.q) - colour.lab_f(t))
    assert d.max() <= fc.eps * (1 + 1e-9)
    # at or below the breakpoint the exact linear segment is used
    lo = t <= colour.LAB_T0
    assert np.all(d[lo] == 0)


@pytest.mark.parametrize("gamma", ["bt709", "srgb", "none"])
def test_mact_lab_bound(fits, gamma):
    fc = fits["cbrt"]
    x = _inputs()
    a = mact.mact_lab(x, fc.p, fc.q, gamma=gamma)
    e = colour.rgb_to_lab(x, gamma)
    # L = 116 fy - 16, a = 500 (fx - fy), b = 200 (fy - fz): each f off by at most eps
    d = np.abs(a - e)
    eps = fc.eps * (1 + 1e-9) + 1e-13
    assert d[:, 0].max() <= 116 * eps
    assert d[:, 1].max() <= 1000 * eps
    assert d[:, 2].max() <= 400 * eps
    f = mact.mact_lab(x, fc.p, fc.q, gamma=gamma, debug=True)
    np.testing.assert_allclose(f, mact.mact_lab_f(colour.lab_t(x, gamma), fc.p, fc.q), rtol=0, atol=0)


def test_mact_hsi_bound(fits):
    fa = fits["atan_sqrt3"]
    x = _inputs()
    a = mact.mact_hsi(x, fa.p)
    e = colour.rgb_to_hsi(x)
    assert colour.angle_diff(a[:, 0], e[:, 0]).max() <= fa.eps * (1 + 1e-9) + 1e-13
    np.testing.assert_array_equal(a[:, 1:], e[:, 1:])
    # gray axis and red ray: H = 0
    g = mact.mact_hsi(np.array([[0.3, 0.3, 0.3], [0.7, 0.2, 0.2]]), fa.p)
    assert g[0, 0] == 0.0 and g[1, 0] == 0.0


def test_mact_sct_bound(fits):
    x = _inputs()
    a = mact.mact_sct(x, fits["asin2"].p, fits["acos"].p, fits["atan"].p, fits["atanc"].p)
    e = colour.rgb_to_sct(x)
    np.testing.assert_array_equal(a[:, 0], e[:, 0])
    pos = e[:, 0] > 0
    epsA = max(fits["asin2"].eps, fits["acos"].eps) * (1 + 1e-9) + 1e-12
    epsB = max(fits["atan"].eps, fits["atanc"].eps) * (1 + 1e-9) + 1e-12
    assert np.abs(a[pos, 1] - e[pos, 1]).max() <= epsA
    rg = (x[:, 0] > 0) & (x[:, 1] > 0)
    assert np.abs(a[rg, 2] - e[rg, 2]).max() <= epsB
    # degenerate points: black -> 0; R = 0 < G -> pi/2; R = G = 0 < B -> angle B = 0
    d = mact.mact_sct(np.array([[0, 0, 0.0], [0, 0.4, 0.1], [0, 0, 0.6]]), fits["asin2"].p, fits["acos"].p,
                      fits["atan"].p, fits["atanc"].p)
    np.testing.assert_array_equal(d[0], [0, 0, 0])
    assert d[1, 2] == np.pi / 2 and d[2, 2] == 0.0


def test_sct_branch_is_b_over_l_half():
    # 3 B^2 >= R^2 + G^2 is B/L >= 1/2 for L > 0
    g = synth.rng(3)
    x = g.random((100000, 3))
    L = np.sqrt((x * x).sum(1))
    np.testing.assert_array_equal(3 * x[:, 2] ** 2 >= x[:, 0] ** 2 + x[:, 1] ** 2, x[:, 2] / L >= 0.5)


def test_clamping_of_float_inputs(fits):
    fc = fits["cbrt"]
    x = np.array([[-0.5, 1.5, 0.3]])
    np.testing.assert_array_equal(mact.mact_lab(x, fc.p, fc.q), mact.mact_lab(np.array([[0, 1, 0.3]]), fc.p, fc.q))


def test_forced_branches_and_the_tie_rule(fits):
    # The forced-branch options evaluate the other side of a boundary; the parity tie rule accepts a
    # value from the other side only for a pixel within 1e-6 of that boundary, and rejects it elsewhere.
    from tests import parity as P
    co = {"asin2": fits["asin2"].p, "acos": fits["acos"].p, "atan": fits["atan"].p, "atanc": fits["atanc"].p}
    # on the angle-A plane 3 B^2 = R^2 + G^2 (B/L = 1/2) and on G = R
    on_a = np.array([[0.3, 0.4, np.sqrt(0.25 / 3.0)]])
    on_b = np.array([[0.6, 0.6 * (1 + 1e-7), 0.1]])
    for x, key in ((on_a, "upper"), (on_b, "g_lt_r")):
        own = mact.mact_sct(x, co["asin2"], co["acos"], co["atan"], co["atanc"])
        sides = [mact.mact_sct(x, co["asin2"], co["acos"], co["atan"], co["atanc"], **{key: np.array([v])})
                 for v in (False, True)]
        # the oracle's own value is one side; the other side approximates the same angle, to the
        # fits' errors, but differs beyond the parity bar
        assert any(np.array_equal(own, s) for s in sides)
        other = sides[1] if np.array_equal(own, sides[0]) else sides[0]
        assert np.abs(other - own).max() < 1e-4
        assert np.any(np.abs(other - own)[0] / P.SCALE[2] > P.REL)
        assert P.assert_parity_ties(2, other, x, co) == 1
        far = x * np.array([1.0, 1.1, 1.0])  # off both planes
        wrong = mact.mact_sct(far, co["asin2"], co["acos"], co["atan"], co["atanc"]) + other - own
        with pytest.raises(AssertionError):
            P.assert_parity_ties(2, wrong, far, co)
    # the BT.709 decoding breakpoint: a channel at 0.081 on the linear side of the polynomial
    cb = fits["cbrt"]
    dec = remez.remez(lambda k: ((k + 0.099) / 1.099) ** (1 / 0.45), 7, 0, 0.081, 1.0).p
    x = np.array([[0.081, 0.5, 0.9]])
    own = mact.mact_lab(x, cb.p, cb.q, decode=dec)
    other = mact.mact_lab(x, cb.p, cb.q, decode=dec, decode_hi=np.array([[False, True, True]]))
    assert np.abs(other - own).max() / 116.0 > P.REL
    assert P.assert_parity_ties(0, other, x, {"p": cb.p, "q": cb.q}, decode=dec) == 1
    with pytest.raises(AssertionError):
        P.assert_parity_ties(0, other, x + np.array([[0.01, 0, 0]]), {"p": cb.p, "q": cb.q}, decode=dec)
    # forcing the side a value is on already changes nothing
    same = mact.mact_lab(x, cb.p, cb.q, decode=dec, decode_hi=x >= 0.081, f_hi=np.ones((1, 3), bool))
    np.testing.assert_array_equal(same, own)
