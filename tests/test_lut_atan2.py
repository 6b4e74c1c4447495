"""The LUT kernels' atan2 (csrc/lut.hip, lut_atan2), which turns the
interpolated (cos, sin) resultants of the angular channels back into angles
(Sec. 3.5.3, angular interpolation).  Its steps are replayed here in float32
from the constants in the source: the polynomial's accuracy on [0, 1], the
octant and quadrant unfolding, and atan2's signed zeros, against numpy's
arctan2 in float64.  The hardware reciprocal is taken as correctly rounded;
the kernel corrects it with one Newton step, and the GPU parity tests check
the result on the device."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1009_0854_amd", "csrc",
                   "lut.hip")


def _coefficients():
    src = open(SRC).read()
    body = re.search(r"float lut_atan2\(float y, float x\) \{(.*?)\n\}", src, re.S).group(1)
    lead = re.search(r"float q = ([-0-9a-fx.p]+)f;", body).group(1)
    rest = re.findall(r"q = __builtin_fmaf\(q, s, ([-0-9a-fx.p]+)f\);", body)
    return [float.fromhex(lead)] + [float.fromhex(c) for c in rest]  # highest degree first


F = np.float32


def _fma(a, b, c):
    # float32 fused multiply-add: the product of two float32 is exact in float64
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F)


def _atan2(y, x, coef):
    y, x = np.asarray(y, F), np.asarray(x, F)
    ax, ay = np.abs(x) * F(2.0 ** 64), np.abs(y) * F(2.0 ** 64)
    mx = np.maximum(np.maximum(ax, ay), F(2.0 ** -100))
    mn = np.minimum(ax, ay)
    r = (1.0 / mx.astype(np.float64)).astype(F)
    t = (mn * r).astype(F)
    t = _fma(_fma(-mx, t, mn), r, t)
    s = (t * t).astype(F)
    q = np.full_like(t, F(coef[0]))
    for c in coef[1:]:
        q = _fma(q, s, np.full_like(t, F(c)))
    a = _fma((t * s).astype(F), q, t)
    pi2 = F(np.pi / 2)
    pi2lo = F(np.pi / 2 - float(pi2))
    pi = F(np.pi)
    pilo = F(np.pi - float(pi))
    a = np.where(ay > ax, ((pi2 - a).astype(F) + pi2lo).astype(F), a)
    a = np.where(np.signbit(x), ((pi - a).astype(F) + pilo).astype(F), a)
    return np.copysign(a, y)


def _ulps(got, ref):
    return np.abs(got.astype(np.float64) - ref) / np.spacing(np.abs(ref).astype(F)).astype(np.float64)


def test_polynomial_degree_and_accuracy_on_the_unit_interval():
    coef = _coefficients()
    assert len(coef) == 8
    t = np.concatenate([np.linspace(0, 1, 1 << 20, dtype=F)[1:], F(2.0) ** -np.arange(1, 40, dtype=F)])
    got = _atan2(t, np.ones_like(t), coef)
    assert _ulps(got, np.arctan(t.astype(np.float64))).max() < 1.5


def test_every_octant_within_two_ulps():
    rng = np.random.default_rng(7)
    ang = rng.uniform(-np.pi, np.pi, 1 << 20)
    rad = rng.uniform(1e-3, 1.0, ang.size)
    x, y = (rad * np.cos(ang)).astype(F), (rad * np.sin(ang)).astype(F)
    got = _atan2(y, x, _coefficients())
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    assert _ulps(got, ref).max() < 2.0
    # the half-plane boundaries and the diagonals
    for yy, xx in [(1, 1), (-1, 1), (1, -1), (-1, -1), (1, 0), (-1, 0), (0, 1), (0, -1), (0.5, 1e-30), (1e-30, -0.5)]:
        g = _atan2(F(yy), F(xx), _coefficients())
        r = np.arctan2(F(yy), F(xx)).astype(np.float64)
        assert abs(float(g) - r) <= 2 * np.spacing(np.float32(abs(r)) if r else np.float32(0)), (yy, xx)


def test_signed_zeros_and_tiny_resultants_follow_atan2():
    coef = _coefficients()
    for yy in (0.0, -0.0):
        for xx in (0.0, -0.0):
            g, r = _atan2(F(yy), F(xx), coef), np.arctan2(F(yy), F(xx))
            assert g == r and np.signbit(g) == np.signbit(r), (yy, xx, g, r)
    # denormal components (float inputs of denormal size reach them) keep their angle
    tiny = F(3e-42)
    for yy, xx in [(tiny, tiny), (tiny, F(2) * tiny), (-tiny, -F(5) * tiny), (F(1e-38), -F(1e-45))]:
        g = _atan2(F(yy), F(xx), coef)
        r = np.arctan2(np.float64(yy), np.float64(xx))
        assert np.isfinite(g) and abs(float(g) - r) < 1e-6, (yy, xx, g, r)
