"""Helpers for GPU-vs-oracle parity tests: the oracle's evaluation of the
exact approximation the GPU uses (its coefficients rounded to float32), and
the per-channel tolerance rule."""
import numpy as np

from oracle import mact as OM

# per-channel full scale (L*, a*, b*), (H, S, I), (L, A, B), (L*, u*, v*): the factor in front of
# each output's bounded part (|u' - u'n|, |v' - v'n| < 1 with L* <= 100 gives 13 * 100)
SCALE = {
    0: np.array([116.0, 1000.0, 400.0]),
    1: np.array([2 * np.pi, 1.0, 1.0]),
    2: np.array([np.sqrt(3.0), np.pi / 2, np.pi / 2]),
    3: np.array([116.0, 1300.0, 1300.0]),
}
REL = 2e-6  # float32 parity bound relative to the channel's full scale


def f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def coeffs(params):
    """Oracle-form coefficients of a Params struct, rounded to float32."""
    xf = params.xform
    if xf in (0, 3):
        a = params.f[0]
        q = a.q_list if a.m > 0 else [1.0]
        return {"p": f32(a.p_list), "q": f32(q)}
    if xf == 1:
        return {"c": f32(params.f[0].p_list)}
    return {k: f32(params.f[i].p_list) for i, k in enumerate(("asin2", "acos", "atan", "atanc"))}


def oracle(xform, x01, co, gamma="bt709", debug=False):
    """The oracle's MACT transform of normalised RGB x01 (..., 3)."""
    if xform == 0:
        return OM.mact_lab(x01, co["p"], co["q"], gamma=gamma, debug=debug)
    if xform == 3:
        return OM.mact_luv(x01, co["p"], co["q"], gamma=gamma)
    if xform == 1:
        return OM.mact_hsi(x01, co["c"])
    return OM.mact_sct(x01, co["asin2"], co["acos"], co["atan"], co["atanc"])


def max_scaled_err(xform, gpu, ref):
    """max over pixels of |gpu - ref| / full scale, per channel."""
    d = np.abs(np.asarray(gpu, dtype=np.float64) - ref).reshape(-1, 3)
    return (d / SCALE[xform]).max(axis=0)


def assert_parity(xform, gpu, ref, rel=REL, what=""):
    e = max_scaled_err(xform, gpu, ref)
    assert np.all(e <= rel), "%s: per-channel error / scale %s exceeds %g" % (what, e, rel)
    return e
