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


# ---------------------------------------------------------------- branch ties
#
# For float inputs a pixel within rounding of a branch boundary may take either branch in
# float32: the SCT planes 3B^2 = R^2 + G^2 (angle A) and G = R (angle B), the BT.709
# decoding breakpoint 0.081, and the CIELAB threshold t = 0.008856.  Such a pixel must
# equal the oracle evaluated on one of the two sides; nothing is dropped from the check.
TIE = 1e-6


def _tie_options(xform, x, gamma, decode):
    """For one pixel x (3,) on the [0, 1] scale: a list of keyword sets for
    the oracle, one per combination of the sides of the branch decisions
    that lie within TIE of their boundary."""
    import itertools
    from oracle import colour as C
    xc = np.clip(np.asarray(x, dtype=np.float64), 0.0, 1.0)
    opts = []
    if xform == 2:
        R, G, B = xc
        rg2 = R * R + G * G
        up = 3 * B * B >= rg2
        gr = G < R
        near_a = abs(3 * B * B - rg2) <= TIE * (rg2 + B * B)
        near_b = R > 0 and G > 0 and abs(G - R) <= TIE * max(R, G)
        for a in ([up, not up] if near_a else [up]):
            for b in ([gr, not gr] if near_b else [gr]):
                opts.append({"upper": np.array(a), "g_lt_r": np.array(b)})
        return opts
    if xform not in (0, 3):
        return [{}]
    dec_hi = xc >= 0.081
    near_d = (np.abs(xc - 0.081) <= TIE) if (decode is not None and gamma == "bt709") else np.zeros(3, bool)
    if decode is not None and gamma == "bt709":
        lin = np.where(dec_hi, ((xc + 0.099) / 1.099) ** (1 / 0.45), xc / 4.5)
    else:
        lin = C.inverse_gamma(xc, gamma)
    t = C.rgb_to_xyz(lin) / C.WHITE_D65
    f_hi = t > C.LAB_T0
    near_f = np.abs(t / C.LAB_T0 - 1.0) <= TIE
    if xform == 3:
        f_hi, near_f = f_hi[1:2], near_f[1:2]
    bits = [("d", i) for i in range(3) if near_d[i]] + [("f", i) for i in range(len(f_hi)) if near_f[i]]
    for flips in itertools.product([False, True], repeat=len(bits)):
        d, f = dec_hi.copy(), f_hi.copy()
        for (kind, i), fl in zip(bits, flips):
            if fl:
                (d if kind == "d" else f)[i] = not (d if kind == "d" else f)[i]
        o = {"f_hi": f if xform == 0 else f[0]}
        if decode is not None and gamma == "bt709":
            o["decode_hi"] = d
        opts.append(o)
    return opts


def _oracle_forced(xform, x, co, gamma, decode, kw):
    x = np.asarray(x, dtype=np.float64)
    if xform == 0:
        return OM.mact_lab(x, co["p"], co["q"], gamma=gamma, decode=decode, **kw)
    if xform == 3:
        return OM.mact_luv(x, co["p"], co["q"], gamma=gamma, decode=decode, **kw)
    if xform == 2:
        return OM.mact_sct(x, co["asin2"], co["acos"], co["atan"], co["atanc"], **kw)
    return OM.mact_hsi(x, co["c"])


def assert_parity_ties(xform, gpu, x01, co, gamma="bt709", decode=None, rel=REL, what=""):
    """Element parity for float inputs: every pixel within `rel` x full scale of
    the oracle, or, for a pixel within TIE of a branch boundary, of the oracle
    evaluated with that decision on the other side.  Returns how many pixels
    matched only the other side."""
    x = np.asarray(x01, dtype=np.float64).reshape(-1, 3)
    g = np.asarray(gpu, dtype=np.float64).reshape(-1, 3)
    if decode is not None and gamma == "bt709" and xform in (0, 3):
        ref = _oracle_forced(xform, x, co, gamma, decode, {})
    else:
        ref = oracle(xform, x, co, gamma=gamma)
    err = np.abs(g - ref) / SCALE[xform]
    bad = np.flatnonzero(np.any(err > rel, axis=1))
    other = 0
    for i in bad:
        best = None
        for kw in _tie_options(xform, x[i], gamma, decode):
            r = _oracle_forced(xform, x[i:i + 1], co, gamma, decode, {k: np.asarray(v)[None] for k, v in kw.items()})
            e = np.abs(g[i] - r[0]) / SCALE[xform]
            best = e if best is None or e.max() < best.max() else best
        assert np.all(best <= rel), \
            "%s: pixel %d %s: gpu %s oracle %s, error / scale %s (other side of a tie: %s)" % (
                what, i, x[i], g[i], ref[i], err[i], best)
        other += 1
    return other
