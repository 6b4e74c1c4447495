"""Writes tests/golden/mact_accuracy.json: the accuracy of the MACT transforms
and of the 3-D LUT interpolators against the exact transforms over all 2^24
8-bit colours, computed by the oracle alone (its own Remez fits of the
library's default degrees and intervals, FP64 evaluation).

    python tests/golden/make_golden.py

CIELAB: Delta E*ab (Sec. 3.2.1).  HSI: D_HSI (Sec. 3.3.1) and the hue error.
SCT: Delta E*ab through the inverse SCT (Sec. 3.4.1) and the angle errors.
CIELUV: Delta E*uv (the CIE 1976 L*u*v* distance; Sec. 4 names the transform).
LUTs: Delta E*ab of the CIELAB LUT at 9^3, 17^3 and 33^3 (Sec. 3.5.3); for
the HSI LUTs D_HSI and the hue error, for the SCT LUTs Delta E*ab through the
inverse SCT and the errors of angles A and B (all four methods, 9^3, 17^3 and
33^3; angular channels interpolated as unit vectors).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import colour, lut, mact, remez, tables as T  # noqa: E402
from tests.cubepool import cube_map  # noqa: E402


def fits():
    return {
        "cbrt": remez.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL),
        "atan_sqrt3": remez.remez(T.f_atan_sqrt3, 5, 0, 0.0, 1.0),
        "asin2": remez.remez(T.f_asin2, 5, 0, *T.T4_INTERVAL),
        "acos": remez.remez(T.f_acos, 5, 0, *T.T5_INTERVAL),
        "atan": remez.remez(T.f_atan, 5, 0, 0.0, 1.0),
        "atanc": remez.remez(T.f_atanc, 5, 0, 0.0, 1.0),
    }


def _chunk(v8, F, luts, xluts):
    x = v8 / 255.0
    out = {}
    ex_lab = colour.rgb_to_lab(x)
    d = colour.delta_e(mact.mact_lab(x, F["cbrt"].p, F["cbrt"].q), ex_lab)
    out["lab"] = (d.sum(), d.max())
    ex_hsi = colour.rgb_to_hsi(x)
    h = mact.mact_hsi(x, F["atan_sqrt3"].p)
    d = colour.d_hsi(h, ex_hsi)
    out["hsi"] = (d.sum(), d.max())
    a = colour.angle_diff(h[:, 0], ex_hsi[:, 0])
    out["hsi_dH"] = (a.sum(), a.max())
    ex_sct = colour.rgb_to_sct(x)
    s = mact.mact_sct(x, F["asin2"].p, F["acos"].p, F["atan"].p, F["atanc"].p)
    d = colour.sct_delta_e(s, ex_sct)
    out["sct"] = (d.sum(), d.max())
    da = np.abs(s[:, 1] - ex_sct[:, 1])
    db = np.abs(s[:, 2] - ex_sct[:, 2])
    out["sct_dA"] = (da.sum(), da.max())
    out["sct_dB"] = (db.sum(), db.max())
    ex_luv = colour.rgb_to_luv(x)
    d = colour.delta_e(mact.mact_luv(x, F["cbrt"].p, F["cbrt"].q), ex_luv)
    out["luv"] = (d.sum(), d.max())
    for key, L in luts.items():
        o, _ = lut.interp(L, "lab", key[0], v8=v8)
        d = colour.delta_e(o, ex_lab)
        out["lut_%s_%d" % key] = (d.sum(), d.max())
    for (xf, m, N), L in xluts.items():
        o, _ = lut.interp(L, xf, m, v8=v8)
        tag = "lut_%s_%s_%d" % (xf, m, N)
        if xf == "hsi":
            d = colour.d_hsi(o, ex_hsi)
            a = colour.angle_diff(o[:, 0], ex_hsi[:, 0])
            out[tag] = (d.sum(), d.max())
            out[tag + "_dH"] = (a.sum(), a.max())
        else:
            d = colour.sct_delta_e(o, ex_sct)
            da = colour.angle_diff(o[:, 1], ex_sct[:, 1])
            db = colour.angle_diff(o[:, 2], ex_sct[:, 2])
            out[tag] = (d.sum(), d.max())
            out[tag + "_dA"] = (da.sum(), da.max())
            out[tag + "_dB"] = (db.sum(), db.max())
    return out


def main():
    F = fits()
    methods = ("trilinear", "prism", "pyramidal", "tetrahedral")
    luts = {(m, N): lut.build("lab", N) for m in methods for N in (9, 17, 33)}
    xluts = {(xf, m, N): lut.build(xf, N) for xf in ("hsi", "sct") for m in methods for N in (9, 17, 33)}
    parts = cube_map(_chunk, F, luts, xluts)
    n = float(1 << 24)
    res = {}
    for k in parts[0]:
        res[k] = {"mean": float(sum(p[k][0] for p in parts) / n), "max": float(max(p[k][1] for p in parts))}
    res["fits"] = {k: {"n": len(f.p) - 1, "m": len(f.q) - 1, "lo": f.a, "hi": f.b, "eps": f.eps} for k, f in F.items()}
    res["what"] = ("oracle FP64, all 2^24 8-bit colours, BT.709 inverse gamma; lab/sct: Delta E*ab, hsi: D_HSI, "
                   "hsi_dH / sct_dA / sct_dB: angle errors in radians; luv: Delta E*uv; lut_<method>_<N>: CIELAB "
                   "LUT Delta E*ab; lut_hsi_*: D_HSI (_dH hue error); lut_sct_*: Delta E*ab through the inverse SCT "
                   "(_dA, _dB angle errors)")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mact_accuracy.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    print(json.dumps(res, indent=1, sort_keys=True))


if __name__ == "__main__":
    main()
