"""The HSI and SCT LUTs (every method at 9^3, 17^3 and 33^3) over all 2^24
8-bit colours on the GPU against the oracle's exhaustive figures in
tests/golden/mact_accuracy.json (written by tests/golden/make_golden.py from
the oracle alone): mean and max of D_HSI and of the hue error for HSI; of
Delta E*ab through the inverse SCT and of the errors of angles A and B for
SCT.  The paper's one HSI angular-LUT figure (Sec. 3.5.3: D_HSI mean 0.000777,
max 1.086255, grid not stated) is not reproduced by any reading tried (33^3
trilinear gives 0.000788 / 1.611); these LUT figures are parity unpinned
against the paper and held here to the oracle."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import colour
from tests.cubepool import cube_map_shared

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
METHODS = ("trilinear", "prism", "pyramidal", "tetrahedral")

# Tolerances from the float32 nodes and sums (each node value rounded once, relative 6e-8; a few
# float32 roundings per weighted sum):
#  - D_HSI: S and I move by ~1e-7, the hue by ~1e-7 / (resultant length); D_HSI is weighted by the
#    saturation, small where the resultant is short: 1e-6 on mean and max;
#  - hue error: its mean moves by ~1e-7; its max is pi on both sides (gray pixels, whose exact hue is
#    0 by convention, against an interpolated hue of pi): 1e-6;
#  - SCT angles: float32 angles near pi/2 are 1.2e-7 apart: 2.4e-7 on mean and max;
#  - SCT Delta E*ab through the inverse: the float32 angles and L become R, G, B through cosines and
#    sines (~1e-7 relative) and then the CIELAB slope, 116 * 7.787 / 4.5 ~ 200 per unit of linear
#    RGB at the dark end; a per-pixel change of ~2e-5 there, ~1e-6 elsewhere: 1e-5 on mean and max.
TOL = {"hsi": {"": 1e-6, "_dH": 1e-6}, "sct": {"": 1e-5, "_dA": 2.4e-7, "_dB": 2.4e-7}}


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "mact_accuracy.json")) as f:
        return json.load(f)


def _metrics(v8, start, shared, key):
    out = shared[key][start:start + len(v8)]
    x = v8 / 255.0
    if key[0] == "hsi":
        ex = colour.rgb_to_hsi(x)
        d = colour.d_hsi(out, ex)
        a = colour.angle_diff(out[:, 0], ex[:, 0])
        return [(float(d.sum()), float(d.max())), (float(a.sum()), float(a.max()))]
    ex = colour.rgb_to_sct(x)
    d = colour.sct_delta_e(out, ex)
    da = colour.angle_diff(out[:, 1], ex[:, 1])
    db = colour.angle_diff(out[:, 2], ex[:, 2])
    return [(float(d.sum()), float(d.max())), (float(da.sum()), float(da.max())), (float(db.sum()), float(db.max()))]


@pytest.mark.parametrize("N", [9, 17, 33])
@pytest.mark.parametrize("xform", ["hsi", "sct"])
def test_exhaustive_lut_accuracy_matches_the_oracle(M, golden, xform, N):
    cube = torch.from_numpy(synth.cube_u8()).cuda()
    L = M.lut_build(xform, N)
    outs = {(xform, m): M.lut_interp(L, N, xform, m, cube).reshape(-1, 3).double().cpu().numpy() for m in METHODS}
    tags = list(TOL[xform])
    for key in outs:
        parts = cube_map_shared(_metrics, outs, key)
        for j, t in enumerate(tags):
            mean = sum(p[j][0] for p in parts) / float(1 << 24)
            mx = max(p[j][1] for p in parts)
            g = golden["lut_%s_%s_%d%s" % (xform, key[1], N, t)]
            assert mean == pytest.approx(g["mean"], abs=TOL[xform][t]), (key, N, t)
            assert mx == pytest.approx(g["max"], abs=TOL[xform][t]), (key, N, t)
