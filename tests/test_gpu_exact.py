"""GPU parity of the exact float32 baseline (mact_transform_exact: the
transforms with the device's elementary functions, the baseline MACT replaces)
against the oracle's exact FP64 transforms over every 8-bit colour, to the
float32 parity bar; float16 output is the float32 result rounded."""
import numpy as np
import pytest

import synth
from oracle import colour as C
from tests import parity as P
from tests.cubepool import cube_map_shared

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EXACT = {0: C.rgb_to_lab, 1: C.rgb_to_hsi, 2: C.rgb_to_sct, 3: C.rgb_to_luv}


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _cmp(v8, start, shared, xform):
    g = shared[start:start + len(v8)]
    return P.max_scaled_err(xform, g, EXACT[xform](v8 / 255.0))


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_exact_every_colour(M, xform):
    cube = torch.from_numpy(synth.cube_u8()).cuda()
    y = M.transform_exact(cube, xform=xform)
    torch.cuda.synchronize()
    gpu = y.reshape(-1, 3).cpu().numpy().astype(np.float64)
    e = np.max(np.stack(cube_map_shared(_cmp, gpu, xform)), axis=0)
    assert np.all(e <= P.REL), e


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_exact_f16_output_and_ragged_sizes(M, xform):
    # float16 output is the float32 result rounded to nearest even; ragged sizes and batches
    g = synth.rng(60 + xform)
    for shape in [(1, 1, 1), (1, 3, 7), (2, 17, 33), (3, 64, 129)]:
        x = torch.from_numpy(g.integers(0, 256, shape + (3,)).astype(np.uint8)).cuda()
        for gm in (["bt709", "srgb", "none"] if xform in (0, 3) else ["none"]):
            a = M.transform_exact(x, xform=xform, gamma=gm)
            h = M.transform_exact(x, xform=xform, gamma=gm, out_dtype=torch.float16)
            torch.cuda.synchronize()
            assert torch.equal(h, a.half()), (shape, gm)
            ref = EXACT[xform](x.cpu().numpy().reshape(-1, 3) / 255.0, gm) if xform in (0, 3) else \
                EXACT[xform](x.cpu().numpy().reshape(-1, 3) / 255.0)
            P.assert_parity(xform, a.reshape(-1, 3).cpu().numpy().astype(np.float64), ref, what=str((shape, gm)))


def test_exact_differs_from_mact_by_the_fit_error(M):
    # the baseline is not MACT: on the 1080p batch the two differ by about the fit's error
    x = torch.from_numpy(synth.smooth_batch_u8(1, 270, 480, 1000)).cuda()
    d = (M.transform_exact(x) - M.transform(x)).abs().amax(dim=(0, 1, 2)).cpu().numpy()
    torch.cuda.synchronize()
    assert 1e-4 < d[1] < 0.02, d  # a*: 500 |f~ - f| differences, the (4,4) fit's eps 1.09e-5 x 1000
