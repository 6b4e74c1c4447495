"""GPU parity of the caching LUT (lut_cache_build / lut_cache_interp, Sec.
3.5.3's second version of every method) against the oracle's caching form:
records, interpolation for every transform, method and size, float inputs,
agreement with the packed form to float32 rounding, and Table 12 from the
GPU's own output (the paper prints one error per method for both versions)."""
import numpy as np
import pytest

import synth
from oracle import colour, lut as OL, tables as T
from tests import parity as P
from tests.cubepool import cube_map_shared
from tests.test_gpu_lut import METHODS, XF, _compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _cache_interp(M, xform, N, method, x_np, layout="hwc"):
    Cb = M.lut_cache_build(xform, N)
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    y = M.lut_cache_interp(Cb, N, xform, method, x, layout=layout)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), Cb


@pytest.mark.parametrize("N", [9, 17, 33])
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_records_are_the_oracle_records_rounded_once(M, xform, N):
    # layout and values: record (i, j, k), entry e, component q; every value the oracle's FP64
    # value rounded once to float32 (an FP64 cosine or sine may differ by an ulp between
    # libraries, so one float32 ulp is allowed; a difference that is zero in exact arithmetic,
    # such as a* along the gray axis, is FP64 rounding noise of either side: 1e-9 absolute)
    Cb = M.lut_cache_build(xform, N)
    torch.cuda.synchronize()
    ref = OL.build_cache(xform, N)
    m, C = N - 1, ref.shape[-1]
    assert M.lut_cache_bytes(xform, N) == (m ** 3 * 13 * C * 4 + 15) // 16 * 16
    got = Cb.cpu().numpy()[:m ** 3 * 13 * C].reshape(m, m, m, 13, C).astype(np.float64)
    want = ref.astype(np.float32).astype(np.float64)
    ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got - want) <= np.maximum(ulp, 1e-9))


@pytest.mark.parametrize("N", [9, 17, 33])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_cache_u8_parity(M, xform, method, N):
    # packed 8-bit HWC (the 4-pixel kernel, LDS-staged for 9^3 LAB, LUV and HSI) with a ragged
    # tail, corners and grays included
    img = synth.uniform_u8(129, 131, seed=N + 40)
    img.reshape(-1, 3)[:6] = [[0, 0, 0], [255, 255, 255], [128, 128, 128], [255, 0, 0], [0, 0, 255], [17, 17, 200]]
    gpu, _ = _cache_interp(M, xform, N, method, img)
    ref, rlen = OL.interp_cache(OL.build_cache(xform, N), xform, method, v8=img)
    _compare(xform, gpu, ref, rlen)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("xform", ["lab", "sct"])
def test_cache_float_chw_and_strided(M, xform, method):
    # float CHW input (values outside [0, 1] clamp) through the one-pixel kernel, and a row-strided
    # 8-bit view
    g = synth.rng(37)
    x = g.uniform(-0.05, 1.05, (3, 45, 47)).astype(np.float32)
    gpu, Cb = _cache_interp(M, xform, 17, method, x, layout="chw")
    xc = np.moveaxis(x.astype(np.float64), 0, -1)
    ref, rlen = OL.interp_cache(OL.build_cache(xform, 17), xform, method, x=xc)
    mask = None
    if method in ("pyramidal", "prism", "tetrahedral"):
        # branch choices within float32 rounding of a cell face or a tie of two fractions
        pos = np.clip(xc.reshape(-1, 3), 0, 1) * 16
        f = pos - np.minimum(np.floor(pos), 15)
        near_face = (np.abs(pos - np.rint(pos)) < 1e-5).any(1)
        near_tie = ((np.abs(f[:, 0] - f[:, 1]) < 1e-5) | (np.abs(f[:, 0] - f[:, 2]) < 1e-5) |
                    (np.abs(f[:, 1] - f[:, 2]) < 1e-5))
        mask = ~(near_face | near_tie)
    _compare(xform, np.moveaxis(gpu, 0, -1), ref, rlen, mask)
    base = torch.from_numpy(synth.uniform_u8(33, 70, seed=3)).cuda()
    view = base[:, 3:3 + 61]
    y = M.lut_cache_interp(Cb, 17, xform, method, view)
    torch.cuda.synchronize()
    v8 = view.cpu().numpy()
    ref, rlen = OL.interp_cache(OL.build_cache(xform, 17), xform, method, v8=v8)
    _compare(xform, y.cpu().numpy().astype(np.float64), ref, rlen)


@pytest.mark.parametrize("N", [9, 17, 33])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_cache_equals_packed_to_rounding(M, xform, method, N):
    # the same interpolant regrouped: the caching and packed forms agree to float32 rounding
    g = torch.Generator(device="cuda").manual_seed(N)
    x = torch.randint(0, 256, (2, 61, 257, 3), dtype=torch.uint8, device="cuda", generator=g)
    a = M.lut_interp(M.lut_build(xform, N), N, xform, method, x)
    b = M.lut_cache_interp(M.lut_cache_build(xform, N), N, xform, method, x)
    torch.cuda.synchronize()
    a = a.reshape(-1, 3).double().cpu().numpy()
    b = b.reshape(-1, 3).double().cpu().numpy()
    for ch, ang in enumerate(OL.ANGULAR[xform]):
        d = colour.angle_diff(a[:, ch], b[:, ch]) if ang else np.abs(a[:, ch] - b[:, ch])
        # angles: short resultants near the gray axis are ill-conditioned; bound by the node spacing
        assert (d.max() if not ang else np.percentile(d, 99.9)) / P.SCALE[XF[xform]][ch] <= P.REL, (ch, d.max())


def test_cache_interior_node_hits(M):
    # at a node input whose fractions are all zero the value is entry 0 exactly
    N = 17
    idx = np.stack(np.meshgrid(*[np.arange(N - 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = (idx / (N - 1.0)).astype(np.float32).reshape(1, -1, 3)
    gpu, Cb = _cache_interp(M, "lab", N, "tetrahedral", x)
    rec = Cb.cpu().numpy()[:(N - 1) ** 3 * 39].reshape(-1, 13, 3)[:, 0, :]
    np.testing.assert_array_equal(gpu.reshape(-1, 3), rec.astype(np.float64))


def _t12(v8, start, shared, key):
    out = shared[key][start:start + len(v8)]
    d = colour.delta_e(out, colour.rgb_to_lab(v8 / 255.0))
    return float(d.sum()), float(d.max())


def test_table12_from_gpu_cache_output(M):
    # Table 12 prints one error pair per method for its standard and caching versions: all 2^24
    # colours through the GPU caching form reproduce it (trilinear, prism, tetrahedral; the
    # pyramidal row is unpinned) to the printed digits within float32 rounding
    cube = torch.from_numpy(synth.cube_u8()).cuda()
    outs = {}
    for method in ("trilinear", "prism", "tetrahedral"):
        for N in (17, 33):
            Cb = M.lut_cache_build("lab", N)
            outs[(method, N)] = M.lut_cache_interp(Cb, N, "lab", method, cube).reshape(-1, 3).double().cpu().numpy()
    for key in list(outs):
        parts = cube_map_shared(_t12, outs, key)
        mean = sum(p[0] for p in parts) / float(1 << 24)
        mx = max(p[1] for p in parts)
        avg_p, max_p = T.T12_LUT_ERR[key]
        assert mean == pytest.approx(avg_p, abs=2e-6), key
        assert mx == pytest.approx(max_p, abs=2e-5), key
