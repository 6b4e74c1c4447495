"""GPU parity of the inverse transforms (mact_inverse; CIELAB, HSI, SCT and
CIELUV) against the oracle's approximated inverses, and of the on-device error statistics
(mact_error_stats) against the oracle's metrics."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import colour as C, mact as OM
from tests import parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _f32(c):
    return np.float32(c).astype(np.float64)


def _inv_coeffs(p):
    """The inverse's approximations as the GPU evaluates them: float32-rounded."""
    f = p.f
    return {"p0": _f32(f[0].p_list), "q0": _f32(f[0].q_list), "p1": _f32(f[1].p_list)}


@pytest.fixture(scope="module")
def colours():
    # every 8-bit colour on a 1/7 subsample of the cube, plus the corners and the grays
    v = synth.cube_u8().reshape(-1, 3)[::7]
    extra = np.array([[0, 0, 0], [255, 255, 255], [255, 0, 0], [0, 255, 0], [0, 0, 255], [128, 128, 128],
                      [255, 255, 0], [0, 255, 255], [255, 0, 255], [1, 0, 0], [0, 0, 1]], dtype=np.uint8)
    return np.concatenate([v, extra]) / 255.0


def _run_inverse(M, x_np, xform, p, gamma="bt709", layout="hwc", dtype=torch.float32, out_dtype=None):
    x = torch.from_numpy(np.ascontiguousarray(x_np.astype(np.float32))).to(dtype).cuda()
    y = M.inverse(x, xform=xform, params=p, layout=layout, gamma=gamma, out_dtype=out_dtype)
    torch.cuda.synchronize()
    return y.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("gamma", ["bt709", "none"])
def test_lab_inverse_parity(M, colours, gamma):
    # float32 rounding bound: the linear values carry about 8 float32 roundings of magnitude
    # sum_j |M^-1 diag(white)|_ij |t_j| <= 5.5, and the encoding's slope is at most 4.5:
    # 4.5 * 5.5 * 8 * 2^-24 = 1.2e-5
    p = M.inverse_params("lab")
    co = _inv_coeffs(p)
    lab = C.rgb_to_lab(colours).astype(np.float32).astype(np.float64)
    gpu = _run_inverse(M, lab.reshape(1, -1, 3), "lab", p, gamma=gamma).reshape(-1, 3)
    ref = OM.mact_lab_inverse(lab, co["p0"], co["q0"], gamma=gamma)
    err = np.abs(gpu - ref)
    if gamma == "bt709":
        # the encoding's two branches differ by 4.7e-4 at 0.018: either branch is right within 1e-6 of it
        lin = OM.mact_lab_inverse(lab, co["p0"], co["q0"], gamma="none")
        err[np.abs(lin - 0.018) <= 1e-6] = 0.0
    print("CIELAB inverse (%s): achieved max error %.3g, bound 1.2e-5" % (gamma, err.max()))
    assert err.max() <= 1.2e-5, err.max()


@pytest.mark.parametrize("gamma", ["bt709", "none"])
def test_luv_inverse_parity(M, colours, gamma):
    # float32 rounding bound: X, Y, Z (each at most the white's) carry about 12 float32 roundings
    # (the cube, 1/(13 L*), u', v', q, the products); the rows of M^-1 weight them by at most
    # sum_j |M^-1_0j| white_j = 5.16, and the encoding's slope is at most 4.5:
    # 4.5 * 5.16 * 12 * 2^-24 = 1.7e-5
    p = M.inverse_params("luv")
    co = _inv_coeffs(p)
    luv = C.rgb_to_luv(colours).astype(np.float32).astype(np.float64)
    gpu = _run_inverse(M, luv.reshape(1, -1, 3), "luv", p, gamma=gamma).reshape(-1, 3)
    ref = OM.mact_luv_inverse(luv, co["p0"], co["q0"], gamma=gamma)
    err = np.abs(gpu - ref)
    if gamma == "bt709":
        lin = OM.mact_luv_inverse(luv, co["p0"], co["q0"], gamma="none")
        err[np.abs(lin - 0.018) <= 1e-6] = 0.0
    print("CIELUV inverse (%s): achieved max error %.3g, bound 1.7e-5" % (gamma, err.max()))
    assert err.max() <= 1.7e-5, err.max()
    # black is black
    blk = _run_inverse(M, np.zeros((1, 1, 3)), "luv", p, gamma=gamma)
    assert np.array_equal(blk, np.zeros((1, 1, 3)))


def test_hsi_inverse_parity(M, colours):
    # |start| <= 3 I with a ratio of two cosine polynomials (each >= 1/2): a few float32 ulps
    p = M.inverse_params("hsi")
    co = _inv_coeffs(p)
    hsi = C.rgb_to_hsi(colours).astype(np.float32).astype(np.float64)
    gpu = _run_inverse(M, hsi.reshape(1, -1, 3), "hsi", p).reshape(-1, 3)
    ref = OM.mact_hsi_inverse(hsi, co["p0"])
    print("HSI inverse: achieved max error %.3g, bound 4e-6" % np.abs(gpu - ref).max())
    assert np.abs(gpu - ref).max() <= 4e-6


def test_sct_inverse_parity(M, colours):
    p = M.inverse_params("sct")
    co = _inv_coeffs(p)
    sct = C.rgb_to_sct(colours).astype(np.float32).astype(np.float64)
    gpu = _run_inverse(M, sct.reshape(1, -1, 3), "sct", p).reshape(-1, 3)
    ref = OM.mact_sct_inverse(sct, co["p0"], co["p1"])
    print("SCT inverse: achieved max error %.3g, bound %.3g" % (np.abs(gpu - ref).max(), 2e-6 * np.sqrt(3.0)))
    assert np.abs(gpu - ref).max() <= 2e-6 * np.sqrt(3.0)


@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_inverse_layouts_and_float16(M, xform):
    # CHW float16 in, HWC float32 out: the same values as packed HWC float32 in
    g = synth.rng(31)
    rgb = g.random((2, 37, 53, 3))
    fwd = {"lab": C.rgb_to_lab, "hsi": C.rgb_to_hsi, "sct": C.rgb_to_sct, "luv": C.rgb_to_luv}[xform](rgb).astype(np.float16)
    p = M.inverse_params(xform)
    a = _run_inverse(M, fwd.astype(np.float32), xform, p)
    chw = np.ascontiguousarray(np.moveaxis(fwd, -1, 1))
    x = torch.from_numpy(chw).cuda()
    b = M.inverse(x, xform=xform, params=p, layout="chw", out_layout="hwc")
    torch.cuda.synchronize()
    assert np.array_equal(a, b.cpu().numpy().astype(np.float64))
    h = M.inverse(x, xform=xform, params=p, layout="chw", out_dtype=torch.float16)
    torch.cuda.synchronize()
    assert torch.equal(h, torch.from_numpy(np.moveaxis(a, -1, 1).astype(np.float32)).cuda().half())


@pytest.mark.parametrize("dtype", [np.float32, np.float16], ids=["f32", "f16"])
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_inverse_chw_equals_hwc(M, xform, dtype):
    # packed CHW planes (the 4-pixel plane kernel where W H is a multiple of 4, the one-pixel kernel
    # otherwise) give the HWC result's bits, plane by plane, for float32 and float16 outputs
    g = synth.rng(77)
    fwd = {"lab": C.rgb_to_lab, "hsi": C.rgb_to_hsi, "sct": C.rgb_to_sct, "luv": C.rgb_to_luv}[xform]
    p = M.inverse_params(xform)
    for (n, h, w) in [(2, 16, 20), (1, 33, 36), (3, 8, 1000), (1, 7, 9)]:
        v = fwd(g.random((n, h, w, 3))).astype(dtype)
        hwc = torch.from_numpy(v).cuda()
        chw = torch.from_numpy(np.ascontiguousarray(np.moveaxis(v, -1, 1))).cuda()
        for gm in (["bt709", "none"] if xform in ("lab", "luv") else ["none"]):
            for od in (torch.float32, torch.float16):
                a = M.inverse(chw, xform=xform, params=p, layout="chw", gamma=gm, out_dtype=od)
                b = M.inverse(hwc, xform=xform, params=p, gamma=gm, out_dtype=od)
                torch.cuda.synchronize()
                assert a.dtype == od and torch.equal(a, b.permute(0, 3, 1, 2).contiguous()), (n, h, w, gm, od)


@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_round_trip_on_the_1080p_batch(M, xform):
    # MACT forward then MACT inverse on the GPU returns the 8-bit colours to within a
    # fraction of one code (sampled pixels of 4 images of the benchmark batch)
    imgs = synth.smooth_batch_u8(4, 1080, 1920, 1000)
    x = torch.from_numpy(imgs).cuda()
    y = M.transform(x, xform=xform)
    gm = "bt709" if xform in ("lab", "luv") else "none"
    back = M.inverse(y, xform=xform, gamma=gm)
    torch.cuda.synchronize()
    idx = torch.from_numpy(synth.rng(5).integers(0, x.numel() // 3, 200000)).cuda()
    got = back.reshape(-1, 3)[idx].cpu().numpy().astype(np.float64)
    want = imgs.reshape(-1, 3)[idx.cpu().numpy()] / 255.0
    tol = {"lab": 2e-3, "hsi": 2e-3, "sct": 2e-4, "luv": 2e-3}[xform]
    assert np.abs(got - want).max() <= tol


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_error_stats_equal_the_oracle_metric_of_the_gpu_output(M, xform):
    # the device's float64 reference and metric against the oracle's, on the same float32
    # MACT outputs: agreement to float64 rounding
    img = synth.uniform_u8(512, 512, seed=1)
    img.reshape(-1, 3)[:5] = [[0, 0, 0], [255, 255, 255], [9, 9, 9], [255, 0, 0], [3, 200, 7]]
    p = M.default_params(xform)
    x = torch.from_numpy(img).cuda()
    y = M.transform(x, xform=xform, params=p).reshape(-1, 3).double().cpu().numpy()
    st = M.error_stats(x, xform=xform, params=p)
    rgb = img.reshape(-1, 3) / 255.0
    if xform == 0:
        ex = C.rgb_to_lab(rgb)
        d = C.delta_e(y, ex)
        ch = np.abs(y - ex).max(axis=0)
    elif xform == 1:
        ex = C.rgb_to_hsi(rgb)
        d = C.d_hsi(y, ex)
        ch = np.array([C.angle_diff(y[:, 0], ex[:, 0]).max(), np.abs(y[:, 1] - ex[:, 1]).max(),
                       np.abs(y[:, 2] - ex[:, 2]).max()])
    elif xform == 2:
        ex = C.rgb_to_sct(rgb)
        d = C.sct_delta_e(y, ex)
        ch = np.abs(y - ex).max(axis=0)
    else:
        ex = C.rgb_to_luv(rgb)
        d = C.delta_e(y, ex)  # Delta E*uv: the Euclidean distance in L*u*v*
        ch = np.abs(y - ex).max(axis=0)
    assert st["count"] == img.shape[0] * img.shape[1]
    # float64 library functions differ by an ulp or so; the oracle's hue is the arccos form,
    # equal to Kender's (the device's) within 1e-12
    assert st["mean"] == pytest.approx(d.mean(), rel=1e-9, abs=1e-11)
    assert st["max"] == pytest.approx(d.max(), rel=1e-9, abs=1e-11)
    np.testing.assert_allclose(st["max_abs"], ch, rtol=1e-9, atol=1e-11)


# The GPU evaluates the approximations in float32 (coefficients rounded to float32); the oracle's
# exhaustive statistics are FP64 with its own FP64 fits.  CIELAB: f~ carries up to about 8 float32
# roundings (8 * 2^-24 ~ 4.8e-7 relative, f <= 1), and a*, b* amplify a difference of two f by 500
# and 200, so one pixel's Delta E moves by at most sqrt(116^2 + 1000^2 + 400^2) * 4.8e-7 ~ 5.2e-4;
# the mean moves far less.  HSI: hue in float32 on [0, 2pi] (a few ulp ~ 2e-6), so 2e-5; SCT: 5e-5.
# CIELUV: L* = 116 f~ - 16 moves by 116 * 4.8e-7 ~ 5.6e-5; u*, v* = 13 L* (u' - u'n) with |u' - u'n|,
# |v' - v'n| < 0.5 and L* <= 100 add 13 * 0.5 * 5.6e-5 ~ 3.6e-4 through L* and about 13 * 100 * 0.6 *
# 2.4e-7 ~ 1.9e-4 through the float32 quotients: 6e-4 for one pixel.
@pytest.mark.parametrize("xform,key,tol_mean,tol_max", [(0, "lab", 2e-5, 5.2e-4), (1, "hsi", 2e-5, 2e-5),
                                                         (2, "sct", 5e-5, 5e-5), (3, "luv", 2e-5, 6e-4)],
                         ids=["lab", "hsi", "sct", "luv"])
def test_error_stats_of_every_colour_match_the_oracle_tables(M, xform, key, tol_mean, tol_max):
    # all 2^24 colours on the GPU against the oracle's exhaustive statistics
    with open(os.path.join(HERE, "golden", "mact_accuracy.json")) as f:
        g = json.load(f)
    cube = torch.from_numpy(synth.cube_u8()).cuda()
    st = M.error_stats(cube, xform=xform)
    assert st["count"] == 1 << 24
    assert st["mean"] == pytest.approx(g[key]["mean"], abs=tol_mean)
    assert st["max"] == pytest.approx(g[key]["max"], abs=tol_max)
    tol = tol_max
    if xform == 1:
        assert st["max_abs"][0] == pytest.approx(g["hsi_dH"]["max"], abs=tol)
    if xform == 2:
        assert st["max_abs"][1] == pytest.approx(g["sct_dA"]["max"], abs=1e-6)
        assert st["max_abs"][2] == pytest.approx(g["sct_dB"]["max"], abs=1e-6)


@pytest.mark.parametrize("shape", [(1, 3), (7, 9), (64, 64), (129, 257)])
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_inverse_fast_path_equals_general(M, xform, shape):
    # packed float32 HWC (LDS-staged chunks, ragged tail) gives the bits of the one-pixel-per-lane
    # kernel, which a row-padded view of the same values forces, for float32 and float16 outputs
    g = synth.rng(sum(shape))
    rgb = g.random((2,) + shape + (3,))
    fwd = {"lab": C.rgb_to_lab, "hsi": C.rgb_to_hsi, "sct": C.rgb_to_sct, "luv": C.rgb_to_luv}[xform](rgb).astype(np.float32)
    x = torch.from_numpy(fwd).cuda()
    p = M.inverse_params(xform)
    big = torch.zeros((2, shape[0], shape[1] + 3, 3), dtype=torch.float32, device="cuda")
    big[:, :, :shape[1]] = x
    for gm in (["bt709", "none"] if xform in ("lab", "luv") else ["none"]):
        for od in (torch.float32, torch.float16):
            fast = M.inverse(x, xform=xform, params=p, gamma=gm, out_dtype=od)
            general = M.inverse(big[:, :, :shape[1]], xform=xform, params=p, gamma=gm, out_dtype=od)
            torch.cuda.synchronize()
            assert fast.dtype == od and torch.equal(fast, general), (gm, od)
        # float16 out is the float32 result rounded to nearest even
        f32 = M.inverse(x, xform=xform, params=p, gamma=gm)
        f16 = M.inverse(x, xform=xform, params=p, gamma=gm, out_dtype=torch.float16)
        torch.cuda.synchronize()
        assert torch.equal(f16, f32.half()), gm
