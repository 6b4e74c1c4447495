"""GPU parity of mact_transform against the oracle's MACT evaluation:
element by element, per-channel |gpu - oracle| <= 2e-6 x full scale (float32
arithmetic of the same approximation), plus the exhaustive 2^24-colour cube."""
import numpy as np
import pytest

import synth
from oracle import mact as OM
from tests import parity as P
from tests.cubepool import cube_map_shared

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _run(M, x_np, xform, params=None, layout="hwc", gamma="bt709", out_dtype=None):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    y = M.transform(x, xform=xform, params=params, layout=layout, gamma=gamma, out_dtype=out_dtype)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_c1_uniform_512(M, xform):
    # 512 x 512 uint8, i.i.d. uniform (seed 1), default approximations
    img = synth.uniform_u8(512, 512, seed=1)
    p = M.default_params(xform)
    gpu = _run(M, img, xform, p)
    ref = P.oracle(xform, img / 255.0, P.coeffs(p))
    P.assert_parity(xform, gpu, ref, what="C1")


def test_lab_debug_f_domain_relative(M):
    img = synth.uniform_u8(256, 300, seed=2)
    p = M.default_params(0)
    p.out_mode = 1
    gpu = _run(M, img, 0, p)
    ref = P.oracle(0, img / 255.0, P.coeffs(p), debug=True)
    rel = np.abs(gpu - ref) / np.abs(ref)
    assert rel.max() <= 2e-6, rel.max()


def test_lab_paper_coefficients(M):
    # Table 2's printed (4, 4) rational (unnormalised denominator) through the same kernel
    img = synth.uniform_u8(128, 129, seed=3)
    p = M.make_params(0, [M.paper_approx(M.FN_CBRT, 4, 4)])
    gpu = _run(M, img, 0, p)
    P.assert_parity(0, gpu, P.oracle(0, img / 255.0, P.coeffs(p)))


@pytest.mark.parametrize("beta,delta", [(0.5, 0.01), (1.0, 0.05)])
def test_lab_weighted_fit_parity_and_error_statistics(M, beta, delta):
    # a weighted (4, 4) fit through the same kernel: element parity with the oracle's
    # evaluation of the same coefficients, and the device's error statistics over a
    # subsample of the cube equal the oracle metric of the device output
    from oracle import colour as C
    ap = M.fit(M.FN_CBRT, 4, 4, 0.008856, 1.0, weight=M.dark_end_weight(beta, delta))
    p = M.make_params(0, [ap])
    img = synth.cube_u8().reshape(-1, 3)[::61].reshape(1, -1, 3)
    gpu = _run(M, img, 0, p)
    P.assert_parity(0, gpu, P.oracle(0, img / 255.0, P.coeffs(p)))
    st = M.error_stats(torch.from_numpy(np.ascontiguousarray(img)).cuda(), params=p)
    d = C.delta_e(gpu.reshape(-1, 3).astype(np.float64), C.rgb_to_lab(img.reshape(-1, 3) / 255.0))
    assert st["mean"] == pytest.approx(d.mean(), rel=1e-9, abs=1e-11)
    assert st["max"] == pytest.approx(d.max(), rel=1e-9, abs=1e-11)


def _cube_cmp(v8, start, shared, xform, co):
    g = shared[start:start + len(v8)]
    return P.max_scaled_err(xform, g, P.oracle(xform, v8 / 255.0, co))


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_exhaustive_cube(M, xform):
    # every 8-bit colour once (4096 x 4096)
    cube = synth.cube_u8()
    p = M.default_params(xform)
    gpu = _run(M, cube, xform, p).reshape(-1, 3)
    errs = cube_map_shared(_cube_cmp, gpu, xform, P.coeffs(p))
    e = np.max(np.stack(errs), axis=0)
    assert np.all(e <= P.REL), e


@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (3, 7), (17, 33), (255, 257)])
@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_ragged_sizes_and_special_colours(M, shape, xform):
    img = synth.uniform_u8(*shape, seed=sum(shape))
    special = np.array([[0, 0, 0], [255, 255, 255], [128, 128, 128], [255, 0, 0], [0, 255, 0], [0, 0, 255],
                        [0, 7, 7], [7, 0, 0], [0, 0, 9], [200, 200, 10], [10, 200, 200], [200, 10, 200]], np.uint8)
    flat = img.reshape(-1, 3)
    k = min(len(flat), len(special))
    flat[:k] = special[:k]
    p = M.default_params(xform)
    gpu = _run(M, img, xform, p)
    P.assert_parity(xform, gpu, P.oracle(xform, img / 255.0, P.coeffs(p)))


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_float_inputs_layouts_and_clamp(M, xform):
    g = synth.rng(21)
    x = g.uniform(-0.1, 1.1, (2, 3, 61, 67)).astype(np.float32)  # N C H W, some values clamp
    p = M.default_params(xform)
    gamma = "none"
    gpu = _run(M, x, xform, p, layout="chw", gamma=gamma)
    ref = P.oracle(xform, np.moveaxis(x.astype(np.float64), 1, -1), P.coeffs(p), gamma=gamma)
    ref = np.moveaxis(ref, -1, 1)
    # float inputs: a pixel within a relative 1e-6 of a branch boundary must equal the oracle on
    # one of the two sides
    P.assert_parity_ties(xform, np.moveaxis(gpu, 1, -1), np.moveaxis(x.astype(np.float64), 1, -1),
                         P.coeffs(p), gamma=gamma)


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_f32_hwc_fast_path(M, xform):
    # packed float32 HWC (the LDS-staged kernel; ragged tails, values outside [0, 1]) equals a
    # row-padded view of the same values (the one-pixel kernel) bitwise, fp32 and fp16 out, and the
    # oracle to the parity bar (the SCT branch guard for float inputs)
    g = synth.rng(40 + xform)
    pars = [M.default_params(xform)]
    if xform in (0, 3):
        pars += [M.make_params(xform, [M.paper_approx(M.FN_CBRT, 4, 4)]), M.default_params(xform, decode=True)]
    for shape in [(1, 1, 3), (3, 7, 5), (2, 16, 32), (1, 37, 300)]:
        x = g.uniform(-0.1, 1.1, shape + (3,)).astype(np.float32)
        packed = torch.from_numpy(x).cuda()
        big = torch.zeros(shape[:2] + (shape[2] + 1, 3), dtype=torch.float32, device="cuda")
        big[:, :, :shape[2]] = packed
        view = big[:, :, :shape[2]]
        for p in pars:
            for gm in (["bt709", "srgb", "none"] if xform in (0, 3) else ["none"]):
                for od in (torch.float32, torch.float16):
                    a = M.transform(packed, xform=xform, params=p, gamma=gm, out_dtype=od)
                    b = M.transform(view, xform=xform, params=p, gamma=gm, out_dtype=od)
                    torch.cuda.synchronize()
                    assert torch.equal(a, b), (shape, gm, od)
    p = M.default_params(xform)
    x = g.uniform(-0.1, 1.1, (2, 33, 129, 3)).astype(np.float32)
    gpu = _run(M, x, xform, p, gamma="none").reshape(-1, 3).astype(np.float64)
    P.assert_parity_ties(xform, gpu, x.astype(np.float64).reshape(-1, 3), P.coeffs(p), gamma="none")


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_u8_input_f16_output(M, xform):
    # C1 through the float16-output form of the hot kernel (9 bytes per pixel moved):
    # the oracle value rounded to float16 within one half-unit of the float16 result
    img = synth.uniform_u8(512, 512, seed=1)
    p = M.default_params(xform)
    gpu16 = _run(M, img, xform, p, out_dtype=torch.float16).astype(np.float64)
    ref = P.oracle(xform, img.reshape(-1, 3) / 255.0, P.coeffs(p)).reshape(gpu16.shape)
    tol = np.abs(ref) * 2.0 ** -11 + 2e-6 * np.asarray(P.SCALE[xform]) + 2.0 ** -25
    assert np.all(np.abs(gpu16 - ref) <= tol)


@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_f16_input_and_f16_output(M, xform):
    g = synth.rng(22)
    xh = g.random((40, 50, 3)).astype(np.float16)
    p = M.default_params(xform)
    gamma = "none"
    gpu = _run(M, xh, xform, p, gamma=gamma)
    ref = P.oracle(xform, xh.astype(np.float64), P.coeffs(p), gamma=gamma)
    P.assert_parity(xform, gpu, ref)
    # float16 output: the oracle value rounded to float16 within one half-unit
    gpu16 = _run(M, xh, xform, p, gamma=gamma, out_dtype=torch.float16).astype(np.float64)
    tol = np.abs(ref) * 2.0 ** -11 + 2e-6 * P.SCALE[xform]
    assert np.all(np.abs(gpu16 - ref) <= tol)


def test_lab_gamma_options_on_float_input(M):
    g = synth.rng(23)
    x = g.random((33, 31, 3)).astype(np.float32)
    p = M.default_params(0)
    for gamma in ("bt709", "srgb"):
        gpu = _run(M, x, 0, p, gamma=gamma)
        P.assert_parity(0, gpu, P.oracle(0, x.astype(np.float64), P.coeffs(p), gamma=gamma), what=gamma)
    for gamma in ("srgb", "none"):
        img = synth.uniform_u8(20, 21, seed=4)
        gpu = _run(M, img, 0, p, gamma=gamma)
        P.assert_parity(0, gpu, P.oracle(0, img / 255.0, P.coeffs(p), gamma=gamma), what="u8 " + gamma)


VIEW_CASES = [  # (images, rows, width, row padding px, padding rows per image)
    (2, 3, 4, 0, 1), (1, 5, 256, 4, 0), (3, 7, 260, 12, 2), (2, 4, 1000, 8, 0), (1, 2, 1028, 4, 3),
    (2, 3, 20, 3, 0),  # rows of 23 pixels: an 8-bit row stride that is not a multiple of 4 bytes
    (1, 3, 18, 2, 0),  # a width that is not a multiple of 4
]


def _base(g, dtype, shape):
    if dtype == "u8":
        return g.integers(0, 256, shape).astype(np.uint8)
    if dtype == "u16":
        return g.integers(0, 65536, shape).astype(np.uint16)
    if dtype == "f16":
        return g.random(shape).astype(np.float16)
    return g.uniform(-0.05, 1.05, shape).astype(np.float32)


@pytest.mark.parametrize("dtype", ["u8", "f16", "u16", "f32"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_row_strided_views_equal_packed(M, dtype, xform):
    # crops of padded rows and images (the row-strided kernel where rows hold a multiple of 4 pixels
    # and the strides are whole words, 16-byte units for float32; the one-pixel kernel otherwise)
    # give the packed input's bits
    g = synth.rng(200 + xform)
    pars = [M.default_params(xform), M.make_params(xform, [M.paper_approx(M.FN_CBRT, 4, 4)])] if xform in (0, 3) \
        else [M.default_params(xform)]
    if xform in (0, 3) and dtype != "u8":
        pars.append(M.default_params(xform, decode=True))
    for (n, h, w, rpad, ipad) in VIEW_CASES:
        base = _base(g, dtype, (n, h + ipad, w + rpad, 3))
        view = torch.from_numpy(base).cuda()[:, :h, :w]
        packed = torch.from_numpy(np.ascontiguousarray(base[:, :h, :w])).cuda()
        for p in pars:
            for gm in (["bt709", "none"] if xform in (0, 3) else ["none"]):
                for od in (torch.float32, torch.float16):
                    a = M.transform(view, xform=xform, params=p, gamma=gm, out_dtype=od)
                    b = M.transform(packed, xform=xform, params=p, gamma=gm, out_dtype=od)
                    torch.cuda.synchronize()
                    assert a.dtype == od and torch.equal(a, b), (n, h, w, rpad, ipad, gm, od)


@pytest.mark.parametrize("dtype", ["u8", "u16", "f16", "f32"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_chw_inputs_equal_packed_hwc(M, dtype, xform):
    # CHW planes into CHW and into HWC, float32 or float16 (the 4-pixel kernels where W H is a
    # multiple of 4, the one-pixel kernel otherwise; a partial last chunk at 3 x 8 x 1000) give the
    # bits of the packed HWC input
    g = synth.rng(300 + xform)
    # (2, 32, 64) and (3, 16, 128): planes of a multiple of 1024 pixels
    for (n, h, w) in [(2, 16, 20), (1, 33, 36), (3, 8, 1000), (1, 7, 9), (2, 32, 64), (3, 16, 128)]:
        if dtype in ("u8", "u16"):
            hwc = g.integers(0, 256 if dtype == "u8" else 65536, (n, h, w, 3)).astype(np.uint8 if dtype == "u8" else np.uint16)
        else:
            hwc = g.uniform(-0.05, 1.05, (n, h, w, 3)).astype(np.float16 if dtype == "f16" else np.float32)
        chw = torch.from_numpy(np.ascontiguousarray(np.moveaxis(hwc, -1, 1))).cuda()
        x = torch.from_numpy(hwc).cuda()
        for gm in (["bt709", "srgb", "none"] if xform in (0, 3) else ["none"]):
            p = M.default_params(xform)
            for od in (torch.float32, torch.float16):
                a = M.transform(chw, xform=xform, params=p, layout="chw", gamma=gm, out_dtype=od)
                c = M.transform(chw, xform=xform, params=p, layout="chw", out_layout="hwc", gamma=gm, out_dtype=od)
                b = M.transform(x, xform=xform, params=p, gamma=gm, out_dtype=od)
                torch.cuda.synchronize()
                assert a.dtype == od and torch.equal(a, b.permute(0, 3, 1, 2).contiguous()), (n, h, w, gm, od)
                assert c.dtype == od and torch.equal(c, b), (n, h, w, gm, od)


@pytest.mark.parametrize("dtype", ["u8", "u16", "f16", "f32"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_chw_row_views_equal_packed(M, dtype, xform):
    # crops of CHW planes and batches with gaps between images (the row-strided CHW kernel where rows
    # hold a multiple of 4 pixels and every stride is a multiple of 4 elements, the one-pixel kernel
    # otherwise), into CHW and HWC, float32 and float16: the packed HWC input's bits
    g = synth.rng(600 + xform)
    cases = VIEW_CASES + [(3, 6, 12, 0, 0)]  # the last one: 4 planes per image, the fourth skipped
    for (n, h, w, rpad, ipad) in cases:
        extra = 1 if (rpad, ipad) == (0, 0) else 0
        base = _base(g, dtype, (n, 3 + extra, h + ipad, w + rpad))
        view = torch.from_numpy(base).cuda()[:, :3, :h, :w]
        hwc = torch.from_numpy(np.ascontiguousarray(np.moveaxis(base[:, :3, :h, :w], 1, -1))).cuda()
        for gm in (["bt709", "none"] if xform in (0, 3) else ["none"]):
            p = M.default_params(xform)
            for od in (torch.float32, torch.float16):
                a = M.transform(view, xform=xform, params=p, layout="chw", gamma=gm, out_dtype=od)
                c = M.transform(view, xform=xform, params=p, layout="chw", out_layout="hwc", gamma=gm, out_dtype=od)
                b = M.transform(hwc, xform=xform, params=p, gamma=gm, out_dtype=od)
                torch.cuda.synchronize()
                assert a.dtype == od and torch.equal(a, b.permute(0, 3, 1, 2).contiguous()), (n, h, w, rpad, ipad, gm, od)
                assert c.dtype == od and torch.equal(c, b), (n, h, w, rpad, ipad, gm, od)


def test_empty_inputs_give_empty_outputs(M):
    # an empty batch or image is a no-op with an empty result (the C ABI reads batch 0 as one
    # image, so the binding never describes an empty tensor to it)
    for shape in [(0, 8, 8, 3), (2, 0, 8, 3), (1, 8, 0, 3)]:
        x = torch.zeros(shape, dtype=torch.uint8, device="cuda")
        y = M.transform(x, xform="lab")
        assert y.shape == shape and y.dtype == torch.float32
        assert M.transform(x.float(), xform="hsi", out_dtype=torch.float16).shape == shape
        assert M.inverse(x.float(), xform="sct").shape == shape
        assert M.error_stats(x, xform="lab")["count"] == 0
        lut = M.lut_build("lab", 17)
        assert M.lut_interp(lut, 17, "lab", "tetrahedral", x).shape == shape
        xc = torch.zeros((shape[0], 3, shape[1], shape[2]), dtype=torch.float32, device="cuda")
        assert M.transform_backward(xc, xc.clone()).shape == xc.shape
        with pytest.raises(ValueError):
            M.image(x)
    # broadcast views (zero strides) are refused rather than read past their storage
    row = torch.zeros((1, 7, 3), dtype=torch.uint8, device="cuda")
    for v in (row.expand(5, 7, 3), row.unsqueeze(0).expand(4, 1, 7, 3).expand(4, 6, 7, 3)):
        with pytest.raises(ValueError):
            M.transform(v)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["u8", "u16", "f16", "f32"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_hwc_to_chw_equals_hwc_permuted(M, dtype, xform):
    # packed HWC into packed float32 or float16 CHW (the 4-pixel kernel where W H is a multiple of
    # 4, the one-pixel kernel otherwise) gives the HWC result's bits, plane by plane
    g = synth.rng(400 + xform)
    for (n, h, w) in [(2, 16, 20), (1, 33, 36), (3, 8, 1000), (1, 7, 9)]:
        if dtype == "u8":
            a = g.integers(0, 256, (n, h, w, 3)).astype(np.uint8)
        elif dtype == "u16":
            a = g.integers(0, 65536, (n, h, w, 3)).astype(np.uint16)
        else:
            a = g.uniform(-0.05, 1.05, (n, h, w, 3)).astype(np.float16 if dtype == "f16" else np.float32)
        x = torch.from_numpy(a).cuda()
        pars = [M.default_params(xform)] + ([M.default_params(xform, decode=True)] if xform in (0, 3) else [])
        for p in pars:
            for gm in (["bt709", "none"] if xform in (0, 3) else ["none"]):
                for od in (torch.float32, torch.float16):
                    c = M.transform(x, xform=xform, params=p, gamma=gm, out_layout="chw", out_dtype=od)
                    r = M.transform(x, xform=xform, params=p, gamma=gm, out_dtype=od)
                    torch.cuda.synchronize()
                    assert c.dtype == od and torch.equal(c, r.permute(0, 3, 1, 2).contiguous()), (n, h, w, gm, od)


def test_chw_batch_with_gaps_between_images(M):
    # CHW images whose batch stride exceeds 3 planes (a slice of a 4-channel batch) are not packed:
    # every path must honour the batch stride (regression: the plane kernels once assumed it)
    g = synth.rng(500)
    base = g.integers(0, 256, (3, 4, 16, 20)).astype(np.uint8)
    view = torch.from_numpy(base).cuda()[:, :3]
    packed = torch.from_numpy(np.ascontiguousarray(base[:, :3])).cuda()
    for xf in (0, 1, 2, 3):
        for ol in ("chw", "hwc"):
            for od in (torch.float32, torch.float16):
                a = M.transform(view, xform=xf, layout="chw", out_layout=ol, out_dtype=od)
                b = M.transform(packed, xform=xf, layout="chw", out_layout=ol, out_dtype=od)
                torch.cuda.synchronize()
                assert torch.equal(a, b), (xf, ol, od)
    f = torch.from_numpy(g.random((2, 4, 8, 12)).astype(np.float32)).cuda()
    a = M.inverse(f[:, :3], xform="sct", layout="chw")
    b = M.inverse(f[:, :3].contiguous(), xform="sct", layout="chw")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_strided_views(M):
    # a row-strided HWC view and a non-packed output take the general kernel: same values
    img = synth.uniform_u8(64, 80, seed=5)
    base = torch.from_numpy(img).cuda()
    view = base[:, 8:72, :]
    p = M.default_params(0)
    out_big = torch.zeros((64, 100, 3), dtype=torch.float32, device="cuda")
    out = out_big[:, 10:74, :]
    M.transform(view, params=p, out=out)
    dense = M.transform(view.contiguous(), params=p)
    torch.cuda.synchronize()
    assert torch.equal(out, dense)
    P.assert_parity(0, out.cpu().numpy(), P.oracle(0, img[:, 8:72] / 255.0, P.coeffs(p)))


def test_batch_of_1080p_sampled(M):
    # the 64 x 1920 x 1080 smooth batch in the benchmark's launch shape; sampled pixels against the oracle
    n = 64
    imgs = synth.smooth_batch_u8(n, 1080, 1920, 1000)
    x = torch.from_numpy(imgs).cuda()
    g = synth.rng(99)
    idx = g.integers(0, n * 1080 * 1920, 200000)
    flat = imgs.reshape(-1, 3)[idx]
    for xform in (0, 1, 2, 3):
        p = M.default_params(xform)
        y = M.transform(x, xform=xform, params=p)
        torch.cuda.synchronize()
        gv = y.reshape(-1, 3)[torch.from_numpy(idx).cuda()].cpu().numpy()
        P.assert_parity(xform, gv, P.oracle(xform, flat / 255.0, P.coeffs(p)))
        del y


def _sample_check(M, x, y, xform, p, n_sample, seed):
    """Sampled pixels of a device batch against the oracle."""
    n = x.numel() // 3
    idx = torch.from_numpy(synth.rng(seed).integers(0, n, n_sample)).cuda()
    xs = x.reshape(-1, 3)[idx].cpu().numpy()
    gv = y.reshape(-1, 3)[idx].cpu().numpy()
    P.assert_parity(xform, gv, P.oracle(xform, xs / 255.0, P.coeffs(p)))


def test_batch_of_4k_sampled(M):
    # 32 x 3840 x 2160 uint8 (i.i.d. uniform bytes from a seeded device generator), in the
    # launch shape the benchmark's 4K form times; 200,000 sampled pixels per transform
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randint(0, 256, (32, 2160, 3840, 3), dtype=torch.uint8, device="cuda", generator=g)
    y = torch.empty((32, 2160, 3840, 3), dtype=torch.float32, device="cuda")
    for xform in (0, 1, 2, 3):
        p = M.default_params(xform)
        M.transform(x, xform=xform, params=p, out=y)
        torch.cuda.synchronize()
        _sample_check(M, x, y, xform, p, 200000, 40 + xform)
    del x, y
    torch.cuda.empty_cache()


def test_batch_spanning_two_launches(M):
    # 2 x 32768 x 32768 = 2^31 pixels: one launch covers fewer than 2^31 pixels, so the batch
    # goes out as two launches; pixels on both sides of the split and at both ends are checked
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randint(0, 256, (2, 32768, 32768, 3), dtype=torch.uint8, device="cuda", generator=g)
    y = torch.empty((2, 32768, 32768, 3), dtype=torch.float32, device="cuda")
    p = M.default_params(0)
    M.transform(x, params=p, out=y)
    torch.cuda.synchronize()
    _sample_check(M, x, y, 0, p, 100000, 50)
    n1 = 32768 * 32768
    edge = torch.tensor([0, 1, n1 - 2, n1 - 1, n1, n1 + 1, 2 * n1 - 1], device="cuda")
    xs = x.reshape(-1, 3)[edge].cpu().numpy()
    gv = y.reshape(-1, 3)[edge].cpu().numpy()
    P.assert_parity(0, gv, P.oracle(0, xs / 255.0, P.coeffs(p)))
    del x, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f16", "f32"])
@pytest.mark.parametrize("layout", ["hwc", "chw", "strided"])
def test_lab_float_input_with_minimax_decoding(M, dtype, layout):
    # BT.709-encoded float inputs with the decoding power replaced by its minimax polynomial
    # (on the fast HWC / CHW kernels and the general one) against the oracle with the same
    # float32 coefficients; inputs within 1e-6 of the 0.081 branch point may take either branch
    g = synth.rng(70)
    x = g.random((2, 45, 67, 3)) * 1.1 - 0.05
    x[0, 0, :5] = [[0.081, 0.5, 1.0], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.0809, 0.0811, 0.2], [1.2, -0.1, 0.5]]
    npdt = np.float16 if dtype == "f16" else np.float32
    xq = x.astype(npdt)
    p = M.default_params(0, decode=True)
    t = torch.from_numpy(xq).cuda()
    if layout == "chw":
        y = M.transform(t.permute(0, 3, 1, 2).contiguous(), params=p, layout="chw", out_layout="hwc")
    elif layout == "strided":
        big = torch.zeros((2, 45, 70, 3), dtype=t.dtype, device="cuda")
        big[:, :, :67] = t
        y = M.transform(big[:, :, :67], params=p)
    else:
        y = M.transform(t, params=p)
    torch.cuda.synchronize()
    gpu = y.reshape(-1, 3).cpu().numpy().astype(np.float64)
    xs = xq.astype(np.float64).reshape(-1, 3)
    co = P.coeffs(p)
    dec = np.float32(p.f[1].p_list).astype(np.float64)
    # a channel within 1e-6 of 0.081 (the fixture puts one there) must match one of the two branches
    P.assert_parity_ties(0, gpu, xs, co, gamma="bt709", decode=dec)
    # and it differs from the exact-power path (the approximation is in use)
    exact = M.transform(t, params=M.default_params(0)).reshape(-1, 3).cpu().numpy()
    assert np.abs(exact - gpu).max() > 0


def test_batched_decoding_equals_plain(M):
    # the decoding polynomial travels in the batched form's coefficient table
    g = torch.Generator(device="cuda").manual_seed(71)
    ins = [torch.rand((h, w, 3), device="cuda", generator=g).half() for (h, w) in [(33, 40), (64, 64), (17, 300)]]
    outs = [torch.empty(i.shape, dtype=torch.float32, device="cuda") for i in ins]
    p = M.default_params(0, decode=True)
    M.batch_run([p] * 3, ins, outs, gammas=["bt709"] * 3)
    torch.cuda.synchronize()
    for i, o in zip(ins, outs):
        assert torch.equal(o, M.transform(i, params=p))


@pytest.mark.parametrize("layout", ["hwc", "chw", "strided"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3], ids=["lab", "hsi", "sct", "luv"])
def test_u16_inputs(M, xform, layout):
    # 16-bit codes (full range, v / 65535) on the fast HWC kernel and the general one, every transfer
    # function for CIELAB / CIELUV, the minimax decoding too; against the oracle on v / 65535.  Branch
    # guards as for float inputs: SCT pixels within 1e-6 (relative) of a branch plane
    g = synth.rng(80 + xform)
    c = g.integers(0, 65536, (2, 29, 71, 3)).astype(np.uint16)
    c[0, 0, :6] = [[0, 0, 0], [65535, 65535, 65535], [65535, 0, 0], [0, 65535, 0], [1, 2, 3], [5308, 5309, 40000]]
    # torch has few 16-bit unsigned kernels on the GPU: every layout is built on the host
    t = torch.from_numpy(c).cuda()
    t_chw = torch.from_numpy(np.ascontiguousarray(np.moveaxis(c, -1, 1))).cuda()
    big = np.zeros((2, 29, 75, 3), dtype=np.uint16)
    big[:, :, :71] = c
    t_strided = torch.from_numpy(big).cuda()[:, :, :71]
    x01 = c.astype(np.float64).reshape(-1, 3) / 65535.0
    cases = [("bt709", False), ("srgb", False), ("none", False), ("bt709", True)] if xform in (0, 3) else [("none", False)]
    for gm, dec in cases:
        p = M.default_params(xform, decode=dec)
        if layout == "chw":
            y = M.transform(t_chw, xform=xform, params=p, layout="chw", gamma=gm, out_layout="hwc")
        elif layout == "strided":
            y = M.transform(t_strided, xform=xform, params=p, gamma=gm)
        else:
            y = M.transform(t, xform=xform, params=p, gamma=gm)
        torch.cuda.synchronize()
        gpu = y.reshape(-1, 3).cpu().numpy().astype(np.float64)
        co = P.coeffs(p)
        decode = np.float32(p.f[1].p_list).astype(np.float64) if dec else None
        P.assert_parity_ties(xform, gpu, x01, co, gamma=gm, decode=decode, what="%s decode=%s" % (gm, dec))


def test_u16_error_stats_and_lut(M):
    # the device's statistics on 16-bit input equal the oracle's metric of the GPU output; the LUT
    # locates 16-bit codes as normalised floats
    from oracle import colour as C, lut as OL
    g = synth.rng(88)
    c = g.integers(0, 65536, (300, 301, 3)).astype(np.uint16)
    t = torch.from_numpy(c).cuda()
    x01 = c.astype(np.float64).reshape(-1, 3) / 65535.0
    p = M.default_params(0)
    y = M.transform(t, params=p).reshape(-1, 3).double().cpu().numpy()
    st = M.error_stats(t, params=p)
    d = C.delta_e(y, C.rgb_to_lab(x01))
    assert st["mean"] == pytest.approx(d.mean(), rel=1e-9) and st["max"] == pytest.approx(d.max(), rel=1e-9)
    L = M.lut_build("lab", 17)
    out = M.lut_interp(L, 17, "lab", "tetrahedral", t)
    torch.cuda.synchronize()
    # the kernel normalises a code as the float32 product code x float32(1/65535); given that same
    # input the oracle's interpolation differs from the GPU's by float32 weights and sums only
    # (x (N - 1) and the fraction are exact for N - 1 = 16): the parity bar per channel
    xg = (c.reshape(-1, 3).astype(np.float32) * np.float32(1.0 / 65535.0)).astype(np.float64)
    ref, _ = OL.interp(OL.build("lab", 17), "lab", "tetrahedral", x=xg)
    err = np.abs(out.reshape(-1, 3).cpu().numpy() - ref.reshape(-1, 3)).max(axis=0) / np.array(P.SCALE[0])
    assert err.max() <= P.REL, err
