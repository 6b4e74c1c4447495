"""Every specialised kernel gives the same bits as the general kernels on the
same data (forced with padded-stride views: k_gather for inputs and output
views, k_generic for outputs not aligned to their element), for every
transform, input type and transfer function."""
import numpy as np
import pytest

import synth
from tests import parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _padded_hwc(x, pad=3):
    """The same pixels in a tensor whose rows are `pad` pixels wider (not packed)."""
    h, w = x.shape[-3], x.shape[-2]
    big = torch.zeros(x.shape[:-3] + (h, w + pad, 3), dtype=x.dtype, device=x.device)
    big[..., :, :w, :] = x
    return big[..., :, :w, :]


def _padded_chw(x, pad=5):
    h, w = x.shape[-2], x.shape[-1]
    big = torch.zeros(x.shape[:-1] + (w + pad,), dtype=x.dtype, device=x.device)
    big[..., :w] = x
    return big[..., :w]


SHAPES = [(1, 4), (5, 7), (64, 96), (257, 300)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", ["u8", "u16", "f16"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3])
def test_hwc_fast_equals_general(M, xform, dtype, shape):
    g = torch.Generator(device="cuda").manual_seed(sum(shape) + xform)
    if dtype == "u8":
        x = torch.randint(0, 256, (2,) + shape + (3,), dtype=torch.uint8, device="cuda", generator=g)
        gammas = ["bt709", "srgb", "none"] if xform in (0, 3) else ["bt709"]
    elif dtype == "u16":
        c = np.random.default_rng(sum(shape) + xform).integers(0, 65536, (2,) + shape + (3,)).astype(np.uint16)
        x = torch.from_numpy(c).cuda()
        gammas = ["bt709", "srgb", "none"] if xform in (0, 3) else ["none"]
    else:
        x = (torch.rand((2,) + shape + (3,), device="cuda", generator=g) * 1.1 - 0.05).half()
        gammas = ["none", "bt709"] if xform in (0, 3) else ["none"]
    p = M.default_params(xform)
    if dtype == "u16":
        # torch has few 16-bit unsigned kernels on the GPU: build the padded copy on the host
        big = np.zeros((2, shape[0], shape[1] + 3, 3), dtype=np.uint16)
        big[:, :, :shape[1]] = c
        padded = torch.from_numpy(big).cuda()[:, :, :shape[1]]
    else:
        padded = _padded_hwc(x)
    for gm in gammas:
        fast = M.transform(x, params=p, gamma=gm)
        general = M.transform(padded, params=p, gamma=gm)
        torch.cuda.synchronize()
        assert torch.equal(fast, general), (gm,)
    if dtype == "f16":
        # and against the oracle
        xs = np.clip(x.float().cpu().numpy().astype(np.float64), 0, 1).reshape(-1, 3)
        got = M.transform(x, params=p, gamma=gammas[0]).reshape(-1, 3).cpu().numpy()
        P.assert_parity_ties(xform, got, xs, P.coeffs(p), gamma=gammas[0])


@pytest.mark.parametrize("shape", SHAPES + [(33, 31)])
@pytest.mark.parametrize("dtype", ["u8", "f16"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3])
def test_hwc_f16_output_fast_equals_general(M, xform, dtype, shape):
    # float16 output: the fast kernel rounds in the same place as the general one
    g = torch.Generator(device="cuda").manual_seed(7 * sum(shape) + xform)
    if dtype == "u8":
        x = torch.randint(0, 256, (3,) + shape + (3,), dtype=torch.uint8, device="cuda", generator=g)
        gm = "bt709" if xform in (0, 3) else "none"
    else:
        x = (torch.rand((3,) + shape + (3,), device="cuda", generator=g) * 1.1 - 0.05).half()
        gm = "none"
    p = M.default_params(xform)
    fast = M.transform(x, params=p, gamma=gm, out_dtype=torch.float16)
    general = _padded_hwc(torch.zeros(x.shape, dtype=torch.float16, device="cuda"))
    M.transform(x, params=p, gamma=gm, out=general)
    f32 = M.transform(x, params=p, gamma=gm)
    torch.cuda.synchronize()
    assert torch.equal(fast, general)
    assert torch.equal(fast, f32.half())  # round to nearest even of the float32 result


@pytest.mark.parametrize("hw", [(4, 1), (16, 24), (64, 64), (129, 20)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
@pytest.mark.parametrize("xform", [0, 1, 2, 3])
def test_chw_fast_equals_general(M, xform, dtype, hw):
    g = torch.Generator(device="cuda").manual_seed(hw[0] * 7 + hw[1] + xform)
    x = (torch.rand((3, 3) + hw, device="cuda", generator=g) * 1.1 - 0.05).to(dtype)
    p = M.default_params(xform)
    gm = "none"
    fast = M.transform(x, params=p, layout="chw", gamma=gm)
    general = M.transform(_padded_chw(x), params=p, layout="chw", gamma=gm)
    torch.cuda.synchronize()
    assert torch.equal(fast, general)


@pytest.mark.parametrize("hw", [(8, 8), (64, 80), (33, 12)])
def test_backward_chw_fast_equals_general(M, hw):
    g = torch.Generator(device="cuda").manual_seed(hw[0] + hw[1])
    x = torch.rand((2, 3) + hw, device="cuda", generator=g) * 1.1 - 0.05
    go = torch.randn(x.shape, device="cuda", generator=g)
    p = M.default_params(0)
    fast = M.transform_backward(x, go, params=p)
    general = M.transform_backward(_padded_chw(x), _padded_chw(go), params=p)
    torch.cuda.synchronize()
    assert torch.equal(fast, general)


@pytest.mark.parametrize("N", [17, 33])
@pytest.mark.parametrize("method", ["trilinear", "prism", "pyramidal", "tetrahedral"])
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct"])
def test_lut_fast_equals_general(M, xform, method, N):
    g = torch.Generator(device="cuda").manual_seed(N)
    x = torch.randint(0, 256, (70, 333, 3), dtype=torch.uint8, device="cuda", generator=g)
    L = M.lut_build(xform, N)
    fast = M.lut_interp(L, N, xform, method, x)
    general = M.lut_interp(L, N, xform, method, _padded_hwc(x))
    torch.cuda.synchronize()
    assert torch.equal(fast, general)


def test_layout_change_hwc_to_chw(M):
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randint(0, 256, (2, 20, 30, 3), dtype=torch.uint8, device="cuda", generator=g)
    p = M.default_params(0)
    chw = M.transform(x, params=p, out_layout="chw")
    hwc = M.transform(x, params=p)
    torch.cuda.synchronize()
    assert chw.shape == (2, 3, 20, 30)
    assert torch.equal(chw.permute(0, 2, 3, 1), hwc)


def _src(dtype, shape, seed):
    """A packed HWC batch of 2 images on the host, values spanning the type's range."""
    rng = np.random.default_rng(seed)
    if dtype == "u8":
        return rng.integers(0, 256, (2,) + shape + (3,)).astype(np.uint8)
    if dtype == "u16":
        return rng.integers(0, 65536, (2,) + shape + (3,)).astype(np.uint16)
    x = (rng.random((2,) + shape + (3,)) * 1.1 - 0.05).astype(np.float32)
    return x.astype(np.float16) if dtype == "f16" else x


def _host_padded(a, last_pad):
    """Host array `a` on the GPU in a tensor whose last axis is `last_pad` wider, as a view of the
    original extent (built on the host: torch has few 16-bit unsigned kernels on the GPU)."""
    big = np.zeros(a.shape[:-1] + (a.shape[-1] + last_pad,), dtype=a.dtype)
    big[..., :a.shape[-1]] = a
    return torch.from_numpy(big).cuda()[..., :a.shape[-1]]


def _padded_rows_hwc(a):
    """Host array `a` (N, H, W, 3) on the GPU in a tensor whose rows are 3 pixels wider, as a view."""
    big = np.zeros(a.shape[:2] + (a.shape[2] + 3, 3), dtype=a.dtype)
    big[:, :, :a.shape[2]] = a
    return torch.from_numpy(big).cuda()[:, :, :a.shape[2]]


ODD_SHAPES = [(5, 7), (33, 31), (129, 67)]


@pytest.mark.parametrize("out_kind", ["hwc_f32", "hwc_f16", "chw_f32", "chw_f16"])
@pytest.mark.parametrize("src_kind", ["hwc_rows", "chw_packed", "chw_rows"])
@pytest.mark.parametrize("dtype", ["u8", "u16", "f16", "f32"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3])
def test_gather_equals_general(M, xform, dtype, src_kind, out_kind):
    # inputs no 4-pixel kernel takes (rows of an odd width, CHW planes of an odd W H) into packed
    # output go to k_gather; the same into a padded (strided) output view to k_generic: same bits
    p = M.default_params(xform)
    layout_out, odt = out_kind.split("_")
    odt = torch.float32 if odt == "f32" else torch.float16
    for si, shape in enumerate(ODD_SHAPES):
        x = _src(dtype, shape, 100 * xform + 10 * si + len(src_kind))
        chw = np.ascontiguousarray(x.transpose(0, 3, 1, 2))
        if src_kind == "hwc_rows":
            src, layout = _padded_rows_hwc(x), "hwc"
        elif src_kind == "chw_packed":
            src, layout = torch.from_numpy(chw).cuda(), "chw"
        else:
            src, layout = _host_padded(chw, 5), "chw"
        oshape = (2,) + shape + (3,) if layout_out == "hwc" else (2, 3) + shape
        packed = torch.empty(oshape, dtype=odt, device="cuda")
        zeros = np.zeros(oshape, dtype=np.float32 if odt == torch.float32 else np.float16)
        strided = _padded_rows_hwc(zeros) if layout_out == "hwc" else _host_padded(zeros, 2)
        gm = "bt709" if dtype in ("u8", "u16") else "none"
        M.transform(src, params=p, layout=layout, gamma=gm, out=packed, out_layout=layout_out)
        M.transform(src, params=p, layout=layout, gamma=gm, out=strided, out_layout=layout_out)
        torch.cuda.synchronize()
        assert torch.equal(packed, strided), (shape,)
        if dtype == "f32" and odt == torch.float32:
            xs = np.clip(x.astype(np.float64), 0, 1).reshape(-1, 3)
            got = packed if layout_out == "hwc" else packed.permute(0, 2, 3, 1)
            P.assert_parity_ties(xform, got.reshape(-1, 3).cpu().numpy(), xs, P.coeffs(p), gamma="none")


OUT_VIEW_SHAPES = [(64, 96), (33, 32), (16, 36), (6, 520)]  # 520: chunks inside one row and across two


@pytest.mark.parametrize("out_dt", [torch.float32, torch.float16])
@pytest.mark.parametrize("kind", ["hwc_u8", "hwc_u16", "hwc_f16", "hwc_f32", "chw_u8", "chw_f32"])
@pytest.mark.parametrize("xform", [0, 1, 2, 3])
def test_output_views_equal_packed(M, xform, kind, out_dt):
    # inputs a 4-pixel kernel takes, into packed output; the same into output views that are not
    # packed (HWC rows 3 pixels wider, CHW rows 2 wider): k_gather writes those from its lanes,
    # or a chunk inside one HWC row as 16-byte groups, same bits, and nothing outside the view.
    # 2 images of 33 x 32: chunks that straddle them; rows of 520: chunks inside one row, whose
    # runs start at every offset from a 16-byte boundary (rows of 523 pixels, 3 floats a pixel)
    layout, dt = kind.split("_")
    p = M.default_params(xform)
    gm = "bt709" if dt in ("u8", "u16") else "none"
    odt = np.float32 if out_dt == torch.float32 else np.float16
    for si, shape in enumerate(OUT_VIEW_SHAPES):
        x = _src(dt, shape, 31 * xform + 7 * si + len(kind))
        src = torch.from_numpy(np.ascontiguousarray(x.transpose(0, 3, 1, 2)) if layout == "chw" else x).cuda()
        for out_layout in ("hwc", "chw"):
            oshape = (2,) + shape + (3,) if out_layout == "hwc" else (2, 3) + shape
            packed = torch.empty(oshape, dtype=out_dt, device="cuda")
            if out_layout == "hwc":
                big = torch.from_numpy(np.zeros((2,) + (shape[0], shape[1] + 3, 3), dtype=odt)).cuda()
                view = big[:, :, :shape[1]]
            else:
                big = torch.from_numpy(np.zeros((2, 3) + (shape[0], shape[1] + 2), dtype=odt)).cuda()
                view = big[..., :shape[1]]
            M.transform(src, params=p, layout=layout, gamma=gm, out=packed, out_layout=out_layout)
            M.transform(src, params=p, layout=layout, gamma=gm, out=view, out_layout=out_layout)
            torch.cuda.synchronize()
            assert torch.equal(packed, view), (shape, out_layout)
            pad = big[:, :, shape[1]:] if out_layout == "hwc" else big[..., shape[1]:]
            assert not pad.any(), (shape, out_layout)
