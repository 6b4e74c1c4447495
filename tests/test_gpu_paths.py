"""Every specialised kernel gives the same bits as the general one-pixel-per-
lane kernel on the same data (the general kernel is forced with a padded-
stride view), for every transform, input type and transfer function."""
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
