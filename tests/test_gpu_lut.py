"""GPU parity of lut_build / lut_interp against the oracle's LUT
interpolators, node hits, and Table 12 reproduced from the GPU's own output."""
import numpy as np
import pytest

import synth
from oracle import colour, lut as OL
from tests import parity as P
from tests.cubepool import cube_map_shared

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

METHODS = ["trilinear", "prism", "pyramidal", "tetrahedral"]
XF = {"lab": 0, "hsi": 1, "sct": 2, "luv": 3}


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _interp(M, xform, N, method, x_np, layout="hwc"):
    L = M.lut_build(xform, N)
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    y = M.lut_interp(L, N, xform, method, x, layout=layout)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), L


def _compare(xform, gpu, ref, rlen, mask=None):
    """Linear channels: |gpu - ref| <= 2e-6 full scale.  Angular channels: the
    wrapped angle difference times the resultant length (the angle of a short
    resultant is ill-conditioned)."""
    xf = XF[xform]
    g = gpu.reshape(-1, 3)
    r = ref.reshape(-1, 3)
    rl = rlen.reshape(-1, 3)
    if mask is not None:
        g, r, rl = g[mask], r[mask], rl[mask]
    for ch, ang in enumerate(OL.ANGULAR[xform]):
        if ang:
            d = colour.angle_diff(g[:, ch], r[:, ch]) * rl[:, ch]
        else:
            d = np.abs(g[:, ch] - r[:, ch])
        worst = d.max() / P.SCALE[xf][ch]
        assert worst <= P.REL, (xform, ch, worst)


@pytest.mark.parametrize("N", [17, 33])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_u8_parity(M, xform, method, N):
    img = synth.uniform_u8(129, 131, seed=N)
    img.reshape(-1, 3)[:6] = [[0, 0, 0], [255, 255, 255], [128, 128, 128], [255, 0, 0], [0, 0, 255], [17, 17, 200]]
    gpu, _ = _interp(M, xform, N, method, img)
    ref, rlen = OL.interp(OL.build(xform, N), xform, method, v8=img)
    _compare(xform, gpu, ref, rlen)


@pytest.mark.parametrize("N", [2, 3, 5, 12, 16, 18, 19])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct"])
def test_u8_parity_odd_grid_sizes(M, xform, method, N):
    # grids staged in LDS are copied there with their G and R strides padded (to 3 and 9 mod 16
    # nodes), by an amount that depends on N (19: none; 18: 1 and 3; 2: 1 and 3; SCT 17^3 and
    # below only), and larger ones are read through the L2: parity for sizes on both sides
    img = synth.uniform_u8(67, 131, seed=N + 5)
    img.reshape(-1, 3)[:4] = [[0, 0, 0], [255, 255, 255], [255, 0, 0], [0, 0, 255]]
    gpu, _ = _interp(M, xform, N, method, img)
    ref, rlen = OL.interp(OL.build(xform, N), xform, method, v8=img)
    _compare(xform, gpu, ref, rlen)


@pytest.mark.parametrize("method", METHODS)
def test_float_inputs_and_chw(M, method):
    g = synth.rng(31)
    x = g.uniform(-0.05, 1.05, (3, 45, 47)).astype(np.float32)
    gpu, _ = _interp(M, "lab", 17, method, x, layout="chw")
    xc = np.moveaxis(x.astype(np.float64), 0, -1)
    ref, rlen = OL.interp(OL.build("lab", 17), "lab", method, x=xc)
    mask = None
    if method == "pyramidal":
        # the pyramidal form is discontinuous: skip inputs within float32 rounding of a
        # cell face or of a pyramid boundary (two fractions equal)
        pos = np.clip(xc.reshape(-1, 3), 0, 1) * 16
        f = pos - np.minimum(np.floor(pos), 15)
        near_face = (np.abs(pos - np.rint(pos)) < 1e-5).any(1)
        near_tie = (np.abs(f[:, 0] - f[:, 1]) < 1e-5) | (np.abs(f[:, 0] - f[:, 2]) < 1e-5) | (np.abs(f[:, 1] - f[:, 2]) < 1e-5)
        mask = ~(near_face | near_tie)
    _compare("lab", np.moveaxis(gpu, 0, -1), ref, rlen, mask)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("N", [9, 17, 33])
def test_node_hits_are_exact(M, method, N):
    # at the node inputs (exact binary fractions for N - 1 a power of two) the output is the
    # stored float32 node, bit for bit
    idx = np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = (idx / (N - 1.0)).astype(np.float32).reshape(1, -1, 3)
    gpu, L = _interp(M, "lab", N, method, x)
    nodes = L.cpu().numpy().reshape(N, N, N, 4)[..., :3].reshape(-1, 3)
    np.testing.assert_array_equal(gpu.reshape(-1, 3), nodes.astype(np.float64))
    # and the stored nodes are the exact transform rounded once
    ref = OL.build("lab", N).reshape(-1, 3)
    assert np.max(np.abs(nodes - ref) / P.SCALE[0]) < 1e-7


def _t12(v8, start, shared, key):
    out = shared[key][start:start + len(v8)]
    d = colour.delta_e(out, colour.rgb_to_lab(v8 / 255.0))
    return float(d.sum()), float(d.max())


def test_table12_from_gpu_output(M):
    # all 2^24 colours through the GPU interpolators reproduce Table 12 (trilinear, prism,
    # tetrahedral; the pyramidal row is unpinned) to the printed digits within float32 rounding
    from oracle import tables as T
    cube = torch.from_numpy(synth.cube_u8()).cuda()
    outs = {}
    for method in ("trilinear", "prism", "tetrahedral"):
        for N in (17, 33):
            L = M.lut_build("lab", N)
            outs[(method, N)] = M.lut_interp(L, N, "lab", method, cube).reshape(-1, 3).double().cpu().numpy()
    for key in list(outs):
        parts = cube_map_shared(_t12, outs, key)
        mean = sum(p[0] for p in parts) / float(1 << 24)
        mx = max(p[1] for p in parts)
        avg_p, max_p = T.T12_LUT_ERR[key]
        assert mean == pytest.approx(avg_p, abs=2e-6), key
        assert mx == pytest.approx(max_p, abs=2e-5), key


def test_lut_33_goes_through_l2_and_17_sct_through_lds(M):
    # sizes: 33^3 x 16 B does not fit 160 KB of LDS; 17^3 x 20 B (SCT) fits beside the 48 KB of
    # the 4-pixel kernel's store buffers
    assert M.lut_bytes("lab", 33) > 163840 >= M.lut_bytes("sct", 17) + 48 * 1024
    img = synth.uniform_u8(40, 41, seed=9)
    for xform, N in (("sct", 17), ("sct", 33), ("hsi", 33)):
        gpu, _ = _interp(M, xform, N, "tetrahedral", img)
        ref, rlen = OL.interp(OL.build(xform, N), xform, "tetrahedral", v8=img)
        _compare(xform, gpu, ref, rlen)


@pytest.mark.parametrize("N", [2, 9, 17, 33])
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct"])
def test_cells_hold_the_corner_nodes(M, xform, N):
    # cell (i, j, k), corner (dR dG dB): the packed node (i + dR, j + dG, k + dB), bit for bit
    L = M.lut_build(xform, N)
    C = M.lut_cells_build(L, N, xform)
    torch.cuda.synchronize()
    n3, m3 = N ** 3, 8 * (N - 1) ** 3
    nodes = L[:4 * n3].view(N, N, N, 4)
    cells = C[:4 * m3].view(N - 1, N - 1, N - 1, 8, 4)
    planes = [(nodes, cells)]
    if xform == "sct":  # the L planes after the float4 nodes
        assert M.lut_bytes(xform, N) == 4 * (4 * n3 + (n3 + 3) // 4 * 4)
        planes.append((L[4 * n3:5 * n3].view(N, N, N), C[4 * m3:5 * m3].view(N - 1, N - 1, N - 1, 8)))
    for nd, cl in planes:
        for c in range(8):
            dr, dg, db = c >> 2, (c >> 1) & 1, c & 1
            ref = nd[dr:dr + N - 1, dg:dg + N - 1, db:db + N - 1]
            assert torch.equal(cl[:, :, :, c], ref), c


@pytest.mark.parametrize("N", [17, 33])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct"])
def test_cells_interp_equals_packed(M, xform, method, N):
    # the cell-major form gives the packed form's bits: packed 8-bit HWC fast path (ragged
    # tail included), the general kernel through a strided view, and float CHW input
    g = torch.Generator(device="cuda").manual_seed(N + 3)
    x = torch.randint(0, 256, (3, 67, 331, 3), dtype=torch.uint8, device="cuda", generator=g)
    L = M.lut_build(xform, N)
    C = M.lut_cells_build(L, N, xform)
    a = M.lut_interp(L, N, xform, method, x)
    b = M.lut_cells_interp(C, N, xform, method, x)
    big = torch.zeros((3, 67, 334, 3), dtype=torch.uint8, device="cuda")
    big[:, :, :331] = x
    c = M.lut_cells_interp(C, N, xform, method, big[:, :, :331])
    xf = (torch.rand((2, 3, 33, 47), device="cuda", generator=g) * 1.1 - 0.05)
    d1 = M.lut_interp(L, N, xform, method, xf, layout="chw")
    d2 = M.lut_cells_interp(C, N, xform, method, xf, layout="chw")
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c) and torch.equal(d1, d2)


@pytest.mark.parametrize("method", METHODS)
def test_cells_u8_parity_33(M, method):
    # against the oracle directly, including the corner colours
    img = synth.uniform_u8(129, 131, seed=5)
    img.reshape(-1, 3)[:6] = [[0, 0, 0], [255, 255, 255], [128, 128, 128], [255, 0, 0], [0, 0, 255], [17, 17, 200]]
    L = M.lut_build("lab", 33)
    C = M.lut_cells_build(L, 33, "lab")
    y = M.lut_cells_interp(C, 33, "lab", method, torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    ref, rlen = OL.interp(OL.build("lab", 33), "lab", method, v8=img)
    _compare("lab", y.cpu().numpy().astype(np.float64), ref, rlen)
