"""GPU backward of the minimax RGB->CIELAB transform (mact_transform_backward,
MactLab) against the oracle's FP64 analytic gradient and central finite
differences."""
import numpy as np
import pytest

import synth
from oracle import colour, grad as OG
from tests import parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _pq(p):
    c = P.coeffs(p)
    return c["p"], c["q"]


def _check_vjp(gpu, ref):
    # float32: relative to the largest component of the pixel's gradient
    scale = np.abs(ref).max(axis=-1, keepdims=True)
    err = np.abs(gpu - ref) / np.maximum(scale, 1e-30)
    # float32 cancellation in 116 g_L - 500 g_a + 200 g_b: about 1e-5 of the largest component
    assert err.max() <= 1e-4, err.max()


def test_vjp_matches_fp64_analytic(M):
    g = synth.rng(41)
    x = g.uniform(-0.05, 1.05, (2, 3, 37, 53)).astype(np.float32)
    go = g.normal(size=x.shape).astype(np.float32)
    p = M.default_params(0)
    xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(go).cuda()
    dx = M.transform_backward(xt, gt, params=p, layout="chw")
    torch.cuda.synchronize()
    gpu = np.moveaxis(dx.cpu().numpy().astype(np.float64), 1, -1).reshape(-1, 3)
    xs = np.moveaxis(x.astype(np.float64), 1, -1).reshape(-1, 3)
    gs = np.moveaxis(go.astype(np.float64), 1, -1).reshape(-1, 3)
    pp, qq = _pq(p)
    ref = OG.vjp(xs, gs, pp, qq)
    # pixels within float32 rounding of the breakpoint may take either branch
    Mw = colour.M_RGB_XYZ / colour.WHITE_D65[:, None]
    t = np.clip(xs, 0, 1) @ Mw.T
    ok = ~(np.abs(t / colour.LAB_T0 - 1) < 1e-6).any(1)
    _check_vjp(gpu[ok], ref[ok])
    # outside [0, 1] the gradient is exactly zero
    out = (xs < 0) | (xs > 1)
    assert np.all(gpu[out] == 0)


def test_c4_full_size_sampled(M):
    # 32 x 3 x 512 x 512 linear RGB, U[0, 1] (seed 4); sampled pixels against the oracle
    x = torch.from_numpy(synth.uniform_f32((32, 3, 512, 512), seed=4)).cuda()
    go = torch.randn(x.shape, generator=torch.Generator(device="cuda").manual_seed(5), device="cuda")
    p = M.default_params(0)
    dx = M.transform_backward(x, go, params=p, layout="chw")
    torch.cuda.synchronize()
    g = synth.rng(6)
    n, h, w = g.integers(0, 32, 5000), g.integers(0, 512, 5000), g.integers(0, 512, 5000)
    xs = x[n, :, h, w].double().cpu().numpy()
    gs = go[n, :, h, w].double().cpu().numpy()
    gpu = dx[n, :, h, w].double().cpu().numpy()
    pp, qq = _pq(p)
    _check_vjp(gpu, OG.vjp(xs, gs, pp, qq))


def test_autograd_loss_gradient_vs_analytic_and_finite_differences(M):
    # loss = mean Delta E*ab to a seeded target; MactLab's gradient against the FP64 analytic
    # gradient of the same loss, and against central differences (h = 1e-3) within their
    # own truncation error
    g = synth.rng(7)
    N, H, W = 2, 24, 40
    x = torch.from_numpy(g.random((N, 3, H, W)).astype(np.float32)).cuda().requires_grad_(True)
    tgt_np = colour.rgb_to_lab(g.random((N, H, W, 3)), gamma="none")
    tgt = torch.from_numpy(np.moveaxis(tgt_np, -1, 1).astype(np.float32)).cuda()
    p = M.default_params(0)
    lab = M.MactLab.apply(x, p)
    loss = torch.sqrt(((lab - tgt) ** 2).sum(1)).mean()
    loss.backward()
    gpu = np.moveaxis(x.grad.double().cpu().numpy(), 1, -1).reshape(-1, 3)
    xs = np.moveaxis(x.detach().double().cpu().numpy(), 1, -1).reshape(-1, 3)
    ts = tgt_np.reshape(-1, 3)
    pp, qq = _pq(p)
    npx = N * H * W
    # the loss's own rounding: the forward Lab is float32, so compare with the analytic
    # gradient evaluated at the float32 Lab output
    lab_gpu = np.moveaxis(lab.detach().double().cpu().numpy(), 1, -1).reshape(-1, 3)
    d = lab_gpu - ts
    gl = d / np.sqrt((d * d).sum(1, keepdims=True)) / npx
    an = OG.vjp(xs, gl, pp, qq)
    _check_vjp(gpu, an)
    # finite differences of the per-pixel term (FP64), guard band around the breakpoint and clamp
    h = 1e-3
    fd = OG.fd_loss_grad_pixel(xs, ts, pp, qq, h=h) / npx
    fd2 = OG.fd_loss_grad_pixel(xs, ts, pp, qq, h=h / 2) / npx
    Mw = colour.M_RGB_XYZ / colour.WHITE_D65[:, None]
    t = xs @ Mw.T
    ok = ~((np.abs(t - colour.LAB_T0) <= 2 * h * np.abs(Mw).sum(1).max()).any(1) | ((xs < h) | (xs > 1 - h)).any(1))
    bound = 2.0 * np.abs(fd - fd2) + 1e-4 * np.abs(an).max(axis=1, keepdims=True)
    assert np.all((np.abs(gpu - fd) <= bound)[ok])
