"""The oracle's analytic gradient of the minimax CIELAB transform against
central finite differences in FP64 (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import colour, grad, mact, remez, tables as T

H = 1e-3


@pytest.fixture(scope="module")
def fit():
    return remez.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL)


def _guard(x):
    # finite differences straddling the breakpoint or the clamp are not derivatives
    Mw = colour.M_RGB_XYZ / colour.WHITE_D65[:, None]
    t = np.clip(x, 0, 1) @ Mw.T
    band = 2 * H * np.abs(Mw).sum(1).max()
    near_t0 = (np.abs(t - colour.LAB_T0) <= band).any(-1)
    near_clamp = ((x < H) | (x > 1 - H)).any(-1)
    return ~(near_t0 | near_clamp)


def test_loss_gradient_matches_finite_differences(fit):
    g = synth.rng(4)
    x = g.random((4096, 3))
    target = colour.rgb_to_lab(g.random((4096, 3)), gamma="none")
    an = grad.delta_e_loss_grad_pixel(x, target, fit.p, fit.q)
    ok = _guard(x)
    assert ok.mean() > 0.95
    scale = np.maximum(np.abs(an), 1e-3 * np.abs(an).max())
    # h = 1e-3: central differences are off by about C h^2; (fd_h - fd_{h/2}) estimates 3/4 of it
    fd = grad.fd_loss_grad_pixel(x, target, fit.p, fit.q, h=H)
    fd2 = grad.fd_loss_grad_pixel(x, target, fit.p, fit.q, h=H / 2)
    bound = 2.0 * np.abs(fd - fd2) + 1e-7 * np.abs(an).max()
    assert np.all((np.abs(an - fd) <= bound)[ok])
    # a small step leaves only rounding: relative agreement to 1e-5
    fds = grad.fd_loss_grad_pixel(x, target, fit.p, fit.q, h=1e-5)
    assert np.max(np.abs(an - fds)[ok] / scale[ok]) < 1e-5


def test_jacobian_matches_finite_differences_of_lab(fit):
    g = synth.rng(12)
    x = g.uniform(0.02, 0.98, (2000, 3))
    J = grad.jacobian(x, fit.p, fit.q)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        d = (mact.mact_lab(x + e, fit.p, fit.q, gamma="none") - mact.mact_lab(x - e, fit.p, fit.q, gamma="none")) / (2 * h)
        ok = _guard(x)
        np.testing.assert_allclose(J[ok, :, k], d[ok], rtol=1e-5, atol=1e-4)


def test_linear_segment_slope_and_clamp(fit):
    t = np.array([0.001, 0.008856])
    np.testing.assert_array_equal(grad.mact_f_prime(t, fit.p, fit.q), [7.787, 7.787])
    x = np.array([[-0.2, 0.5, 1.3]])
    J = grad.jacobian(x, fit.p, fit.q)
    assert np.all(J[0, :, 0] == 0) and np.all(J[0, :, 2] == 0) and np.any(J[0, :, 1] != 0)


def test_vjp_is_transpose_product(fit):
    g = synth.rng(13)
    x = g.random((50, 3))
    gv = g.normal(size=(50, 3))
    J = grad.jacobian(x, fit.p, fit.q)
    np.testing.assert_allclose(grad.vjp(x, gv, fit.p, fit.q), np.einsum("ni,nik->nk", gv, J), rtol=1e-14)
