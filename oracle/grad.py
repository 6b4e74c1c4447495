"""Gradients of the minimax RGB->CIELAB transform, FP64 (oracle; test
infrastructure only).

The transform (Sec. 3.2 with the cube root replaced by p/q) on linear RGB
input x in [0, 1]^3 (inputs outside are clamped first) is
    t = diag(1/white) M x,   f = f~(t) per channel,
    (L*, a*, b*) = J f + (-16, 0, 0),
    J = [[0, 116, 0], [500, -500, 0], [0, 200, -200]].
Its Jacobian is J diag(f~'(t)) diag(1/white) M, times the clamp's derivative
(1 inside [0, 1], 0 outside), with f~' = (p' q - p q') / q^2 above 0.008856
and 7.787 at or below it.  The paper does not differentiate the transform;
this is the chain rule applied to its definition.
"""
import numpy as np
from numpy.polynomial import polynomial as Pm

from . import colour, mact

J_LAB = np.array([[0.0, 116.0, 0.0], [500.0, -500.0, 0.0], [0.0, 200.0, -200.0]])


def mact_f_prime(t, p, q):
    t = np.asarray(t, dtype=np.float64)
    hi = t > colour.LAB_T0
    ts = np.where(hi, t, 0.5)
    pv, qv = Pm.polyval(ts, p), Pm.polyval(ts, q)
    dp, dq = Pm.polyval(ts, Pm.polyder(p)), Pm.polyval(ts, Pm.polyder(q))
    return np.where(hi, (dp * qv - pv * dq) / (qv * qv), colour.LAB_K)


def jacobian(x, p, q):
    """d(L*, a*, b*)/dx, shape (..., 3, 3), for linear RGB x (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    xc = np.clip(x, 0.0, 1.0)
    Mw = colour.M_RGB_XYZ / colour.WHITE_D65[:, None]
    t = xc @ Mw.T
    d = mact_f_prime(t, p, q)
    inside = ((x >= 0.0) & (x <= 1.0)).astype(np.float64)
    # J diag(d) Mw diag(inside)
    return np.einsum("ij,...j,jk,...k->...ik", J_LAB, d, Mw, inside)


def vjp(x, g, p, q):
    """Vector-Jacobian product g^T d(Lab)/dx, shape (..., 3)."""
    return np.einsum("...i,...ik->...k", np.asarray(g, dtype=np.float64), jacobian(x, p, q))


def delta_e_loss_grad_pixel(x, target, p, q):
    """Gradient of the per-pixel term ||Lab(x) - target|| with respect to x."""
    lab = mact.mact_lab(x, p, q, gamma="none")
    d = lab - target
    n = np.sqrt(np.sum(d * d, axis=-1, keepdims=True))
    g = d / np.where(n > 0, n, 1.0)
    return vjp(x, g, p, q)


def fd_loss_grad_pixel(x, target, p, q, h=1e-3):
    """Central finite differences of the per-pixel term ||Lab(x) - target||."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fp = colour.delta_e(mact.mact_lab(x + e, p, q, gamma="none"), target)
        fm = colour.delta_e(mact.mact_lab(x - e, p, q, gamma="none"), target)
        out[..., k] = (fp - fm) / (2.0 * h)
    return out
