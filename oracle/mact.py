"""FP64 evaluation of the MACT transforms (oracle; test infrastructure only).

These are the transforms of Sec. 3.2-3.4 with the costly elementary functions
replaced by the minimax approximations whose coefficients are passed in.  The
steps are the paper's, in its order; the arithmetic is float64 throughout, so
a GPU evaluating the same approximation in float32 differs from these values
by float32 rounding only (the caller rounds the coefficients to float32 and
passes them here promoted to float64 when it wants exactly the GPU's
approximation).

Inputs are (..., 3) arrays of R, G, B on the normalised scale [0, 1]; float
inputs outside [0, 1] are clamped to it first (the approximations are fitted
on the image of [0, 1] only).
"""
import numpy as np

from . import colour


def horner(c, x):
    """Polynomial sum_k c[k] x^k by Horner's rule, float64."""
    x = np.asarray(x, dtype=np.float64)
    c = [float(v) for v in c]
    acc = np.full_like(x, c[-1])
    for a in reversed(c[:-1]):
        acc = acc * x + a
    return acc


def clamp01(rgb):
    return np.clip(np.asarray(rgb, dtype=np.float64), 0.0, 1.0)


def mact_lab_f(t, p, q, hi=None):
    """The approximated CIELAB nonlinearity: p(t)/q(t) above 0.008856 (the
    minimax rational standing in for the cube root, Sec. 3.2.2), the exact
    linear segment at or below it.  ``hi`` (a boolean mask like t), when
    given, chooses the branch instead of the comparison: a test uses it to
    evaluate a value within rounding of the threshold on either side."""
    t = np.asarray(t, dtype=np.float64)
    hi = t > colour.LAB_T0 if hi is None else np.asarray(hi, dtype=bool)
    ts = np.where(hi, t, 0.5)  # keep q away from any root on the unused branch
    return np.where(hi, horner(p, ts) / horner(q, ts), colour.LAB_K * t + colour.LAB_C)


def mact_decode709(k, c_dec, hi=None):
    """BT.709 decoding with ((k + 0.099)/1.099)^(1/0.45) replaced by the
    polynomial ``c_dec`` (fitted on [0.081, 1]): k/4.5 below 0.081.  ``hi``
    (a boolean mask like k), when given, chooses the polynomial branch in
    place of the comparison k >= 0.081."""
    k = np.asarray(k, dtype=np.float64)
    lo = k < 0.081 if hi is None else ~np.asarray(hi, dtype=bool)
    return np.where(lo, k / 4.5, horner(c_dec, k))


def mact_lab(rgb, p, q, gamma="bt709", debug=False, decode=None, decode_hi=None, f_hi=None):
    """RGB -> CIELAB with the cube root replaced by p/q (Sec. 3.2).

    Steps: inverse gamma (BT.709 by default), RGB -> XYZ, divide by the D65
    white, approximated f, then L*, a*, b*.  With ``debug`` the three values
    f~(X/X0), f~(Y/Y0), f~(Z/Z0) are returned instead of L*a*b*.  With
    ``decode`` (polynomial coefficients) and gamma 'bt709' the decoding power
    is replaced as well.  ``decode_hi`` and ``f_hi`` (boolean masks like rgb)
    force the branch of the decoding (per input channel) and of f (per X, Y,
    Z) instead of the comparisons with 0.081 and 0.008856.
    """
    if decode is not None and gamma == "bt709":
        lin = mact_decode709(clamp01(rgb), decode, decode_hi)
        t = colour.rgb_to_xyz(lin) / colour.WHITE_D65
    else:
        t = colour.lab_t(clamp01(rgb), gamma)
    f = mact_lab_f(t, p, q, f_hi)
    if debug:
        return f
    fx, fy, fz = f[..., 0], f[..., 1], f[..., 2]
    return np.stack([116.0 * fy - 16.0, 500.0 * (fx - fy), 200.0 * (fy - fz)], axis=-1)


def mact_luv(rgb, p, q, gamma="bt709", decode=None, decode_hi=None, f_hi=None):
    """RGB -> CIE 1976 L*u*v* with the cube root of L* replaced by p/q (the
    CIELAB nonlinearity, Sec. 3.2.2); u', v' by their exact divisions.
    ``decode_hi`` (a mask like rgb) and ``f_hi`` (a mask over pixels, for
    Y / Yn) force branches as in ``mact_lab``."""
    if decode is not None and gamma == "bt709":
        lin = mact_decode709(clamp01(rgb), decode, decode_hi)
    else:
        lin = colour.inverse_gamma(clamp01(rgb), gamma)
    xyz = colour.rgb_to_xyz(lin)
    X, Y, Z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    Xn, Yn, Zn = colour.WHITE_D65
    dn = Xn + 15.0 * Yn + 3.0 * Zn
    un, vn = 4.0 * Xn / dn, 9.0 * Yn / dn
    d = X + 15.0 * Y + 3.0 * Z
    pos = d > 0
    ds = np.where(pos, d, 1.0)
    L = 116.0 * mact_lab_f(Y / Yn, p, q, f_hi) - 16.0
    u = np.where(pos, 13.0 * L * (4.0 * X / ds - un), 0.0)
    v = np.where(pos, 13.0 * L * (9.0 * Y / ds - vn), 0.0)
    return np.stack([L, u, v], axis=-1)


def odd_poly(c, x):
    """P approximates an odd function on [0, 1]; negative arguments use
    arctan(-x) = -arctan(x) (Sec. 3.3.2): -P(-x) for x < 0, P(x) otherwise."""
    x = np.asarray(x, dtype=np.float64)
    v = horner(c, np.abs(x))
    return np.where(x < 0, -v, v)


def mact_hsi(rgb, c_atan):
    """RGB -> HSI by Kender's form with arctan(sqrt(3) x) replaced by the
    polynomial ``c_atan`` (Sec. 3.3.2).  H in [0, 2pi]; H = 0 on the red ray
    and on the gray axis; S = 0 for black."""
    rgb = clamp01(rgb)
    _, case, x = colour.kender_hue(rgb)
    base = np.where(case == 1, np.pi / 3.0, np.where(case == 2, np.pi, 5.0 * np.pi / 3.0))
    active = (case >= 1) & (case <= 3)
    H = np.where(active, base + odd_poly(c_atan, x), 0.0)
    hsi = colour.rgb_to_hsi(rgb)
    return np.stack([H, hsi[..., 1], hsi[..., 2]], axis=-1)


def mact_sct(rgb, c_asin2, c_acos, c_atan, c_atanc, upper=None, g_lt_r=None):
    """RGB -> SCT with the inverse trigonometric functions replaced by
    polynomials (Sec. 3.4.2, 3.4.3).

    angle A: for B/L >= 0.5 (tested as 3 B^2 >= R^2 + G^2) it is
    2 arcsin(y / sqrt 2) with y = sqrt(1 - B/L) ("c_asin2"); below 0.5 it is
    arccos(B/L) ("c_acos").  1 - B/L is formed as (R^2+G^2) / (L (L + B)),
    the same quantity without the cancellation.
    angle B: arctan(G/R) split at G = R: for G < R the polynomial f of G/R
    ("c_atan"); for 0 < R <= G the polynomial of g, pi/2 - arctan(R/G)
    ("c_atanc"); pi/2 for R = 0 < G; 0 for R = G = 0.
    L = 0 gives (0, 0, 0).
    ``upper`` and ``g_lt_r`` (boolean masks over pixels), when given, choose
    the branch of angle A (the arcsin form) and of angle B (f of G/R) instead
    of the comparisons, for evaluating a pixel within rounding of a branch
    plane on either side; g_lt_r applies where R and G are both positive.
    """
    rgb = clamp01(rgb)
    R, G, B = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    rg2 = R * R + G * G
    L = np.sqrt(rg2 + B * B)
    pos = L > 0
    Ls = np.where(pos, L, 1.0)
    upper = 3.0 * B * B >= rg2 if upper is None else np.asarray(upper, dtype=bool)
    y = np.sqrt(rg2 / (Ls * (Ls + B)))
    A = np.where(upper, horner(c_asin2, y), horner(c_acos, B / Ls))
    A = np.where(pos, A, 0.0)
    r_pos = R > 0
    g_pos = G > 0
    gr = G < R if g_lt_r is None else np.where(r_pos & g_pos, np.asarray(g_lt_r, dtype=bool), G < R)
    Bf = horner(c_atan, G / np.where(r_pos, R, 1.0))
    Bg = horner(c_atanc, R / np.where(g_pos, G, 1.0))
    Bang = np.where(gr, Bf, np.where(r_pos, Bg, np.where(g_pos, 0.5 * np.pi, 0.0)))
    return np.stack([L, A, Bang], axis=-1)


# ---------------------------------------------------------------- inverses
#
# The inverse transforms with their elementary functions replaced by minimax
# approximations in the same way: the BT.709 encoding power by a rational on
# [0.018, 1], sine and cosine by polynomials on [0, pi/2] (SCT) and cosine on
# [0, 2pi/3] (HSI).  The cube of the CIELAB inverse is exact.


def mact_encode709(lin, p, q):
    """BT.709 encoding with 1.099 L^0.45 - 0.099 replaced by p/q: 4.5 L below
    0.018, p(L)/q(L) at or above, L clamped to [0, 1] first (the rational is
    fitted on [0.018, 1] only)."""
    x = clamp01(lin)
    hi = x >= 0.018
    xs = np.where(hi, x, 0.5)
    return np.where(hi, horner(p, xs) / horner(q, xs), 4.5 * x)


def mact_lab_inverse(lab, p_enc, q_enc, gamma="bt709"):
    """L*a*b* -> R'G'B': f from L*, a*, b*, t by the exact cube (or the linear
    segment), linear RGB = M^-1 (t * white) clamped to [0, 1], then the
    approximated encoding (gamma 'bt709') or none ('none')."""
    lab = np.asarray(lab, dtype=np.float64)
    fy = (lab[..., 0] + 16.0) / 116.0
    f = np.stack([fy + lab[..., 1] / 500.0, fy, fy - lab[..., 2] / 200.0], axis=-1)
    lin = clamp01((colour.lab_f_inv(f) * colour.WHITE_D65) @ colour.M_XYZ_RGB.T)
    if gamma == "bt709":
        return mact_encode709(lin, p_enc, q_enc)
    if gamma == "none":
        return lin
    raise ValueError(gamma)


def mact_luv_inverse(luv, p_enc, q_enc, gamma="bt709"):
    """L*u*v* -> R'G'B': XYZ by the definition (colour.luv_to_xyz: the exact
    cube or linear segment for Y, then u', v' and the two quotients), linear
    RGB = M^-1 XYZ clamped to [0, 1], then the approximated encoding, as in
    ``mact_lab_inverse``."""
    lin = clamp01(colour.luv_to_xyz(luv) @ colour.M_XYZ_RGB.T)
    if gamma == "bt709":
        return mact_encode709(lin, p_enc, q_enc)
    if gamma == "none":
        return lin
    raise ValueError(gamma)


def mact_hsi_inverse(hsi, c_cos):
    """HSI -> RGB by sectors (as colour.hsi_to_rgb) with cos replaced by the
    polynomial ``c_cos`` on [0, 2pi/3], evaluated at |argument|.  H is taken
    modulo 2pi."""
    hsi = np.asarray(hsi, dtype=np.float64)
    H = np.mod(hsi[..., 0], 2.0 * np.pi)
    S, I = hsi[..., 1], hsi[..., 2]
    sector = np.minimum((H // (2.0 * np.pi / 3.0)).astype(int), 2)
    h = H - sector * (2.0 * np.pi / 3.0)
    behind = I * (1.0 - S)
    start = I * (1.0 + S * horner(c_cos, h) / horner(c_cos, np.abs(np.pi / 3.0 - h)))
    third = 3.0 * I - (behind + start)
    R = np.where(sector == 0, start, np.where(sector == 1, behind, third))
    G = np.where(sector == 0, third, np.where(sector == 1, start, behind))
    B = np.where(sector == 0, behind, np.where(sector == 1, third, start))
    return np.stack([R, G, B], axis=-1)


def mact_sct_inverse(sct, c_sin, c_cos):
    """SCT -> RGB (the inverse of Sec. 3.4.1: R = L sin A cos B, G = L sin A
    sin B, B = L cos A) with sin and cos replaced by polynomials on
    [0, pi/2], the range of both angles for non-negative RGB."""
    sct = np.asarray(sct, dtype=np.float64)
    L, A, Bang = sct[..., 0], sct[..., 1], sct[..., 2]
    sa = horner(c_sin, A)
    return np.stack([L * sa * horner(c_cos, Bang), L * sa * horner(c_sin, Bang), L * horner(c_cos, A)], axis=-1)
