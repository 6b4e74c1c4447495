"""Exact colour-space transforms and error metrics, FP64 (oracle; test
infrastructure only).

Every function takes arrays whose last axis holds the three channels.  RGB
values are on the normalised scale [0, 1] (an 8-bit value v enters as v/255).
The formulas are the paper's definitions written out, and their inverses
(the definitions solved for R, G, B), nothing else.
"""
import numpy as np

# ITU-R BT.709 primaries, linear RGB -> CIEXYZ (Sec. 3.2.1, RGB->XYZ equation).
M_RGB_XYZ = np.array([[0.412391, 0.357584, 0.180481],
                      [0.212639, 0.715169, 0.072192],
                      [0.019331, 0.119195, 0.950532]], dtype=np.float64)

# D65 reference white (Sec. 3.2.1, reference-white equation).
WHITE_D65 = np.array([0.950456, 1.0, 1.089058], dtype=np.float64)

# CIELAB breakpoint and linear segment, as printed (XYZ->CIELAB equation).
LAB_T0 = 0.008856
LAB_K = 7.787
LAB_C = 16.0 / 116.0


def inverse_gamma(k, kind="bt709"):
    """Nonlinear R'G'B' in [0,1] -> linear RGB.

    ``bt709``: the inverse gamma of Sec. 3.2.1 (ITU-R BT.709): k/4.5 below
    0.081, else ((k+0.099)/1.099)^(1/0.45).  Values below 0.081, negative ones
    included, take the linear branch.
    ``srgb``: the IEC 61966-2-1 curve (an option; the paper uses BT.709).
    ``none``: the input is already linear.
    """
    k = np.asarray(k, dtype=np.float64)
    if kind == "bt709":
        hi = np.maximum(k, 0.081)  # keep the power's base positive on the unused branch
        return np.where(k < 0.081, k / 4.5, ((hi + 0.099) / 1.099) ** (1.0 / 0.45))
    if kind == "srgb":
        hi = np.maximum(k, 0.04045)
        return np.where(k <= 0.04045, k / 12.92, ((hi + 0.055) / 1.055) ** 2.4)
    if kind == "none":
        return k
    raise ValueError(kind)


def rgb_to_xyz(lin):
    """Linear RGB -> CIEXYZ with the BT.709 matrix (Sec. 3.2.1)."""
    lin = np.asarray(lin, dtype=np.float64)
    return lin @ M_RGB_XYZ.T


def lab_f(t):
    """The CIELAB nonlinearity f(t): cube root above 0.008856, the linear
    segment 7.787 t + 16/116 at or below it (XYZ->CIELAB equation)."""
    t = np.asarray(t, dtype=np.float64)
    return np.where(t > LAB_T0, np.cbrt(t), LAB_K * t + LAB_C)


def xyz_to_lab(xyz):
    """CIEXYZ -> CIELAB relative to D65 (XYZ->CIELAB equation)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    f = lab_f(xyz / WHITE_D65)
    fx, fy, fz = f[..., 0], f[..., 1], f[..., 2]
    return np.stack([116.0 * fy - 16.0, 500.0 * (fx - fy), 200.0 * (fy - fz)], axis=-1)


def rgb_to_lab(rgb, gamma="bt709"):
    """R'G'B' (or linear RGB with gamma='none') in [0,1] -> L*a*b*: the three
    steps of Sec. 3.2.1 in order."""
    return xyz_to_lab(rgb_to_xyz(inverse_gamma(rgb, gamma)))


def lab_t(rgb, gamma="bt709"):
    """The arguments X/X0, Y/Y0, Z/Z0 of f (used for the call probabilities of
    Sec. 3.2.2)."""
    return rgb_to_xyz(inverse_gamma(rgb, gamma)) / WHITE_D65


def xyz_to_luv(xyz):
    """CIEXYZ -> CIE 1976 L*u*v* relative to D65, with the paper's L* (the
    same f as CIELAB, so L* is CIELAB's L*): u' = 4X / (X + 15Y + 3Z),
    v' = 9Y / (X + 15Y + 3Z), u* = 13 L* (u' - u'n), v* = 13 L* (v' - v'n)
    with u'n, v'n those of the white.  Where X + 15Y + 3Z = 0 (black)
    u* = v* = 0.  (CIELUV is the extension the paper names in Sec. 4.)"""
    xyz = np.asarray(xyz, dtype=np.float64)
    X, Y, Z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    Xn, Yn, Zn = WHITE_D65
    dn = Xn + 15.0 * Yn + 3.0 * Zn
    un, vn = 4.0 * Xn / dn, 9.0 * Yn / dn
    d = X + 15.0 * Y + 3.0 * Z
    pos = d > 0
    ds = np.where(pos, d, 1.0)
    L = 116.0 * lab_f(Y / Yn) - 16.0
    u = np.where(pos, 13.0 * L * (4.0 * X / ds - un), 0.0)
    v = np.where(pos, 13.0 * L * (9.0 * Y / ds - vn), 0.0)
    return np.stack([L, u, v], axis=-1)


def rgb_to_luv(rgb, gamma="bt709"):
    """R'G'B' (or linear RGB with gamma='none') in [0,1] -> L*u*v*."""
    return xyz_to_luv(rgb_to_xyz(inverse_gamma(rgb, gamma)))


def rgb_to_hsi(rgb):
    """RGB -> HSI by the arccos definition (Sec. 3.3.1).

    H in [0, 2pi) radians, S and I in [0, 1].  Hue is undefined on the gray
    axis; it is returned as 0 there.  Black has S = 0.
    """
    rgb = np.asarray(rgb, dtype=np.float64)
    R, G, B = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    num = 0.5 * ((R - G) + (R - B))
    den = np.sqrt((R - G) ** 2 + (R - B) * (G - B))
    gray = den == 0
    c = np.clip(num / np.where(gray, 1.0, den), -1.0, 1.0)
    H = np.arccos(c)
    H = np.where(B > G, 2.0 * np.pi - H, H)
    H = np.where(gray, 0.0, H)
    s = R + G + B
    S = np.where(s > 0, 1.0 - 3.0 * np.minimum(np.minimum(R, G), B) / np.where(s > 0, s, 1.0), 0.0)
    I = s / 3.0
    return np.stack([H, S, I], axis=-1)


def kender_hue(rgb):
    """Hue by Kender's branch form (Sec. 3.3.1), with the exact arctan.

    Returns (H, case, x): case 1..3 selects the base angle pi/3, pi, 5pi/3 and
    x is the arctan argument before the factor sqrt(3); case 4 is the red ray
    (H = 0) and case 0 the gray axis (undefined, H = 0).
    """
    rgb = np.asarray(rgb, dtype=np.float64)
    R, G, B = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    c1 = (R > B) & (G > B)
    c2 = ~c1 & (G > R)
    c3 = ~c1 & ~c2 & (B > G)
    c4 = ~c1 & ~c2 & ~c3 & (R > B)
    num = np.where(c1, G - R, np.where(c2, B - G, R - B))
    den = np.where(c1, (G - B) + (R - B), np.where(c2, (B - R) + (G - R), (R - G) + (B - G)))
    active = c1 | c2 | c3
    x = np.where(active, num / np.where(active, den, 1.0), 0.0)
    base = np.where(c1, np.pi / 3.0, np.where(c2, np.pi, 5.0 * np.pi / 3.0))
    H = np.where(active, base + np.arctan(np.sqrt(3.0) * x), 0.0)
    case = np.where(c1, 1, np.where(c2, 2, np.where(c3, 3, np.where(c4, 4, 0))))
    return H, case, x


def rgb_to_hsi_kender(rgb):
    """RGB -> HSI with Kender's hue; S and I as in the definition."""
    rgb = np.asarray(rgb, dtype=np.float64)
    H, _, _ = kender_hue(rgb)
    hsi = rgb_to_hsi(rgb)
    return np.stack([H, hsi[..., 1], hsi[..., 2]], axis=-1)


def rgb_to_sct(rgb):
    """RGB -> SCT (Sec. 3.4.1): L = |RGB|, angle A = arccos(B/L), angle B =
    arctan(G/R) (the simplified form).  Degenerate cases: L = 0 gives A = B = 0;
    R = G = 0 gives B = 0; R = 0 < G gives B = pi/2."""
    rgb = np.asarray(rgb, dtype=np.float64)
    R, G, B = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    L = np.sqrt(R * R + G * G + B * B)
    pos = L > 0
    A = np.where(pos, np.arccos(np.clip(B / np.where(pos, L, 1.0), -1.0, 1.0)), 0.0)
    Bang = np.arctan2(G, R)
    return np.stack([L, A, Bang], axis=-1)


def rgb_to_sct_arccos(rgb):
    """SCT with angle B by its original arccos form R/(L sin A) (Sec. 3.4.1);
    defined where L sin A > 0."""
    rgb = np.asarray(rgb, dtype=np.float64)
    R, G, B = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    L = np.sqrt(R * R + G * G + B * B)
    A = np.arccos(np.clip(B / L, -1.0, 1.0))
    Bang = np.arccos(np.clip(R / (L * np.sin(A)), -1.0, 1.0))
    return np.stack([L, A, Bang], axis=-1)


def sct_to_rgb(sct):
    """SCT -> RGB, the inverse of Sec. 3.4.1.  No clipping."""
    sct = np.asarray(sct, dtype=np.float64)
    L, A, Bang = sct[..., 0], sct[..., 1], sct[..., 2]
    return np.stack([L * np.sin(A) * np.cos(Bang), L * np.sin(A) * np.sin(Bang), L * np.cos(A)], axis=-1)


# CIEXYZ -> linear RGB: the inverse of the BT.709 matrix above.
M_XYZ_RGB = np.linalg.inv(M_RGB_XYZ)


def encode_gamma(lin, kind="bt709"):
    """Linear RGB -> nonlinear R'G'B': the inverse of ``inverse_gamma``.

    ``bt709``: 4.5 L below 0.018 (= 0.081 / 4.5, the decoding breakpoint),
    else 1.099 L^0.45 - 0.099; negative values take the linear branch.
    ``srgb``: 12.92 L up to 0.0031308, else 1.055 L^(1/2.4) - 0.055.
    ``none``: unchanged.
    """
    lin = np.asarray(lin, dtype=np.float64)
    if kind == "bt709":
        hi = np.maximum(lin, 0.018)
        return np.where(lin < 0.018, 4.5 * lin, 1.099 * hi ** 0.45 - 0.099)
    if kind == "srgb":
        hi = np.maximum(lin, 0.0031308)
        return np.where(lin <= 0.0031308, 12.92 * lin, 1.055 * hi ** (1.0 / 2.4) - 0.055)
    if kind == "none":
        return lin
    raise ValueError(kind)


def lab_f_inv(f):
    """The inverse of the CIELAB nonlinearity: f^3 where that exceeds the
    breakpoint 0.008856, else (f - 16/116) / 7.787.  (With the printed
    constants f jumps at the breakpoint from 0.2068927 to cbrt(0.008856) =
    0.2068930, so the two branches never overlap; f in the gap, which the
    forward transform never produces, takes the linear branch.)"""
    f = np.asarray(f, dtype=np.float64)
    t = f * f * f
    return np.where(t > LAB_T0, t, (f - LAB_C) / LAB_K)


def lab_to_rgb(lab, gamma="bt709"):
    """L*a*b* -> R'G'B' (or linear RGB with gamma='none'): the steps of
    Sec. 3.2.1 inverted in reverse order.  No clipping."""
    lab = np.asarray(lab, dtype=np.float64)
    fy = (lab[..., 0] + 16.0) / 116.0
    f = np.stack([fy + lab[..., 1] / 500.0, fy, fy - lab[..., 2] / 200.0], axis=-1)
    xyz = lab_f_inv(f) * WHITE_D65
    return encode_gamma(xyz @ M_XYZ_RGB.T, gamma)


def luv_to_xyz(luv):
    """CIE 1976 L*u*v* -> CIEXYZ (relative to D65), the definition solved for
    X, Y, Z: Y from L* as in CIELAB (``lab_f_inv`` of (L* + 16) / 116),
    u' = u* / (13 L*) + u'n, v' = v* / (13 L*) + v'n, and from u' = 4X / D,
    v' = 9Y / D: X = Y 9u' / (4v'), Z = Y (12 - 3u' - 20v') / (4v').  L* = 0
    (black, the only colour with Y = 0) gives X = Y = Z = 0."""
    luv = np.asarray(luv, dtype=np.float64)
    L, u, v = luv[..., 0], luv[..., 1], luv[..., 2]
    Xn, Yn, Zn = WHITE_D65
    dn = Xn + 15.0 * Yn + 3.0 * Zn
    un, vn = 4.0 * Xn / dn, 9.0 * Yn / dn
    pos = L > 0
    Ls = np.where(pos, L, 1.0)
    Y = np.where(pos, Yn * lab_f_inv((L + 16.0) / 116.0), 0.0)
    up = u / (13.0 * Ls) + un
    vp = v / (13.0 * Ls) + vn
    vs = np.where(pos, vp, 1.0)
    X = np.where(pos, Y * 9.0 * up / (4.0 * vs), 0.0)
    Z = np.where(pos, Y * (12.0 - 3.0 * up - 20.0 * vp) / (4.0 * vs), 0.0)
    return np.stack([X, Y, Z], axis=-1)


def luv_to_rgb(luv, gamma="bt709"):
    """L*u*v* -> R'G'B' (or linear RGB with gamma='none'): XYZ, the inverse
    matrix, then the encoding.  No clipping."""
    return encode_gamma(luv_to_xyz(luv) @ M_XYZ_RGB.T, gamma)


def hsi_to_rgb(hsi):
    """HSI -> RGB, the inverse of the arccos definition (Sec. 3.3.1), by
    sectors of 2pi/3: in the sector starting at hue h0 with h = H - h0, the
    channel 'behind' the sector is I (1 - S), the channel at its start is
    I (1 + S cos h / cos(pi/3 - h)), and the third makes the sum 3 I.
    Sectors: [0, 2pi/3) B, R, G; [2pi/3, 4pi/3) R, G, B; [4pi/3, 2pi) G, B, R
    (behind, start, third)."""
    hsi = np.asarray(hsi, dtype=np.float64)
    H = np.mod(hsi[..., 0], 2.0 * np.pi)
    S, I = hsi[..., 1], hsi[..., 2]
    sector = np.minimum((H // (2.0 * np.pi / 3.0)).astype(int), 2)
    h = H - sector * (2.0 * np.pi / 3.0)
    behind = I * (1.0 - S)
    start = I * (1.0 + S * np.cos(h) / np.cos(np.pi / 3.0 - h))
    third = 3.0 * I - (behind + start)
    R = np.where(sector == 0, start, np.where(sector == 1, behind, third))
    G = np.where(sector == 0, third, np.where(sector == 1, start, behind))
    B = np.where(sector == 0, behind, np.where(sector == 1, third, start))
    return np.stack([R, G, B], axis=-1)


def delta_e(lab1, lab2):
    """CIELAB distance Delta E*ab (Sec. 3.2.1): the Euclidean norm."""
    d = np.asarray(lab1, dtype=np.float64) - np.asarray(lab2, dtype=np.float64)
    return np.sqrt(np.sum(d * d, axis=-1))


def d_hsi(hsi1, hsi2):
    """HSI distance (Sec. 3.3.1) with the hue difference wrapped to [0, pi]."""
    a = np.asarray(hsi1, dtype=np.float64)
    b = np.asarray(hsi2, dtype=np.float64)
    dh = np.abs(a[..., 0] - b[..., 0])
    th = np.where(dh <= np.pi, dh, 2.0 * np.pi - dh)
    sx, sy = a[..., 1], b[..., 1]
    v = sx * sx + sy * sy - 2.0 * sx * sy * np.cos(th) + (a[..., 2] - b[..., 2]) ** 2
    return np.sqrt(np.maximum(v, 0.0))


def sct_delta_e(sct1, sct2, gamma="bt709"):
    """The SCT error measure of Sec. 3.4.1: invert both SCT triples to RGB,
    convert each to CIELAB, take Delta E*ab.  The inverse is not clipped."""
    return delta_e(rgb_to_lab(sct_to_rgb(sct1), gamma), rgb_to_lab(sct_to_rgb(sct2), gamma))


def angle_diff(a, b, period=2.0 * np.pi):
    """|a - b| wrapped to [0, period/2]."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) % period
    return np.minimum(d, period - d)
