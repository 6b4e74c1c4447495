"""3-D LUT packing and interpolation, FP64 (oracle; test infrastructure only).

Sec. 3.5.3 describes three steps -- packing, extraction, interpolation --
and four interpolators (trilinear with 8 lattice points, prism with 6,
pyramidal with 5, tetrahedral with 4), deferring their formulas to the
literature.  Readings used here:

  * packing: an N x N x N grid whose node (i, j, k) holds the exact transform
    of the normalised input (i, j, k)/(N - 1) (8-bit value i 255/(N-1)),
    endpoints included;
  * extraction: pos = x (N - 1), cell i = min(floor(pos), N - 2), fraction
    f = pos - i, per channel;
  * every method is a weighted sum of cell corners, sum_k w_k c_k, with
    weights that sum to one:
      trilinear    the tensor product of (1 - f, f) on the three axes;
      tetrahedral  the fractions sorted in decreasing order f1 >= f2 >= f3,
                   walking from corner 000 along the axes in that order:
                   weights 1 - f1, f1 - f2, f2 - f3, f3;
      prism        linear along R; in the (G, B) face the triangle is chosen by
                   f_G >= f_B: corners (0,0), (1,0), (1,1) with weights
                   1 - f_G, f_G - f_B, f_B, else (0,0), (0,1), (1,1) with
                   weights 1 - f_B, f_B - f_G, f_G;
      pyramidal    apex corner 111, base the cell face through 000 normal to
                   the axis of the smallest fraction; value
                   c000 + (c111 - c011) f_R + (c010 - c000) f_G
                   + (c001 - c000) f_B + (c011 - c001 - c010 + c000) f_G f_B
                   for f_R smallest, and the same under axis permutation.
                   PARITY UNPINNED: no variant reproduces the paper's Table 12
                   pyramidal row; held to invariants and to this reading's
                   special cases (bilinear on the base face, linear on the
                   edge from the base's far corner to the apex).
  * angular channels (H of HSI; angles A and B of SCT) are interpolated as
    circular data (Sec. 3.5.3): the weighted sum of unit vectors
    (cos theta_k, sin theta_k) with the method's own weights, then the angle
    of the resultant.  PARITY UNPINNED against the paper (its grid is not
    stated); held to invariants and, on cell edges, to the closed-form
    resultant of two weighted unit vectors.
"""
import numpy as np

from . import colour

# Which output channels are angles, per transform.
ANGULAR = {"lab": (False, False, False), "hsi": (True, False, False), "sct": (False, True, True),
           "luv": (False, False, False)}


def node_inputs(N):
    return np.arange(N, dtype=np.float64) / (N - 1)


def build(xform, N, gamma="bt709"):
    """The packed LUT: (N, N, N, 3) exact FP64 outputs at the node inputs,
    indexed [i_R, i_G, i_B]."""
    v = node_inputs(N)
    grid = np.stack(np.meshgrid(v, v, v, indexing="ij"), axis=-1)
    if xform == "lab":
        return colour.rgb_to_lab(grid, gamma)
    if xform == "hsi":
        return colour.rgb_to_hsi(grid)
    if xform == "sct":
        return colour.rgb_to_sct(grid)
    if xform == "luv":
        return colour.rgb_to_luv(grid, gamma)
    raise ValueError(xform)


def locate(x, N):
    """Cell index and fraction per channel for inputs x in [0, 1]."""
    pos = np.clip(np.asarray(x, dtype=np.float64), 0.0, 1.0) * (N - 1)
    i = np.minimum(np.floor(pos).astype(np.int64), N - 2)
    return i, pos - i


def locate_u8(v, N):
    """Extraction for 8-bit inputs: pos = v (N - 1) / 255 in exact integer
    arithmetic for the cell, the fraction from the remainder."""
    v = np.asarray(v, dtype=np.int64)
    num = v * (N - 1)
    i = np.minimum(num // 255, N - 2)
    f = (num - 255 * i) / 255.0
    return i, f


def corner_weights(method, f):
    """List of (corner offset (dr, dg, db), weight array) for fractions f (..., 3)."""
    fr, fg, fb = f[..., 0], f[..., 1], f[..., 2]
    one = np.ones_like(fr)
    if method == "trilinear":
        out = []
        for dr in (0, 1):
            for dg in (0, 1):
                for db in (0, 1):
                    w = (fr if dr else 1 - fr) * (fg if dg else 1 - fg) * (fb if db else 1 - fb)
                    out.append(((dr, dg, db), w))
        return out
    if method == "tetrahedral":
        # decreasing order of the fractions; the path 000 -> ... -> 111 along the axes
        order = np.argsort(-f, axis=-1, kind="stable")
        fs = np.take_along_axis(f, order, axis=-1)
        # express as weights on all 8 corners: corner reached after k steps
        corners = {}
        steps = [np.zeros(f.shape[:-1] + (3,), dtype=np.int64)]
        cur = steps[0].copy()
        for k in range(3):
            cur = cur.copy()
            np.put_along_axis(cur, order[..., k:k + 1], 1, axis=-1)
            steps.append(cur)
        ws = [1 - fs[..., 0], fs[..., 0] - fs[..., 1], fs[..., 1] - fs[..., 2], fs[..., 2]]
        for dr in (0, 1):
            for dg in (0, 1):
                for db in (0, 1):
                    w = np.zeros_like(fr)
                    for st, wk in zip(steps, ws):
                        hit = (st[..., 0] == dr) & (st[..., 1] == dg) & (st[..., 2] == db)
                        w = w + np.where(hit, wk, 0.0)
                    corners[(dr, dg, db)] = w
        return list(corners.items())
    if method == "prism":
        up = fg >= fb
        tri = [((0, 0), np.where(up, 1 - fg, 1 - fb)),
               ((1, 0), np.where(up, fg - fb, 0.0)),
               ((0, 1), np.where(up, 0.0, fb - fg)),
               ((1, 1), np.where(up, fb, fg))]
        out = []
        for dr in (0, 1):
            for (dg, db), w in tri:
                out.append(((dr, dg, db), (fr if dr else 1 - fr) * w))
        return out
    if method == "pyramidal":
        # axis of the smallest fraction (first on ties, R before G before B)
        kmin = np.argmin(f, axis=-1)
        w = {c: np.zeros_like(fr) for c in [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]}
        for k in range(3):
            sel = kmin == k
            # local axes: s = the smallest axis, u, v = the other two in R, G, B order
            others = [j for j in range(3) if j != k]
            fs_, fu, fv = f[..., k], f[..., others[0]], f[..., others[1]]

            def corner(ds, du, dv):
                c = [0, 0, 0]
                c[k], c[others[0]], c[others[1]] = ds, du, dv
                return tuple(c)
            # c000 + (c111 - c011) fs + (c010 - c000) fu + (c001 - c000) fv + (c011 - c001 - c010 + c000) fu fv
            contrib = {
                corner(0, 0, 0): 1 - fu - fv + fu * fv,
                corner(1, 1, 1): fs_,
                corner(0, 1, 1): -fs_ + fu * fv,
                corner(0, 1, 0): fu - fu * fv,
                corner(0, 0, 1): fv - fu * fv,
            }
            for c, wc in contrib.items():
                w[c] = w[c] + np.where(sel, wc, 0.0)
        return list(w.items())
    raise ValueError(method)


def interp(lut, xform, method, x=None, v8=None):
    """Interpolate the LUT (N, N, N, 3) at normalised inputs x (..., 3) or at
    8-bit inputs v8 (..., 3).  Linear channels: sum_k w_k c_k.  Angular
    channels: angle of sum_k w_k (cos theta_k, sin theta_k); H of HSI is
    returned in [0, 2 pi), the SCT angles in (-pi, pi].
    Returns (values (..., 3), resultant length per channel (..., 3); 1 for
    linear channels)."""
    N = lut.shape[0]
    if v8 is not None:
        i, f = locate_u8(v8, N)
    else:
        i, f = locate(x, N)
    ang = ANGULAR[xform]
    acc = np.zeros(f.shape[:-1] + (3,))
    acc_c = np.zeros(f.shape[:-1] + (3,))
    acc_s = np.zeros(f.shape[:-1] + (3,))
    for (dr, dg, db), w in corner_weights(method, f):
        c = lut[i[..., 0] + dr, i[..., 1] + dg, i[..., 2] + db]
        acc += w[..., None] * c
        acc_c += w[..., None] * np.cos(c)
        acc_s += w[..., None] * np.sin(c)
    out = acc.copy()
    rlen = np.ones_like(acc)
    for ch in range(3):
        if ang[ch]:
            th = np.arctan2(acc_s[..., ch], acc_c[..., ch])
            if xform == "hsi":
                th = np.mod(th, 2.0 * np.pi)
            out[..., ch] = th
            rlen[..., ch] = np.hypot(acc_s[..., ch], acc_c[..., ch])
    return out, rlen


# ---------------------------------------------------------------- caching form
#
# Sec. 3.5.3 times a second version of every method, "caching": the
# differences between neighbouring lattice points are computed ahead of time
# and stored in each node.  Reading: a node, as the 000 corner of its cell,
# stores its own value and the differences along the 12 edges of that cell,
# 13 values per channel (33^3 nodes x 3 channels x 13 values x 8 bytes is the
# 10.7 MB the paper quotes as the largest LUT storage).  Each method then
# needs no subtraction per pixel: its value is the node value plus a weighted
# sum of edge differences, algebraically the standard weighted corner sum.
#
# Entry order in a record: 0 the node value c000; 1-4 the R edges
# c(1,g,b) - c(0,g,b) for (g, b) = 00, 01, 10, 11; 5-8 the G edges
# c(r,1,b) - c(r,0,b) for (r, b) = 00, 01, 10, 11; 9-12 the B edges
# c(r,g,1) - c(r,g,0) for (r, g) = 00, 01, 10, 11.


def edge_r(g, b):
    return 1 + 2 * g + b


def edge_g(r, b):
    return 5 + 2 * r + b


def edge_b(r, g):
    return 9 + 2 * r + g


def components(lut, xform):
    """The values a node contributes to a weighted sum: linear channels as
    they are, each angular channel as its unit vector (cos, sin)."""
    parts = []
    for ch, ang in enumerate(ANGULAR[xform]):
        if ang:
            parts += [np.cos(lut[..., ch]), np.sin(lut[..., ch])]
        else:
            parts.append(lut[..., ch])
    return np.stack(parts, axis=-1)


def build_cache(xform, N, gamma="bt709"):
    """The caching LUT: (N-1, N-1, N-1, 13, C) records, FP64, record (i, j, k)
    for the node (i, j, k) as the 000 corner of its cell; C the components of
    ``components`` (3 for CIELAB and CIELUV, 4 for HSI, 5 for SCT)."""
    c = components(build(xform, N, gamma), xform)
    m = N - 1

    def node(dr, dg, db):
        return c[dr:dr + m, dg:dg + m, db:db + m]

    rec = np.empty((m, m, m, 13, c.shape[-1]))
    rec[..., 0, :] = node(0, 0, 0)
    for u in (0, 1):
        for v in (0, 1):
            rec[..., edge_r(u, v), :] = node(1, u, v) - node(0, u, v)
            rec[..., edge_g(u, v), :] = node(u, 1, v) - node(u, 0, v)
            rec[..., edge_b(u, v), :] = node(u, v, 1) - node(u, v, 0)
    return rec


def cache_terms(method, f):
    """(entry, weight) pairs of a method in the caching form: the value is
    entry 0 plus sum weight x entry.  Derived from the corner weights of
    ``corner_weights`` by writing every corner as c000 plus the edges of a
    path to it:
      trilinear    c000 + f_B dB(00) + f_G [(1-f_B) dG(00) + f_B dG(01)]
                   + f_R [bilinear blend in (f_G, f_B) of the four R edges];
      tetrahedral  along the path of decreasing fractions: c000 + f1 (first
                   edge) + f2 (second) + f3 (third);
      prism        c000 + f_R dR(00) + the triangle's two edges, each blended
                   linearly along R;
      pyramidal    c000 + f_s (s edge at u = v = 1) + f_u (1 - f_v) (u edge at
                   s = v = 0) + f_v (v edge at s = u = 0) + f_u f_v (u edge at
                   s = 0, v = 1), for s the axis of the smallest fraction."""
    fr, fg, fb = f[..., 0], f[..., 1], f[..., 2]
    zero = np.zeros_like(fr)
    if method == "trilinear":
        return [(edge_b(0, 0), fb), (edge_g(0, 0), fg * (1 - fb)), (edge_g(0, 1), fg * fb),
                (edge_r(0, 0), fr * (1 - fg) * (1 - fb)), (edge_r(0, 1), fr * (1 - fg) * fb),
                (edge_r(1, 0), fr * fg * (1 - fb)), (edge_r(1, 1), fr * fg * fb)]
    if method == "prism":
        up = fg >= fb
        return [(edge_r(0, 0), fr),
                (edge_g(0, 0), np.where(up, fg * (1 - fr), zero)), (edge_g(1, 0), np.where(up, fg * fr, zero)),
                (edge_b(0, 1), np.where(up, fb * (1 - fr), zero)), (edge_b(1, 1), np.where(up, fb * fr, zero)),
                (edge_b(0, 0), np.where(up, zero, fb * (1 - fr))), (edge_b(1, 0), np.where(up, zero, fb * fr)),
                (edge_g(0, 1), np.where(up, zero, fg * (1 - fr))), (edge_g(1, 1), np.where(up, zero, fg * fr))]
    if method == "tetrahedral":
        # the six orders of the fractions, ties broken R before G before B as in corner_weights
        order = np.argsort(-f, axis=-1, kind="stable")
        fs = np.take_along_axis(f, order, axis=-1)
        terms = []
        for a1 in range(3):
            for a2 in range(3):
                if a2 == a1:
                    continue
                a3 = 3 - a1 - a2
                sel = (order[..., 0] == a1) & (order[..., 1] == a2)
                pos = [0, 0, 0]
                for k, a in enumerate((a1, a2, a3)):
                    others = [pos[j] for j in range(3) if j != a]
                    idx = (edge_r, edge_g, edge_b)[a](*others)
                    terms.append((idx, np.where(sel, fs[..., k], zero)))
                    pos[a] = 1
        return terms
    if method == "pyramidal":
        kmin = np.argmin(f, axis=-1)
        terms = []
        for s in range(3):
            sel = kmin == s
            u, v = [j for j in range(3) if j != s]

            def edge(axis, at):  # edge along `axis`, the other two coordinates from the dict `at`
                others = [at[j] for j in range(3) if j != axis]
                return (edge_r, edge_g, edge_b)[axis](*others)

            fs_, fu, fv = f[..., s], f[..., u], f[..., v]
            terms += [(edge(s, {u: 1, v: 1}), np.where(sel, fs_, zero)),
                      (edge(u, {s: 0, v: 0}), np.where(sel, fu * (1 - fv), zero)),
                      (edge(v, {s: 0, u: 0}), np.where(sel, fv, zero)),
                      (edge(u, {s: 0, v: 1}), np.where(sel, fu * fv, zero))]
        return terms
    raise ValueError(method)


def interp_cache(cache, xform, method, x=None, v8=None):
    """Interpolate with the caching form (``build_cache``) at normalised x or
    8-bit v8: the record of the pixel's cell, entry 0 plus the method's
    weighted edge differences, per component; angular channels are the angle
    of their (cos, sin) resultant, as in ``interp``.  Returns (values,
    resultant length per channel)."""
    N = cache.shape[0] + 1
    if v8 is not None:
        i, f = locate_u8(v8, N)
    else:
        i, f = locate(x, N)
    rec = cache[i[..., 0], i[..., 1], i[..., 2]]  # (..., 13, C)
    acc = rec[..., 0, :].copy()
    for e, w in cache_terms(method, f):
        acc += w[..., None] * rec[..., e, :]
    out = np.empty(f.shape[:-1] + (3,))
    rlen = np.ones_like(out)
    k = 0
    for ch, ang in enumerate(ANGULAR[xform]):
        if ang:
            th = np.arctan2(acc[..., k + 1], acc[..., k])
            if xform == "hsi":
                th = np.mod(th, 2.0 * np.pi)
            out[..., ch] = th
            rlen[..., ch] = np.hypot(acc[..., k], acc[..., k + 1])
            k += 2
        else:
            out[..., ch] = acc[..., k]
            k += 1
    return out, rlen
