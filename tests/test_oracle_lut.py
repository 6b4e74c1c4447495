"""Invariants of the oracle's LUT interpolators, checked against independent
constructions (CPU only).  Table 12 is checked in test_oracle_paper.py."""
import itertools

import numpy as np
import pytest
import scipy.interpolate

import synth
from oracle import lut

METHODS = ["trilinear", "prism", "pyramidal", "tetrahedral"]


def _affine_lut(N, A, c):
    v = lut.node_inputs(N)
    g = np.stack(np.meshgrid(v, v, v, indexing="ij"), axis=-1)
    return g @ A.T + c


@pytest.mark.parametrize("method", METHODS)
def test_weights_partition_unity(method):
    f = synth.rng(1).random((5000, 3))
    ws = lut.corner_weights(method, f)
    total = sum(w for _, w in ws)
    np.testing.assert_allclose(total, 1.0, atol=1e-15)
    if method != "pyramidal":
        assert min(w.min() for _, w in ws) >= -1e-15


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("N", [9, 17, 33])
def test_affine_precision(method, N):
    g = synth.rng(N)
    A = g.normal(size=(3, 3))
    c = g.normal(size=3)
    L = _affine_lut(N, A, c)
    x = g.random((20000, 3))
    out, _ = lut.interp(L, "lab", method, x=x)
    np.testing.assert_allclose(out, x @ A.T + c, atol=1e-12)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct"])
def test_node_hits(method, xform):
    N = 17
    L = lut.build(xform, N)
    idx = np.array(list(itertools.product(range(N), repeat=3)))
    out, _ = lut.interp(L, xform, method, x=idx / (N - 1.0))
    want = L[idx[:, 0], idx[:, 1], idx[:, 2]]
    for ch, ang in enumerate(lut.ANGULAR[xform]):
        if ang:
            d = np.abs(np.angle(np.exp(1j * (out[:, ch] - want[:, ch]))))
            assert d.max() < 1e-12
        else:
            np.testing.assert_allclose(out[:, ch], want[:, ch], atol=1e-12)


def test_trilinear_equals_library_grid_interpolator():
    N = 9
    L = lut.build("lab", N)
    x = synth.rng(5).random((10000, 3))
    v = lut.node_inputs(N)
    ref = scipy.interpolate.RegularGridInterpolator((v, v, v), L, method="linear")(x)
    out, _ = lut.interp(L, "lab", "trilinear", x=x)
    np.testing.assert_allclose(out, ref, atol=1e-11)


def _barycentric(verts, p):
    # solve p = sum l_k v_k with sum l_k = 1
    M = np.vstack([np.asarray(verts, dtype=float).T, np.ones(len(verts))])
    return np.linalg.solve(M, np.append(p, 1.0))


def test_tetrahedral_is_barycentric_in_sorted_simplex():
    # the cube splits into 6 tetrahedra {f_a >= f_b >= f_c}; inside one the value is the
    # barycentric interpolation of its 4 vertices
    N = 5
    L = lut.build("lab", N)
    g = synth.rng(6)
    for _ in range(300):
        x = g.random(3)
        pos = x * (N - 1)
        i = np.minimum(np.floor(pos).astype(int), N - 2)
        f = pos - i
        order = np.argsort(-f)
        verts = [np.zeros(3)]
        for k in order:
            v = verts[-1].copy()
            v[k] = 1
            verts.append(v)
        lam = _barycentric(verts, f)
        want = sum(l * L[tuple(i + v.astype(int))] for l, v in zip(lam, verts))
        out, _ = lut.interp(L, "lab", "tetrahedral", x=x[None])
        np.testing.assert_allclose(out[0], want, atol=1e-11)


def test_prism_is_triangle_barycentric_times_lerp_along_r():
    N = 5
    L = lut.build("lab", N)
    g = synth.rng(7)
    for _ in range(300):
        x = g.random(3)
        pos = x * (N - 1)
        i = np.minimum(np.floor(pos).astype(int), N - 2)
        f = pos - i
        tri = [(0, 0), (1, 0), (1, 1)] if f[1] >= f[2] else [(0, 0), (0, 1), (1, 1)]
        M = np.vstack([np.array(tri, dtype=float).T, np.ones(3)])
        lam = np.linalg.solve(M, np.array([f[1], f[2], 1.0]))
        want = 0
        for dr, wr in ((0, 1 - f[0]), (1, f[0])):
            for l, (dg, db) in zip(lam, tri):
                want = want + wr * l * L[i[0] + dr, i[1] + dg, i[2] + db]
        out, _ = lut.interp(L, "lab", "prism", x=x[None])
        np.testing.assert_allclose(out[0], want, atol=1e-11)


def test_pyramidal_base_face_is_bilinear_and_apex_edge_is_linear():
    # the reading of the pyramidal method: apex at corner 111, base the cell face through 000
    # normal to the axis s of the smallest fraction.  On that face (f_s = 0) the value is the
    # bilinear interpolation of the face's four corners (the library's 2-D grid interpolator);
    # on the edge from the base's far corner (f_u = f_v = 1) to the apex it is the linear
    # interpolation of the edge's two nodes (np.interp).  CIELAB nodes, which are not affine
    N = 5
    L = lut.build("lab", N)
    g = synth.rng(8)
    for s in range(3):
        u, v = [j for j in range(3) if j != s]
        for _ in range(100):
            # base face: f_s = 0 in a random cell, the other two fractions in (0, 1)
            i = g.integers(0, N - 1, 3)
            f = np.zeros(3)
            f[u], f[v] = g.uniform(0.01, 0.99, 2)
            x = (i + f) / (N - 1)
            face = np.empty((2, 2, 3))
            for du in (0, 1):
                for dv in (0, 1):
                    c = i.copy()
                    c[u] += du
                    c[v] += dv
                    face[du, dv] = L[tuple(c)]
            want = scipy.interpolate.RegularGridInterpolator(([0.0, 1.0], [0.0, 1.0]), face)([[f[u], f[v]]])[0]
            out, _ = lut.interp(L, "lab", "pyramidal", x=x[None])
            np.testing.assert_allclose(out[0], want, atol=1e-11)
            # apex edge: f_u = f_v = 1 (the last cell along u and v), f_s in [0, 1)
            j = g.integers(0, N - 1, 3)
            j[u] = j[v] = N - 2
            fs = g.uniform(0.0, 0.99)
            x = np.empty(3)
            x[s] = (j[s] + fs) / (N - 1)
            x[u] = x[v] = 1.0
            a = j.copy()
            a[u] += 1
            a[v] += 1
            b = a.copy()
            b[s] += 1
            want = np.array([np.interp(fs, [0.0, 1.0], [L[tuple(a)][ch], L[tuple(b)][ch]]) for ch in range(3)])
            out, _ = lut.interp(L, "lab", "pyramidal", x=x[None])
            np.testing.assert_allclose(out[0], want, atol=1e-11)


@pytest.mark.parametrize("method", ["trilinear", "prism", "tetrahedral"])
def test_continuity_across_cell_faces(method):
    # the pyramidal polynomial form is not continuous (neither across cell faces nor across
    # its own pyramid boundaries), so it is held to node hits and affine precision only
    N = 9
    L = lut.build("lab", N)
    g = synth.rng(8)
    x = g.random((2000, 3))
    ax = g.integers(0, 3, 2000)
    face = g.integers(1, N - 1, 2000) / (N - 1.0)
    x[np.arange(2000), ax] = face
    d = 1e-10
    lo, hi = x.copy(), x.copy()
    lo[np.arange(2000), ax] -= d
    hi[np.arange(2000), ax] += d
    a, _ = lut.interp(L, "lab", method, x=lo)
    b, _ = lut.interp(L, "lab", method, x=hi)
    assert np.abs(a - b).max() < 1e-6


def test_u8_extraction_matches_float_extraction():
    v = np.arange(256)
    for N in (9, 17, 33, 2, 256):
        i8, f8 = lut.locate_u8(v, N)
        i, f = lut.locate(v / 255.0, N)
        np.testing.assert_array_equal(i8, i)
        np.testing.assert_allclose(f8, f, atol=1e-13)
        assert f8.min() >= 0 and f8.max() <= 1


def test_angular_channels_wrap_and_constant():
    N = 3
    L = np.zeros((N, N, N, 3))
    L[..., 0] = 0.7
    x = synth.rng(9).random((1000, 3))
    for m in METHODS:
        out, r = lut.interp(L, "hsi", m, x=x)
        np.testing.assert_allclose(out[:, 0], 0.7, atol=1e-12)
        np.testing.assert_allclose(r[:, 0], 1.0, atol=1e-12)
    # angles 0.1 and 2 pi - 0.1 meet at 0, not at pi
    L[..., 0] = 0.1
    L[1:, ..., 0] = 2 * np.pi - 0.1
    out, _ = lut.interp(L, "hsi", "trilinear", x=np.array([[0.25, 0.0, 0.0]]))
    assert np.angle(np.exp(1j * out[0, 0])) == pytest.approx(0.0, abs=1e-12)


def test_angular_channel_on_a_cell_edge_is_the_two_vector_resultant():
    # on the R edge of a cell (f_G = f_B = 0) every method weighs the edge's two nodes by
    # 1 - f and f.  The resultant of the unit vectors at angles t1 and t2 with those weights,
    # in a frame rotated by t1: angle t1 + atan2(f sin d, 1 - f + f cos d) with d = t2 - t1
    # wrapped into (-pi, pi], length sqrt((1 - f)^2 + f^2 + 2 f (1 - f) cos d) (law of cosines)
    N = 4
    g = synth.rng(10)
    L = np.zeros((N, N, N, 3))
    L[..., 0] = g.uniform(0.0, 2 * np.pi, (N, N, N))
    for m in METHODS:
        for _ in range(200):
            i, j, k = g.integers(0, N - 1, 3)
            f = g.uniform(0.0, 1.0)
            x = np.array([[(i + f) / (N - 1), j / (N - 1), k / (N - 1)]])
            t1, t2 = L[i, j, k, 0], L[i + 1, j, k, 0]
            d = np.angle(np.exp(1j * (t2 - t1)))
            want = t1 + np.arctan2(f * np.sin(d), 1 - f + f * np.cos(d))
            length = np.sqrt((1 - f) ** 2 + f ** 2 + 2 * f * (1 - f) * np.cos(d))
            out, r = lut.interp(L, "hsi", m, x=x)
            assert abs(np.angle(np.exp(1j * (out[0, 0] - want)))) < 1e-9, (m, i, j, k, f)
            assert r[0, 0] == pytest.approx(length, abs=1e-12), (m, i, j, k, f)


def test_pyramidal_form_is_discontinuous_at_pyramid_boundary():
    # documents the reading: with only c010 = 1, the R-pyramid form gives f (1 - f_B) on
    # the plane f_R = f_G while the G-pyramid form gives 0
    L = np.zeros((2, 2, 2, 3))
    L[0, 1, 0, :] = 1.0
    f = 0.3
    fb = 0.6
    below, _ = lut.interp(L, "lab", "pyramidal", x=np.array([[f - 1e-12, f, fb]]))
    above, _ = lut.interp(L, "lab", "pyramidal", x=np.array([[f, f - 1e-12, fb]]))
    assert below[0, 0] == pytest.approx(f * (1 - fb), abs=1e-9)
    assert above[0, 0] == pytest.approx(0.0, abs=1e-9)


@pytest.mark.parametrize("method", ["trilinear", "prism", "pyramidal", "tetrahedral"])
@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_caching_form_equals_the_standard_form(xform, method):
    # Sec. 3.5.3's caching version stores per node its value and the differences to its
    # neighbours; every method then adds weighted differences to the node value.  It is the same
    # interpolant: equal to the weighted corner sum to FP64 rounding, at float and 8-bit inputs,
    # at nodes and on cell faces (where the pyramidal form's choice of pyramid changes)
    g = synth.rng(17)
    for N in (2, 9, 17):
        std, cache = lut.build(xform, N), lut.build_cache(xform, N)
        x = np.concatenate([g.random((5000, 3)), lut.node_inputs(N)[g.integers(0, N, (500, 3))],
                            np.repeat(g.random((500, 1)), 3, axis=1)])
        v8 = np.concatenate([g.integers(0, 256, (5000, 3)), [[0, 0, 0], [255, 255, 255], [255, 0, 0], [7, 7, 200]]])
        for kw in ({"x": x}, {"v8": v8}):
            a, ra = lut.interp(std, xform, method, **kw)
            b, rb = lut.interp_cache(cache, xform, method, **kw)
            d = np.abs(a - b)
            ang = np.array(lut.ANGULAR[xform])
            d[:, ang] = np.minimum(d[:, ang], 2 * np.pi - d[:, ang]) * ra[:, ang]
            assert d.max() <= 1e-12 * max(1.0, np.abs(a).max()), (N, list(kw), d.max())
            np.testing.assert_allclose(rb, ra, rtol=0, atol=1e-12)


def test_caching_record_size_is_the_papers_storage():
    # 13 values per channel and node (the node value and its cell's 12 edge differences): the
    # 33^3 three-channel CIELAB LUT in FP64 is the 10.7 MB the paper quotes as the largest storage
    rec = lut.build_cache("lab", 33)
    assert rec.shape == (32, 32, 32, 13, 3)
    assert round(33 ** 3 * rec.shape[-1] * rec.shape[-2] * 8 / 2 ** 20, 1) == 10.7
    # the four edges along one axis of a cell differ by the second differences, and a cell's
    # edges close: going round a face (R then G, or G then R) reaches the same corner
    r, gg = rec[..., lut.edge_r(0, 0), :] + rec[..., lut.edge_g(1, 0), :], \
        rec[..., lut.edge_g(0, 0), :] + rec[..., lut.edge_r(1, 0), :]
    np.testing.assert_allclose(r, gg, rtol=0, atol=1e-12)
