"""The scalar C oracle (oracle/cbase.c), pinned to what the paper and the
definitions fix: the D65 white and black, Table 8 (all nine rows, printed
rationals, every 8-bit colour), Table 12's tetrahedral rows at 9^3, 17^3 and
33^3, and exact node hits; cross-checked against the numpy oracle.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import cbase, colour, lut as OL, mact, tables as T

THREADS = 8


@pytest.fixture(scope="module")
def cube():
    return synth.cube_u8().reshape(-1, 3)


@pytest.fixture(scope="module")
def exact(cube):
    return cbase.lab_exact_u8(cube, threads=THREADS)


def test_white_and_black():
    out = cbase.lab_exact_u8(np.array([[255, 255, 255], [0, 0, 0]], dtype=np.uint8))
    np.testing.assert_allclose(out[0], [100.0, 0.0, 0.0], atol=1e-9)
    np.testing.assert_allclose(out[1], [0.0, 0.0, 0.0], atol=1e-12)


def test_table8_with_the_printed_rationals(cube, exact):
    # every row of Table 8: mean and max Delta E*ab of the MACT transform against the exact one
    # over all 2^24 colours, to the printed digits (the printed coefficients carry 7)
    for key, (_, p, q) in T.T2_CBRT_RAT.items():
        d = colour.delta_e(cbase.lab_mact_u8(cube, p, q, threads=THREADS), exact)
        avg, mx = T.T8_CIELAB_ERR[key]
        assert d.mean() == pytest.approx(avg, abs=6e-6), key
        assert d.max() == pytest.approx(mx, abs=6e-6), key


@pytest.mark.parametrize("N", [9, 17, 33])
def test_table12_tetrahedral_rows(cube, exact, N):
    lut = cbase.lut_build_lab(N)
    d = colour.delta_e(cbase.lut_tetra_u8(lut, cube, threads=THREADS), exact)
    avg, mx = T.T12_LUT_ERR[("tetrahedral", N)]
    assert d.mean() == pytest.approx(avg, abs=2e-6)
    assert d.max() == pytest.approx(mx, abs=2e-6)


def test_node_hits_and_lut_nodes():
    # 8-bit inputs on the nodes of a 17^3 grid (multiples of 255/16 are not integers, so use the
    # 2^k + 1 grids whose nodes 0 and 255 are codes): the corners of the cube give the nodes
    lut = cbase.lut_build_lab(17)
    v = np.array([[0, 0, 0], [255, 255, 255], [255, 0, 0], [0, 255, 255]], dtype=np.uint8)
    got = cbase.lut_tetra_u8(lut, v)
    np.testing.assert_array_equal(got, lut[[0, 16, 16, 0], [0, 16, 0, 16], [0, 16, 0, 16]])
    np.testing.assert_allclose(lut, OL.build("lab", 17), rtol=0, atol=1e-12)


def test_agrees_with_the_numpy_oracle():
    v = synth.uniform_u8(200, 300, seed=11).reshape(-1, 3)
    x = v / 255.0
    np.testing.assert_allclose(cbase.lab_exact_u8(v), colour.rgb_to_lab(x), rtol=0, atol=1e-11)
    _, p, q = T.T2_CBRT_RAT[(4, 4)]
    np.testing.assert_allclose(cbase.lab_mact_u8(v, p, q), mact.mact_lab(x, p, q), rtol=0, atol=1e-11)
    lut = cbase.lut_build_lab(33)
    ref, _ = OL.interp(OL.build("lab", 33), "lab", "tetrahedral", v8=v)
    np.testing.assert_allclose(cbase.lut_tetra_u8(lut, v), ref, rtol=0, atol=1e-11)


def test_threads_give_the_same_bits(cube):
    v = cube[::97]
    _, p, q = T.T2_CBRT_RAT[(3, 3)]
    np.testing.assert_array_equal(cbase.lab_mact_u8(v, p, q, threads=1), cbase.lab_mact_u8(v, p, q, threads=7))
    lut = cbase.lut_build_lab(17)
    np.testing.assert_array_equal(cbase.lut_tetra_u8(lut, v, threads=1), cbase.lut_tetra_u8(lut, v, threads=5))
