"""Pins of the oracle's Remez exchange: textbook closed forms, the Chebyshev
equioscillation characterisation, an independent LP discrete minimax, and
the errors printed in the paper's Tables 1-7 (CPU only)."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as Pm

from oracle import remez, tables as T


def _alternation_ok(fit, f, rel=1e-6):
    e = fit(fit.alt) - f(fit.alt)
    n_pts = len(fit.p) + len(fit.q)  # n + m + 2
    assert len(fit.alt) == n_pts
    assert np.all(np.sign(e[1:]) == -np.sign(e[:-1])), e
    np.testing.assert_allclose(np.abs(e), fit.eps, rtol=rel)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_chebyshev_monomial_closed_form(n):
    # best degree-n approximation of x^(n+1) on [-1, 1]: error 2^-n, alternation at cos(k pi/(n+1))
    f = lambda x: np.asarray(x, dtype=np.float64) ** (n + 1)
    fit = remez.remez(f, n, 0, -1.0, 1.0)
    assert fit.converged
    assert fit.eps == pytest.approx(2.0 ** (-n), rel=1e-10)
    want = np.sort(np.cos(np.pi * np.arange(n + 2) / (n + 1)))
    np.testing.assert_allclose(np.sort(fit.alt), want, atol=1e-7)
    _alternation_ok(fit, f)


def test_degree_one_convex_closed_form():
    # the linear minimax of a convex f: secant slope; tangent point xi with f'(xi) = slope
    a, b = 0.0, 1.0
    c1 = (np.e - 1.0) / (b - a)
    xi = np.log(c1)
    c0 = 0.5 * (1.0 + np.exp(xi)) - c1 * 0.5 * (a + xi)
    fit = remez.remez(np.exp, 1, 0, a, b)
    np.testing.assert_allclose(fit.p, [c0, c1], rtol=1e-12)
    assert fit.eps == pytest.approx(abs(np.exp(xi) - (c0 + c1 * xi)), rel=1e-10)


POLY_TABLES = [
    ("cbrt", T.T1_CBRT_POLY, T.T1_INTERVAL),
    ("atan_sqrt3", T.T3_ATAN_SQRT3, T.T3_INTERVAL),
    ("asin2", T.T4_ASIN2, T.T4_INTERVAL),
    ("acos", T.T5_ACOS, T.T5_INTERVAL),
    ("atan", T.T6_ATAN, T.T6_INTERVAL),
    ("atanc", T.T7_ATANC, T.T7_INTERVAL),
]


@pytest.mark.parametrize("name,table,interval", POLY_TABLES, ids=[t[0] for t in POLY_TABLES])
def test_polynomial_tables(name, table, interval):
    f = T.FUNCS[name]
    a, b = interval
    for n, (eps_printed, coeffs) in table.items():
        fit = remez.remez(f, n, 0, a, b)
        # a true minimax fit is never worse than the printed one, and the printed errors are
        # those of near-optimal fits on these intervals (within 0.2%)
        assert fit.eps <= eps_printed * (1 + 2e-5), (name, n, fit.eps, eps_printed)
        assert fit.eps >= eps_printed * (1 - 2e-3), (name, n, fit.eps, eps_printed)
        _alternation_ok(fit, f, rel=1e-5)


def test_table3_coefficients_and_sign_reading():
    # the fitted coefficients on [0, 254/256] equal the printed ones to their 7 digits
    for n, (eps, c) in T.T3_ATAN_SQRT3.items():
        fit = remez.remez(T.f_atan_sqrt3, n, 0, *T.T3_INTERVAL)
        np.testing.assert_allclose(fit.p, c, atol=1e-6)
    # the n = 2 row as printed (a2 > 0) is far from arctan(sqrt 3 x); with a2 < 0 it levels at eps
    x = np.linspace(0, 254 / 256, 10001)
    c = list(T.T3_ATAN_SQRT3[2][1])
    assert np.max(np.abs(Pm.polyval(x, c) - T.f_atan_sqrt3(x))) == pytest.approx(6.9079e-3, rel=1e-3)
    c[2] = -c[2]
    assert np.max(np.abs(Pm.polyval(x, c) - T.f_atan_sqrt3(x))) > 1.0


def test_table1_interval_is_0_1():
    # for n >= 3 the printed error equals a0: the error at t = 0 is eps, so the fit starts at 0
    for n in (3, 4, 5):
        eps, c = T.T1_CBRT_POLY[n]
        assert c[0] == pytest.approx(eps, rel=1e-5)


def test_table2_interval_and_printed_levels():
    # every printed rational has its error +eps at t = 0.008856 (left end of the fit interval)
    for (n, m), (eps, p, q) in T.T2_CBRT_RAT.items():
        e0 = Pm.polyval(T.T2_INTERVAL[0], p) / Pm.polyval(T.T2_INTERVAL[0], q) - np.cbrt(T.T2_INTERVAL[0])
        assert e0 == pytest.approx(eps, rel=2e-3), (n, m)


@pytest.mark.parametrize("nm", [(2, 2), (2, 3), (3, 2)])
def test_rational_small_rows_match_table2(nm):
    eps_printed = T.T2_CBRT_RAT[nm][0]
    fit = remez.remez(T.f_cbrt, nm[0], nm[1], *T.T2_INTERVAL)
    assert fit.converged
    assert eps_printed * (1 - 1.5e-2) <= fit.eps <= eps_printed
    _alternation_ok(fit, T.f_cbrt, rel=1e-5)


@pytest.mark.parametrize("nm", [(2, 2), (3, 3), (4, 4)])
def test_rational_matches_lp_minimax(nm):
    # an independent algorithm (LP on a 3001-point grid) reaches the same optimum
    n, m = nm
    fit = remez.remez(T.f_cbrt, n, m, *T.T2_INTERVAL)
    _, _, eps_lp = remez.lp_minimax(T.f_cbrt, n, m, *T.T2_INTERVAL)
    assert fit.eps <= eps_lp * (1 + 1e-3)
    assert fit.eps >= eps_lp * (1 - 1e-2)
    _alternation_ok(fit, T.f_cbrt, rel=1e-5)


def test_rational_44_beats_printed_row():
    # the printed (4, 4) row is not levelled (its extrema decay from 3.9e-5 to ~5e-6);
    # the minimax optimum is about 1.089e-5
    fit = remez.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL)
    assert fit.eps == pytest.approx(1.0887e-5, rel=2e-3)
    assert np.all(fit.q > 0)


def test_polynomial_matches_lp_minimax():
    fit = remez.remez(T.f_atan, 5, 0, 0.0, 1.0)
    _, _, eps_lp = remez.lp_minimax(T.f_atan, 5, 0, 0.0, 1.0)
    assert fit.eps == pytest.approx(eps_lp, rel=1e-4)


# ----------------------------------------------------------------- weighted fits


def _weighted_alternation_ok(fit, f, w, rel=1e-6):
    e = w(fit.alt) * (fit(fit.alt) - f(fit.alt))
    assert len(fit.alt) == len(fit.p) + len(fit.q)
    assert np.all(np.sign(e[1:]) == -np.sign(e[:-1])), e
    np.testing.assert_allclose(np.abs(e), fit.eps, rtol=rel)


def test_weighted_relative_sqrt_closed_form():
    # relative-error (w = 1/f) linear minimax of sqrt on [a, b]: the weighted error
    # (c0 + c1 x)/sqrt(x) - 1 is convex in sqrt(x) with its minimum at x* = c0/c1; levelling
    # it at a, x*, b gives c0 = c1 sqrt(ab), c1 = 2 / (a^(1/4) + b^(1/4))^2 and the level
    # c1 (sqrt(a) + sqrt(b)) - 1
    a, b = 0.25, 1.0
    c1 = 2.0 / (a ** 0.25 + b ** 0.25) ** 2
    c0 = c1 * np.sqrt(a * b)
    level = c1 * (np.sqrt(a) + np.sqrt(b)) - 1.0
    w = lambda x: 1.0 / np.sqrt(x)
    fit = remez.remez(np.sqrt, 1, 0, a, b, w=w)
    assert fit.converged
    np.testing.assert_allclose(fit.p, [c0, c1], rtol=1e-10)
    assert fit.eps == pytest.approx(level, rel=1e-9)
    np.testing.assert_allclose(np.sort(fit.alt), [a, np.sqrt(a * b), b], atol=1e-7)
    _weighted_alternation_ok(fit, np.sqrt, w)


def test_weighted_constant_closed_form():
    # best constant for f(x) = x on [0, 1] under w = 1 + x: w(0) c = w(1) (1 - c), so c = 2/3
    # and the level is 2/3 (w (c - x) falls on [0, c] and w (x - c) rises on [c, 1])
    w = lambda x: 1.0 + np.asarray(x, dtype=np.float64)
    fit = remez.remez(lambda x: np.asarray(x, dtype=np.float64), 0, 0, 0.0, 1.0, w=w)
    assert fit.p[0] == pytest.approx(2.0 / 3.0, rel=1e-12)
    assert fit.eps == pytest.approx(2.0 / 3.0, rel=1e-9)


def test_constant_weight_scales_the_level_only():
    # a constant weight c leaves the best approximation unchanged and scales the level by c
    plain = remez.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL)
    w3 = remez.remez(T.f_cbrt, 4, 4, *T.T2_INTERVAL, w=lambda x: np.full_like(np.asarray(x, dtype=np.float64), 3.0))
    np.testing.assert_allclose(w3.p, plain.p, rtol=1e-7)
    np.testing.assert_allclose(w3.q, plain.q, rtol=1e-7)
    assert w3.eps == pytest.approx(3.0 * plain.eps, rel=1e-6)


def _damped(beta, delta, a=T.T2_INTERVAL[0], b=T.T2_INTERVAL[1]):
    return lambda x: ((np.asarray(x, dtype=np.float64) - a + delta) / (b - a + delta)) ** beta


@pytest.mark.parametrize("nm", [(2, 2), (3, 3), (4, 4)])
def test_weighted_rational_matches_lp_minimax(nm):
    # an independent algorithm (LP with the weight in its bounds) reaches the same weighted optimum
    n, m = nm
    w = _damped(0.5, 0.02)
    fit = remez.remez(T.f_cbrt, n, m, *T.T2_INTERVAL, w=w)
    assert fit.converged
    _, _, eps_lp = remez.lp_minimax(T.f_cbrt, n, m, *T.T2_INTERVAL, w=w)
    assert fit.eps <= eps_lp * (1 + 1e-3)
    assert fit.eps >= eps_lp * (1 - 1e-2)
    _weighted_alternation_ok(fit, T.f_cbrt, w, rel=1e-5)


def test_weighted_polynomial_matches_lp_minimax():
    w = lambda x: 1.0 + 4.0 * np.asarray(x, dtype=np.float64) ** 2
    fit = remez.remez(T.f_atan, 5, 0, 0.0, 1.0, w=w)
    _, _, eps_lp = remez.lp_minimax(T.f_atan, 5, 0, 0.0, 1.0, w=w)
    # the LP solver's feasibility tolerance (1e-7 on constraints scaled by w up to 5) leaves
    # its level a few 1e-4 above the optimum; the alternation below is the optimality proof
    assert eps_lp * (1 - 1e-2) <= fit.eps <= eps_lp * (1 + 1e-3)
    _weighted_alternation_ok(fit, T.f_atan, w)
