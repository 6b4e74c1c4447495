"""Coefficient tables printed in the paper (oracle; test infrastructure only).

Coefficients are monomial, lowest degree first, as printed (7 significant
digits).  Each entry records the function approximated, the interval the
printed error refers to, and the printed maximum error eps^A_max.

Readings of the printed tables (each is justified by a test in
tests/test_oracle_remez.py or tests/test_oracle_paper.py):
  * Table 1 (cube-root polynomials): the figure caption suggests
    [0.008856, 1], but the printed errors are those of fits on [0, 1]
    (the error at 0 equals a0 = eps); interval [0, 1].
  * Table 2 (cube-root rationals): interval [0.008856, 1]; the printed
    denominators are not normalised (neither q0 = 1 nor monic).
  * Table 3 (arctan(sqrt(3) x)), n = 2: a2 is printed as +7.497879e-01; the
    sign was lost: with + the error at x = 1 is about 1.5, with - the row
    equioscillates at the printed eps.  Interval [0, 254/256].
  * Table 4: 2 arcsin(y / sqrt 2) on [0, 1/sqrt 2].
  * Table 5: arccos on [0, 0.5].
  * Table 6: arctan on [0, 254/255].
  * Table 7: pi/2 - arctan(t) on [1/255, 1] (the arctan inside g takes
    R/G there).
"""
import numpy as np

SQRT3 = np.sqrt(3.0)


def f_cbrt(t):
    return np.cbrt(t)


def f_atan_sqrt3(x):
    return np.arctan(SQRT3 * np.asarray(x, dtype=np.float64))


def f_asin2(y):
    return 2.0 * np.arcsin(np.asarray(y, dtype=np.float64) / np.sqrt(2.0))


def f_acos(x):
    return np.arccos(x)


def f_atan(x):
    return np.arctan(x)


def f_atanc(t):
    return 0.5 * np.pi - np.arctan(t)


FUNCS = {
    "cbrt": f_cbrt,
    "atan_sqrt3": f_atan_sqrt3,
    "asin2": f_asin2,
    "acos": f_acos,
    "atan": f_atan,
    "atanc": f_atanc,
}

# Table 1: minimax polynomials for the cube root, fitted on [0, 1].
T1_CBRT_POLY = {
    2: (1.271154e-01, [1.268979e-01, 2.393873, -1.647669]),
    3: (9.787829e-02, [9.787826e-02, 4.057495, -7.388864, 4.331370]),
    4: (8.111150e-02, [8.111133e-02, 5.926004, -2.017165e+01, 2.833070e+01, -1.324728e+01]),
    5: (7.002956e-02, [7.002910e-02, 7.961214, -4.329352e+01, 1.063182e+02, -1.135685e+02, 4.358268e+01]),
}
T1_INTERVAL = (0.0, 1.0)

# Table 2: minimax rationals p/q for the cube root on [0.008856, 1].
# key (n, m) -> (eps, p, q)
T2_CBRT_RAT = {
    (2, 2): (2.060996e-03, [6.309655e-03, 5.785782e-01, 1.591005],
             [4.482646e-02, 1.175862, 9.596879e-01]),
    (2, 3): (7.210231e-04, [2.500705e-03, 3.447113e-01, 1.942708],
             [1.978701e-02, 8.542797e-01, 1.664540, -2.503267e-01]),
    (3, 2): (5.931593e-04, [1.776519e-03, 2.632323e-01, 1.751297, 3.836709e-01],
             [1.432256e-02, 6.779998e-01, 1.706260]),
    (2, 4): (3.107735e-04, [1.317899e-03, 2.390113e-01, 2.099395],
             [1.124254e-02, 6.726679e-01, 2.184656, -7.511150e-01, 2.229717e-01]),
    (3, 3): (1.858694e-04, [4.370889e-04, 9.526952e-02, 1.252009, 1.302733],
             [3.912364e-03, 2.954084e-01, 1.717143, 6.343408e-01]),
    (4, 2): (2.334688e-04, [7.589302e-04, 1.519784e-01, 1.663584, 8.368075e-01, -1.657269e-01],
             [6.644723e-03, 4.506424e-01, 2.030622]),
    (3, 4): (8.539863e-05, [1.683667e-04, 4.667675e-02, 9.106812e-01, 1.810577],
             [1.610864e-03, 1.617974e-01, 1.494070, 1.218468, -1.079451e-01]),
    (4, 3): (8.052920e-05, [1.349673e-04, 3.832079e-02, 7.870174e-01, 1.799062, 2.071170e-01],
             [1.299250e-03, 1.345420e-01, 1.330358, 1.365369]),
    (4, 4): (3.856930e-05, [3.927283e-05, 1.392318e-02, 4.114739e-01, 1.734853, 8.679223e-01],
             [4.022100e-04, 5.414536e-02, 8.221526e-01, 1.800167, 3.513617e-01]),
}
T2_INTERVAL = (0.008856, 1.0)

# Table 3: minimax polynomials for arctan(sqrt(3) x); n = 2 row with the
# sign of a2 restored (see module docstring).
T3_ATAN_SQRT3 = {
    2: (6.907910e-03, [5.959793e-03, 1.782975, -7.497879e-01]),
    3: (3.654156e-03, [-3.654076e-03, 1.884080, -9.805583e-01, 1.430580e-01]),
    4: (1.286371e-03, [-1.286369e-03, 1.796716, -4.958969e-01, -6.927404e-01, 4.421541e-01]),
    5: (1.801311e-04, [-1.801283e-04, 1.739333, -2.039848e-02, -2.065512, 2.052837, -6.591729e-01]),
}
T3_INTERVAL = (0.0, 254.0 / 256.0)

# Table 4: 2 arcsin(y / sqrt 2) on [0, 1/sqrt 2].
T4_ASIN2 = {
    4: (2.097814e-05, [2.097797e-05, 1.412840, 1.429881e-02, 6.704361e-02, 6.909677e-02]),
    5: (2.370540e-06, [-2.370048e-06, 1.414434, -3.300037e-03, 1.354670e-01, -3.994259e-02, 6.099502e-02]),
}
T4_INTERVAL = (0.0, 1.0 / np.sqrt(2.0))

# Table 5: arccos on [0, 0.5].
T5_ACOS = {
    4: (1.048949e-05, [1.570786, -9.990285e-01, -1.429899e-02, -9.481335e-02, -1.381942e-01]),
    5: (1.186403e-06, [1.570798, -1.000156, 3.299810e-03, -1.915780e-01, 7.988231e-02, -1.725177e-01]),
}
T5_INTERVAL = (0.0, 0.5)

# Table 6: f = arctan on [0, 254/255].
T6_ATAN = {
    4: (1.036515e-04, [-1.036508e-04, 1.003740, -1.773538e-02, -3.390563e-01, 1.386796e-01]),
    5: (2.073939e-05, [2.073866e-05, 9.982666e-01, 2.352573e-02, -4.506862e-01, 2.635050e-01, -4.920822e-02]),
}
T6_INTERVAL = (0.0, 254.0 / 255.0)

# Table 7: g's polynomial, pi/2 - arctan(t) on [1/255, 1].
T7_ATANC = {
    4: (1.051643e-04, [1.570917, -1.004004, 1.885694e-02, 3.373159e-01, -1.377930e-01]),
    5: (2.012104e-05, [1.570769, -9.981253e-01, -2.440212e-02, 4.528921e-01, -2.659181e-01, 5.016228e-02]),
}
T7_INTERVAL = (1.0 / 255.0, 1.0)

# Tables 8-10 and 12: transformation errors over all 2^24 8-bit colours
# (eps^T_avg, eps^T_max).
T8_CIELAB_ERR = {
    (2, 2): (0.787741, 2.225399), (2, 3): (0.295577, 0.774404), (3, 2): (0.239033, 0.636929),
    (2, 4): (0.131411, 0.331015), (3, 3): (0.061127, 0.193565), (4, 2): (0.090846, 0.247291),
    (3, 4): (0.018092, 0.085046), (4, 3): (0.014927, 0.079935), (4, 4): (0.003201, 0.036481),
}
T9_HSI_ERR = {2: (0.002523, 0.007134), 3: (0.001259, 0.003693), 4: (0.000448, 0.001320), 5: (0.000063, 0.000190)}
T10_SCT_ERR = {
    (4, 4, 4): (0.006596, 0.024273), (4, 5, 4): (0.006553, 0.024273), (5, 4, 4): (0.006266, 0.022820),
    (5, 5, 4): (0.006224, 0.021810), (4, 4, 5): (0.002139, 0.008371), (4, 5, 5): (0.002011, 0.008371),
    (5, 4, 5): (0.001381, 0.005793), (5, 5, 5): (0.001254, 0.004543),
}
T12_LUT_ERR = {
    ("trilinear", 9): (0.359677, 5.409771), ("trilinear", 17): (0.100026, 1.987040), ("trilinear", 33): (0.025089, 0.653506),
    ("prism", 9): (0.349128, 5.409771), ("prism", 17): (0.095150, 2.343905), ("prism", 33): (0.024172, 0.826651),
    ("pyramidal", 9): (0.319163, 5.872591), ("pyramidal", 17): (0.088116, 2.909481), ("pyramidal", 33): (0.022466, 1.042665),
    ("tetrahedral", 9): (0.284339, 5.783921), ("tetrahedral", 17): (0.077870, 2.702448), ("tetrahedral", 33): (0.020253, 1.185788),
}

# Call probabilities over all 2^24 colours (Sec. 3.2.2 and 3.4.3).
P_CBRT = (0.999626, 0.999165, 0.997184)
P_ARCSIN = 0.557723
P_ARCTAN = 0.999985
