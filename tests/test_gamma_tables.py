"""The library's 8-bit decoding tables (csrc/gamma_table.inc: float32 for the
kernels, float64 for the error statistics' reference) against the oracle's
inverse transfer functions (Sec. 3.2.1 for BT.709; IEC sRGB; identity)."""
import os
import re

import numpy as np

from oracle import colour

INC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1009_0854_amd", "csrc",
                   "gamma_table.inc")


def _table(name):
    src = open(INC).read()
    body = re.search(r"%s\[3\]\[256\] = \{(.*?)\};" % name, src, re.S).group(1)
    rows = re.findall(r"\{([^{}]*)\}", body)
    assert len(rows) == 3
    return np.array([[float.fromhex(v.strip().rstrip("f")) for v in r.split(",")] for r in rows])


def _oracle_rows():
    k = np.arange(256) / 255.0
    return np.stack([colour.inverse_gamma(k, "bt709"), colour.inverse_gamma(k, "srgb"), k])


def test_float64_table_equals_the_oracle_to_rounding():
    t64, ref = _table("k_gamma_table64"), _oracle_rows()
    assert t64.shape == (3, 256)
    # both are the formula evaluated in double precision: agreement to a few units in the last place
    np.testing.assert_allclose(t64, ref, rtol=4e-16, atol=0)
    assert t64[0, 0] == 0.0 and t64[0, 255] == 1.0 and t64[2, 128] == 128 / 255.0


def test_float32_table_is_the_double_value_rounded_once():
    t32, t64 = _table("k_gamma_table"), _table("k_gamma_table64")
    assert np.array_equal(t32, t64.astype(np.float32).astype(np.float64))
    # and against the oracle: within half a float32 unit of its double value
    ref = _oracle_rows()
    assert np.all(np.abs(t32 - ref) <= np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64) / 2 + 1e-300)
