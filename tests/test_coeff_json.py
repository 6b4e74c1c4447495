"""Coefficient sets persisted as JSON (approx_to_dict / save_approx /
load_approx): every field of a fitted, a printed and a default approximation
survives the round trip bit for bit, and malformed entries are refused.  CPU
only (host calls of the library)."""
import ctypes
import json

import pytest


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    M.lib()
    return M


def test_round_trip_is_exact(M, tmp_path):
    from paper_1009_0854_amd import _abi as A
    sets = {"fit_cbrt_33": M.fit(A.FN_CBRT, 3, 3, 0.008856, 1.0), "paper_cbrt_44": M.paper_approx(A.FN_CBRT, 4, 4),
            "default_atan": M.default_approx(A.FN_ATAN), "default_dec709": M.default_approx(A.FN_DEC709)}
    path = tmp_path / "coeffs.json"
    M.save_approx(str(path), sets)
    back = M.load_approx(str(path))
    assert sorted(back) == sorted(sets)
    for k, a in sets.items():
        assert bytes(memoryview(back[k])) == bytes(memoryview(a)), k
    d = json.loads(path.read_text())
    assert d["fit_cbrt_33"]["function"] == "cbrt" and d["fit_cbrt_33"]["interval"] == [0.008856, 1.0]
    assert len(d["fit_cbrt_33"]["alternation"]) == 3 + 3 + 2  # n + m + 2 points of a levelled rational
    # params built from the loaded set equal those built from the original
    p1, p2 = M.make_params("lab", [sets["fit_cbrt_33"]]), M.make_params("lab", [back["fit_cbrt_33"]])
    assert bytes(memoryview(p1)) == bytes(memoryview(p2))


def test_malformed_entries_are_refused(M):
    from paper_1009_0854_amd import _abi as A
    d = M.approx_to_dict(M.paper_approx(A.FN_CBRT, 2, 2))
    bad = dict(d, p=d["p"][:-1])
    with pytest.raises(ValueError):
        M.approx_from_dict(bad)
    with pytest.raises(ValueError):
        M.approx_from_dict(dict(d, n=9))
    with pytest.raises(ValueError):
        M.approx_from_dict(dict(d, alternation=[0.0] * 19))
