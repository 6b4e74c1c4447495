"""The allocation-free error statistics (mact_error_stats_noalloc) against
mact_error_stats, through the C ABI: two calls in a row on one GPU, the second
on a smaller input, each equal to the allocating form's result."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _same(a, b):
    # count and maxima are exact (integer count; the maxima are atomic maxima of the same
    # per-pixel float64 values); the mean is a float64 sum whose atomic additions may come in
    # another order: equal to float64 rounding of the sum
    assert a["count"] == b["count"]
    assert a["max"] == b["max"]
    assert a["max_abs"] == b["max_abs"]
    assert a["mean"] == pytest.approx(b["mean"], rel=1e-12, abs=0.0)


@pytest.mark.parametrize("xform", ["lab", "hsi", "sct", "luv"])
def test_noalloc_equals_the_allocating_form_on_two_calls(M, xform):
    big = torch.from_numpy(synth.smooth_batch_u8(2, 480, 640, 11)).cuda()
    small = torch.from_numpy(synth.uniform_u8(13, 29, seed=5)).cuda()
    p = M.default_params(xform)
    first = M.error_stats_noalloc(big, params=p)
    _same(first, M.error_stats(big, params=p))
    second = M.error_stats_noalloc(small, params=p)
    _same(second, M.error_stats(small, params=p))
    assert second["count"] == 13 * 29 and first["count"] == 2 * 480 * 640
    # the second call starts from a cleared record: nothing of the first call's sums is left
    assert second["mean"] != first["mean"]


def test_noalloc_float_input_and_repeat(M):
    # float32 linear input (no decoding), then the same call again: the same record each time
    x = torch.rand(3, 64, 96, 3, generator=torch.Generator().manual_seed(3)).cuda()
    p = M.default_params("lab")
    ref = M.error_stats(x, params=p, gamma="none")
    for _ in range(2):
        _same(M.error_stats_noalloc(x, params=p, gamma="none"), ref)
    y = x[:1, :7, :5].contiguous()
    _same(M.error_stats_noalloc(y, params=p, gamma="none"), M.error_stats(y, params=p, gamma="none"))


def test_noalloc_validation_is_the_allocating_forms(M):
    from paper_1009_0854_amd import _abi as A
    p = M.default_params("lab")
    p.out_mode = 1
    x = torch.zeros(4, 4, 3, dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MactError) as e:
        M.error_stats_noalloc(x, params=p)
    assert e.value.status == A.E_INVALID
    assert M.error_stats_noalloc(x[:0])["count"] == 0
