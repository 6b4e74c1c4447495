"""Batches above 2^26 pixels run as several equal launches (float32 outputs):
every entry point that splits gives, for such a batch, the bits of its images
transformed one call each (one launch each)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def test_split_batches_equal_per_image_calls(M):
    n, h, w = 34, 1080, 1920  # 70.5 Mpx: two launches of 17 images
    assert n * h * w > (1 << 26)
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randint(0, 256, (n, h, w, 3), dtype=torch.uint8, device="cuda", generator=g)
    lut = M.lut_build("lab", 17)
    checks = {
        "transform": lambda t: M.transform(t, xform="lab"),
        "transform_hsi": lambda t: M.transform(t, xform="hsi"),
        "exact": lambda t: M.transform_exact(t, xform="lab"),
        "lut": lambda t: M.lut_interp(lut, 17, "lab", "tetrahedral", t),
    }
    for name, fn in checks.items():
        whole = fn(x)
        torch.cuda.synchronize()
        for i in (0, 16, 17, 33):  # both sides of the split
            one = fn(x[i:i + 1])
            torch.cuda.synchronize()
            assert torch.equal(whole[i:i + 1], one), (name, i)
        del whole
    lab = M.transform(x, xform="lab")
    back = M.inverse(lab, xform="lab")
    torch.cuda.synchronize()
    for i in (0, 16, 17, 33):
        one = M.inverse(lab[i:i + 1], xform="lab")
        torch.cuda.synchronize()
        assert torch.equal(back[i:i + 1], one), ("inverse", i)
