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


def test_split_of_odd_sized_images_keeps_the_coalesced_kernel(M):
    # 17 images of 3841 x 2161 (an odd pixel count, 141 Mpx): split into equal launches, the
    # launches after the first would start 3 bytes x odd off the 4-byte alignment of the 8-bit
    # kernel; the count per launch is rounded up to keep it (8, 8, 1 images).  Every image equals
    # its own call, and the batch runs at about the speed of 17 single-image calls (each of which
    # starts aligned); with the one-pixel kernel on most of the batch it ran about 2.5x slower
    n, h, w = 17, 2161, 3841
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randint(0, 256, (n, h, w, 3), dtype=torch.uint8, device="cuda", generator=g)
    y = torch.empty((n, h, w, 3), dtype=torch.float32, device="cuda")
    p = M.default_params("lab")
    M.transform(x, params=p, out=y)
    torch.cuda.synchronize()
    for i in (0, 7, 8, 15, 16):
        assert torch.equal(y[i:i + 1], M.transform(x[i:i + 1], params=p)), i

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return sorted(ts)[reps // 2]

    whole = timed(lambda: M.transform(x, params=p, out=y))
    each = timed(lambda: [M.transform(x[i:i + 1], params=p, out=y[i:i + 1]) for i in range(n)])
    assert whole < 1.5 * each, (whole, each)


def test_split_of_odd_planes_through_the_gather_kernel(M):
    # 17 CHW images of 2161 x 2161 (odd W H; 79 Mpx): no 4-pixel kernel takes them, so each
    # launch of the split goes to k_gather, into packed CHW and HWC output; every image equals
    # its own call, on both sides of the split
    n, h, w = 17, 2161, 2161
    assert n * h * w > (1 << 26)
    g = torch.Generator(device="cuda").manual_seed(23)
    x = torch.randint(0, 256, (n, 3, h, w), dtype=torch.uint8, device="cuda", generator=g)
    p = M.default_params("sct")
    for out_layout in ("chw", "hwc"):
        y = M.transform(x, params=p, layout="chw", out_layout=out_layout)
        torch.cuda.synchronize()
        for i in (0, 7, 8, 9, 16):
            one = M.transform(x[i:i + 1], params=p, layout="chw", out_layout=out_layout)
            torch.cuda.synchronize()
            assert torch.equal(y[i:i + 1], one), (out_layout, i)
        del y
