"""The batched form (mact_batch_plan_*): a graph-captured launch (one
persistent launch, or equal launches of at most 2^26 pixels) over uneven
images of mixed element types, layouts and transforms gives the same bits as
one plain mact_transform per image, for every launch shape; graph replays
equal eager launches; sampled pixels match the oracle; the autotuner's cache
file round-trips."""
import numpy as np
import pytest

import synth
from tests import parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _mixed_batch(M, n, seed, lo=17, hi=700):
    """n images: sizes log-uniform in [lo, hi]; dtype/layout/transform drawn per image."""
    sizes, g = synth.uneven_sizes(n, seed, lo, hi)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    params, ins, outs, lays, gams, olays, xfs = [], [], [], [], [], [], []
    for i, (h, w) in enumerate(sizes):
        kind = int(g.integers(0, 5))
        xf = int(g.integers(0, 3))
        if kind in (0, 1):  # packed 8-bit HWC (the 4-pixel path)
            x = torch.randint(0, 256, (h, w, 3), dtype=torch.uint8, device="cuda", generator=gen)
            lay, gam = "hwc", "bt709"
        elif kind == 2:  # float16 linear HWC
            x = torch.rand((h, w, 3), device="cuda", generator=gen).half()
            lay, gam = "hwc", "none"
        elif kind == 3:  # float32 CHW, some values outside [0, 1]
            x = torch.rand((3, h, w), device="cuda", generator=gen) * 1.1 - 0.05
            lay, gam = "chw", "none"
        else:  # row-strided 8-bit view
            base = torch.randint(0, 256, (h, w + 5, 3), dtype=torch.uint8, device="cuda", generator=gen)
            x = base[:, 2:2 + w, :]
            lay, gam = "hwc", "srgb"
        out = torch.empty(x.shape, dtype=torch.float32, device="cuda")
        params.append(M.default_params(xf))
        ins.append(x)
        outs.append(out)
        lays.append(lay)
        gams.append(gam)
        olays.append(lay)
        xfs.append(xf)
    return params, ins, outs, lays, gams, olays, xfs


def _plain(M, params, ins, lays, gams):
    return [M.transform(x, params=p, layout=l, gamma=gm) for p, x, l, gm in zip(params, ins, lays, gams)]


TUNES = [None, (256, 4096, 4, 32), (1024, 16384, 4, 16), (256, 4096, 1, 32), (64, 256, 1, 8), (512, 65536, 4, 64),
         (1024, 8192, 4, 0), (256, 1024, 1, 0), (256, 4096, 4, 32, 1), (512, 2048, 4, 0, 1)]


@pytest.mark.parametrize("tune", TUNES, ids=["autotuned", "b256v4", "b1024v4", "b256v1", "b64t256", "b512big",
                                             "b1024v4full", "b256v1full", "b256v4one", "b512v4fullone"])
def test_batch_equals_plain_bitwise(M, tune):
    params, ins, outs, lays, gams, olays, _ = _mixed_batch(M, 40, seed=3)
    ref = _plain(M, params, ins, lays, gams)
    t = M.Tune(*tune) if tune else None
    plan = M.BatchPlan(params, ins, outs, lays, gams, olays, tune=t)
    for use_graph in (True, False):
        for o in outs:
            o.fill_(float("nan"))
        plan.launch(use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (i, use_graph)
    tt = plan.tune
    assert tt.block in (64, 128, 256, 512, 1024) and tt.vec in (1, 4)
    plan.close()


@pytest.mark.parametrize("tune", [None, (256, 4096, 4, 32), (256, 4096, 1, 32), (512, 2048, 4, 0)],
                         ids=["autotuned", "v4", "v1", "v4full"])
def test_batch_16bit_and_cieluv_equal_plain_bitwise(M, tune):
    # packed 16-bit HWC takes the 4-pixel path (24 bytes per lane), a row-strided 16-bit view the
    # one-pixel path; every transform incl. CIELUV, every transfer function, the minimax decoding
    g = synth.rng(91)
    sizes = [(1, 1), (3, 85), (16, 16), (37, 300), (64, 129), (200, 203), (511, 17)]
    params, ins, outs, lays, gams = [], [], [], [], []
    for i, (h, w) in enumerate(sizes):
        c = g.integers(0, 65536, (h, w + 3, 3)).astype(np.uint16)
        # torch has few 16-bit unsigned kernels on the GPU: packed copies are made on the host
        if i % 3 != 2:
            x = torch.from_numpy(np.ascontiguousarray(c[:, :w])).cuda()
        else:
            x = torch.from_numpy(c).cuda()[:, :w]
        xf = i % 4
        gm = ["bt709", "srgb", "none"][i % 3] if xf in (0, 3) else "none"
        p = M.default_params(xf, decode=(xf in (0, 3) and i % 2 == 1))
        params.append(p)
        ins.append(x)
        outs.append(torch.empty((h, w, 3), dtype=torch.float32, device="cuda"))
        lays.append("hwc")
        gams.append(gm)
    ref = _plain(M, params, ins, lays, gams)
    t = M.Tune(*tune) if tune else None
    plan = M.BatchPlan(params, ins, outs, lays, gams, lays, tune=t)
    for use_graph in (True, False):
        for o in outs:
            o.fill_(float("nan"))
        plan.launch(use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (i, use_graph)
    plan.close()


def test_graph_replays_with_eager_work_between(M):
    params, ins, outs, lays, gams, olays, _ = _mixed_batch(M, 25, seed=4)
    ref = _plain(M, params, ins, lays, gams)
    plan = M.BatchPlan(params, ins, outs, lays, gams, olays)
    side = torch.empty((300, 301, 3), dtype=torch.float32, device="cuda")
    xin = torch.randint(0, 256, (300, 301, 3), dtype=torch.uint8, device="cuda")
    for rep in range(4):
        for o in outs:
            o.zero_()
        M.transform(xin, params=M.default_params(rep % 3), out=side)  # eager work between replays
        plan.launch(use_graph=True)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (rep, i)
    plan.close()


def test_config3_uneven_1000_images_against_plain_and_oracle(M):
    # 1000 images, width and height log-uniform in 64..4096 (seed 3), 8-bit encoded or float16
    # linear inputs, a transform per image: one persistent launch vs 1000 plain launches
    sizes, g = synth.uneven_sizes(1000, 3, 64, 4096)
    gen = torch.Generator(device="cuda").manual_seed(3)
    params, ins, outs, lays, gams = [], [], [], [], []
    for (h, w) in sizes:
        if g.random() < 0.5:
            x = torch.randint(0, 256, (h, w, 3), dtype=torch.uint8, device="cuda", generator=gen)
            gams.append("bt709")
        else:
            x = torch.rand((h, w, 3), device="cuda", generator=gen).half()
            gams.append("none")
        params.append(M.default_params(int(g.integers(0, 3))))
        ins.append(x)
        outs.append(torch.empty((h, w, 3), dtype=torch.float32, device="cuda"))
        lays.append("hwc")
    plan = M.BatchPlan(params, ins, outs, lays, gams)
    plan.launch()
    torch.cuda.synchronize()
    for i in range(0, 1000, 1):
        r = M.transform(ins[i], params=params[i], gamma=gams[i])
        assert torch.equal(outs[i], r), i
    # sampled pixels of a few images against the oracle
    for i in range(0, 1000, 97):
        x = ins[i].reshape(-1, 3)
        k = g.integers(0, x.shape[0], 2000)
        xv = x[torch.from_numpy(k).cuda()].float().cpu().numpy().astype(np.float64)
        if ins[i].dtype == torch.uint8:
            xv = xv / 255.0
        gv = outs[i].reshape(-1, 3)[torch.from_numpy(k).cuda()].cpu().numpy()
        # float inputs near a branch plane must match the oracle on one of the two sides
        P.assert_parity_ties(params[i].xform, gv, xv, P.coeffs(params[i]), gamma=gams[i], what="image %d" % i)
    plan.close()


@pytest.mark.parametrize("tune", [(256, 4096, 4, 0, 0), (1024, 8192, 4, 32, 0), (256, 4096, 1, 16, 0),
                                  (1024, 8192, 4, 32, 1), (256, 4096, 4, 0, 1)],
                         ids=["full_grid", "persistent", "vec1_persistent", "persistent_one_launch",
                              "full_grid_one_launch"])
def test_split_launches_equal_plain_for_fixed_shapes(M, tune):
    # 200 large images (about 0.4 Gpx): the tile list runs as several launches of at most 2^26
    # pixels, each with the shape's grid (one workgroup per tile, or a persistent grid walking
    # its part of the list); every image equals its plain launch bitwise
    gen = torch.Generator(device="cuda").manual_seed(9)
    g = synth.rng(9)
    params, ins, outs, gams = [], [], [], []
    px = 0
    for i in range(200):
        h, w = int(g.integers(1000, 1600)), int(g.integers(1000, 1600))
        if i % 2 == 0:
            x = torch.randint(0, 256, (h, w, 3), dtype=torch.uint8, device="cuda", generator=gen)
            gams.append("bt709")
        else:
            x = torch.rand((h, w, 3), device="cuda", generator=gen).half()
            gams.append("none")
        params.append(M.default_params(i % 4))
        ins.append(x)
        outs.append(torch.empty((h, w, 3), dtype=torch.float32, device="cuda"))
        px += h * w
    assert px > 4 * (1 << 26)
    from paper_1009_0854_amd import _abi as A
    t = A.Tune()
    t.block, t.tile, t.vec, t.waves_per_cu, t.one_launch = tune
    plan = M.BatchPlan(params, ins, outs, gammas=gams, tune=t)
    for use_graph in (True, False):
        for o in outs:
            o.fill_(float("nan"))
        plan.launch(use_graph=use_graph)
        torch.cuda.synchronize()
        for i in range(200):
            r = M.transform(ins[i], params=params[i], gamma=gams[i])
            assert torch.equal(outs[i], r), (tune, use_graph, i)
    plan.close()


def test_batch_run_convenience(M):
    params, ins, outs, lays, gams, olays, _ = _mixed_batch(M, 7, seed=5)
    ref = _plain(M, params, ins, lays, gams)
    M.batch_run(params, ins, outs, lays, gams, olays, tune=M.Tune(256, 4096, 4, 32))
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)


_TUNE_CHILD = r"""
import json, sys
import torch
import paper_1009_0854_amd as M
sys.path.insert(0, %(root)r)
from tests.test_gpu_batch import _mixed_batch
params, ins, outs, lays, gams, olays, _ = _mixed_batch(M, 12, seed=21)
plan = M.BatchPlan(params, ins, outs, lays, gams, olays)
t = plan.tune
ref = [M.transform(x, params=p, layout=l, gamma=gm) for p, x, l, gm in zip(params, ins, lays, gams)]
plan.launch()
torch.cuda.synchronize()
same = all(torch.equal(o, r) for o, r in zip(outs, ref))
plan.close()
print(json.dumps({"tune": [t.block, t.tile, t.vec, t.waves_per_cu, t.one_launch], "same": same}))
"""


def test_autotune_cache_file_round_trip(tmp_path):
    # a first process tunes the batch and writes the cache file; a second process, given a file
    # whose entry for that key names another valid shape, takes that shape without tuning; its
    # outputs still equal the plain calls' (one process at a time on the GPU)
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    env = dict(os.environ, MACT_AUTOTUNE_CACHE=str(cache), PYTHONPATH=root)
    code = _TUNE_CHILD % {"root": root}

    def child():
        r = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = child()
    assert first["same"]
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    key, val = next(iter(entries.items()))
    assert val == first["tune"]
    assert key.startswith("gfx950") or "|cu" in key
    seeded = [64, 256, 1, 3, 1] if val != [64, 256, 1, 3, 1] else [128, 512, 4, 5, 0]
    cache.write_text(json.dumps({key: seeded}))
    second = child()
    assert second["tune"] == seeded and second["same"]
    # an entry in the older four-number form reads as one_launch 0
    cache.write_text('{"%s": [%d, %d, %d, %d]}' % (key, 256, 4096, 4, 7))
    third = child()
    assert third["tune"] == [256, 4096, 4, 7, 0] and third["same"]


def test_classes_by_coefficients_and_transfer_function(M):
    # 8-bit images of one transform but different coefficient sets (the library's fit, the paper's
    # printed (4,4) and (2,2) rows) and transfer functions fall into separate classes, each run with
    # its own kernel arguments; every image equals its plain call bitwise, in any interleaving
    g = torch.Generator(device="cuda").manual_seed(23)
    sets = [M.default_params("lab"), M.make_params("lab", [M.paper_approx(M.FN_CBRT, 4, 4)]),
            M.make_params("lab", [M.paper_approx(M.FN_CBRT, 2, 2)]), M.default_params("hsi")]
    params, ins, outs, gams = [], [], [], []
    for i in range(16):
        h, w = 37 + 13 * i, 301 - 7 * i
        params.append(sets[i % 4])
        ins.append(torch.randint(0, 256, (h, w, 3), dtype=torch.uint8, device="cuda", generator=g))
        outs.append(torch.empty((h, w, 3), dtype=torch.float32, device="cuda"))
        gams.append(("bt709", "srgb")[(i // 4) % 2] if i % 4 != 3 else "none")
    ref = [M.transform(x, params=p, gamma=gm) for p, x, gm in zip(params, ins, gams)]
    for tune in (None, M.Tune(256, 2048, 4, 0, 0), M.Tune(256, 4096, 4, 8, 1)):
        plan = M.BatchPlan(params, ins, outs, None, gams, tune=tune)
        for o in outs:
            o.fill_(float("nan"))
        plan.launch(use_graph=True)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (i, tune)
        plan.close()
