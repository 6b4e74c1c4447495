"""The serving form (mact_server_*): requests of mixed sizes, element types
and transforms admitted by device memory and run in overlapping batches;
every result is bitwise the plain path's, alone and in the mix."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1009_0854_amd as M
    return M


def _requests(n, seed, lo=16, hi=600):
    sizes, g = synth.uneven_sizes(n, seed, lo, hi)
    reqs = []
    for (h, w) in sizes:
        xf = int(g.integers(0, 4))  # CIELAB, HSI, SCT, CIELUV
        kind = g.random()
        if kind < 0.4:
            x = torch.from_numpy(g.integers(0, 256, (h, w, 3), dtype=np.uint8)).pin_memory()
            gamma = "bt709"
        elif kind < 0.6:
            x = torch.from_numpy(g.integers(0, 65536, (h, w, 3)).astype(np.uint16)).pin_memory()
            gamma = "bt709"
        else:
            x = torch.from_numpy(g.random((h, w, 3)).astype(np.float16)).pin_memory()
            gamma = "none"
        odt = torch.float32 if g.random() < 0.8 else torch.float16
        y = torch.empty((h, w, 3), dtype=odt).pin_memory()
        reqs.append((x, y, xf, gamma))
    return reqs


def _plain(M, x, xf, gamma, odt):
    return M.transform(x.cuda(), xform=xf, gamma=gamma, out_dtype=odt).cpu()


def test_mixed_requests_equal_plain(M):
    reqs = _requests(120, seed=6)
    srv = M.Server(arena_bytes=64 << 20, max_batch=16, compute_streams=3)
    ids = [srv.submit(x, y, xf, gm) for x, y, xf, gm in reqs]
    for i in ids:
        srv.wait(i, 60000)
    st = srv.stats()
    assert st.completed == len(reqs) and st.submitted == len(reqs)
    assert st.batches >= 1 and st.mean_batch >= 1.0
    for (x, y, xf, gm), i in zip(reqs, ids):
        assert torch.equal(y, _plain(M, x, xf, gm, y.dtype)), i
        assert srv.latency_ms(i) > 0
    srv.close()


def test_alone_equals_in_the_mix(M):
    reqs = _requests(40, seed=7)
    srv = M.Server(arena_bytes=256 << 20, max_batch=64, compute_streams=4)
    x0, y0, xf0, g0 = reqs[0]
    i = srv.submit(x0, y0, xf0, g0)
    srv.wait(i)
    alone = y0.clone()
    y0.zero_()
    ids = [srv.submit(x, y, xf, gm) for x, y, xf, gm in reqs]
    for j in ids:
        srv.wait(j)
    assert torch.equal(alone, y0)
    assert srv.stats().mean_batch > 1.0  # the mix did batch requests together
    srv.close()


def test_admission_limits(M):
    from paper_1009_0854_amd import _abi
    srv = M.Server(arena_bytes=2 << 20, max_batch=4, compute_streams=2, max_queue=3)
    big = torch.zeros((400, 400, 3), dtype=torch.uint8).pin_memory()  # 480 KB in + 1.9 MB out > 2 MiB
    out = torch.empty((400, 400, 3), dtype=torch.float32).pin_memory()
    with pytest.raises(_abi.MactError) as e:
        srv.submit(big, out)
    assert e.value.status == _abi.E_INVALID
    # requests that fit only one at a time: every accepted one completes; refusals are MACT_E_BUSY
    reqs = [(torch.full((300, 300, 3), k, dtype=torch.uint8).pin_memory(),
             torch.empty((300, 300, 3), dtype=torch.float32).pin_memory()) for k in range(12)]
    ids, busy = [], 0
    for x, y in reqs:
        try:
            ids.append((srv.submit(x, y), x, y))
        except _abi.MactError as err:
            assert err.status == _abi.E_BUSY
            busy += 1
    for i, x, y in ids:
        srv.wait(i)
        assert torch.equal(y, _plain(M, x, 0, "bt709", torch.float32))
    assert srv.stats().rejected == busy
    srv.close()


def test_concurrent_submitters_and_waiters(M):
    # four threads submit, poll and wait at once on one server: every request completes once,
    # with the plain path's bits, and the counters add up
    import threading
    reqs = _requests(96, seed=8, lo=16, hi=300)
    srv = M.Server(arena_bytes=32 << 20, max_batch=8, compute_streams=2)
    ids = [None] * len(reqs)
    errors = []

    def worker(k):
        try:
            for j in range(k, len(reqs), 4):
                x, y, xf, gm = reqs[j]
                ids[j] = srv.submit(x, y, xf, gm)
                if j % 3 == 0:
                    srv.wait(ids[j], 60000)
            for j in range(k, len(reqs), 4):
                srv.wait(ids[j], 60000)
                assert srv.poll(ids[j])
        except Exception as e:  # reported by the main thread
            errors.append(e)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    assert len(set(ids)) == len(reqs)
    st = srv.stats()
    assert st.submitted == len(reqs) and st.completed == len(reqs) and st.rejected == 0
    for (x, y, xf, gm), i in zip(reqs, ids):
        assert torch.equal(y, _plain(M, x, xf, gm, y.dtype)), i
    srv.close()


def test_destroy_drains_queued_requests(M):
    # closing right after submitting completes every request first
    reqs = _requests(24, seed=9, lo=64, hi=400)
    srv = M.Server(arena_bytes=8 << 20, max_batch=4, compute_streams=1)
    for x, y, xf, gm in reqs:
        y.zero_()
        srv.submit(x, y, xf, gm)
    srv.close()
    for x, y, xf, gm in reqs:
        assert torch.equal(y, _plain(M, x, xf, gm, y.dtype))


def test_c5_sized_requests_against_plain_and_oracle(M):
    # requests of the served workload's sizes (256 x 256 to 3840 x 2160, 8-bit or float16, all
    # three transforms) mixed with small ones: every output equals the plain path bitwise, and
    # sampled pixels of each equal the oracle to the parity bar (float inputs near a branch plane
    # may take either side)
    from tests import parity as P
    g = synth.rng(60)
    shapes = [(2160, 3840, "u8", 0), (2160, 3840, "f16", 2), (256, 256, "u8", 1), (1080, 1920, "f16", 0),
              (1500, 2000, "u8", 2), (720, 1280, "f16", 1), (31, 45, "u8", 0), (64, 17, "f16", 2), (300, 257, "u8", 1)]
    reqs = []
    for h, w, kind, xf in shapes:
        if kind == "u8":
            x = torch.from_numpy(g.integers(0, 256, (h, w, 3), dtype=np.uint8)).pin_memory()
            gm = "bt709"
        else:
            x = torch.from_numpy(g.random((h, w, 3)).astype(np.float16)).pin_memory()
            gm = "none"
        reqs.append((x, torch.empty((h, w, 3), dtype=torch.float32).pin_memory(), xf, gm))
    srv = M.Server(arena_bytes=1 << 30, max_batch=64, compute_streams=2)
    ids = [srv.submit(x, y, xf, gm) for x, y, xf, gm in reqs]
    for i in ids:
        srv.wait(i, 120000)
    srv.close()
    for (x, y, xf, gm), i in zip(reqs, ids):
        assert torch.equal(y, _plain(M, x, xf, gm, torch.float32)), i
        flat = x.reshape(-1, 3)
        k = g.integers(0, flat.shape[0], min(20000, flat.shape[0]))
        xv = flat[torch.from_numpy(k)].double().numpy()
        if x.dtype == torch.uint8:
            xv = xv / 255.0
        got = y.reshape(-1, 3)[torch.from_numpy(k)].double().numpy()
        P.assert_parity_ties(xf, got, xv, P.coeffs(M.default_params(xf)), gamma=gm,
                             what="request %d %s %s" % (i, tuple(x.shape), x.dtype))


def test_failed_request_reports_its_status(M):
    # a request whose descriptors are rejected when its batch is built (forced from the host with
    # the configuration's fault-injection field) completes at once with MACT_E_INVALID: wait and
    # poll report it, instead of a completion with the output unwritten or a time-out; the other
    # requests of the same batches complete with the plain path's bits
    import time
    from paper_1009_0854_amd import _abi
    reqs = _requests(8, seed=11, lo=16, hi=200)
    srv = M.Server(arena_bytes=64 << 20, max_batch=4, compute_streams=1, fail_request=3)
    ids = [srv.submit(x, y, xf, gm) for x, y, xf, gm in reqs]
    assert ids[2] == 3
    for (x, y, xf, gm), i in zip(reqs, ids):
        if i == 3:
            t0 = time.perf_counter()
            with pytest.raises(_abi.MactError) as e:
                srv.wait(i, 60000)
            assert e.value.status == _abi.E_INVALID and time.perf_counter() - t0 < 30.0
            assert "rejected" in str(e.value)
            with pytest.raises(_abi.MactError) as e:
                srv.poll(i)
            assert e.value.status == _abi.E_INVALID
            with pytest.raises(_abi.MactError):
                srv.latency_ms(i)
            continue
        srv.wait(i, 60000)
        assert srv.poll(i)
        assert torch.equal(y, _plain(M, x, xf, gm, y.dtype)), i
    st = srv.stats()
    assert st.failed == 1 and st.completed == len(reqs) - 1 and st.submitted == len(reqs)
    srv.close()


def test_cancel_before_admission(M):
    # the arena holds one 3840 x 2160 float16 request at a time: a second one waits for admission
    # while the first is copied in, transformed and copied back (milliseconds), and is withdrawn
    # there; it completes with MACT_E_CANCELLED and its output buffer is never written.  A request
    # already admitted cannot be withdrawn.  Later requests run as usual.
    from paper_1009_0854_amd import _abi as A
    h, w = 2160, 3840
    g = synth.rng(71)
    need = (h * w * 6 + 255) // 256 * 256 + (h * w * 12 + 255) // 256 * 256
    srv = M.Server(arena_bytes=need + (1 << 20), max_batch=8, compute_streams=2)
    xs = [torch.from_numpy(g.random((h, w, 3)).astype(np.float16)).pin_memory() for _ in range(3)]
    ys = [torch.full((h, w, 3), -7.0, dtype=torch.float32).pin_memory() for _ in range(3)]
    a = srv.submit(xs[0], ys[0], "lab", "none")
    b = srv.submit(xs[1], ys[1], "hsi", "none")
    assert srv.cancel(b)
    with pytest.raises(M.MactError) as e:
        srv.wait(b, 60000)
    assert e.value.status == A.E_CANCELLED
    srv.wait(a, 60000)
    assert not srv.cancel(a)  # completed: admitted long ago
    c = srv.submit(xs[2], ys[2], "sct", "none")
    srv.wait(c, 60000)
    st = srv.stats()
    assert st.cancelled == 1 and st.completed >= 2
    srv.close()
    assert torch.equal(ys[1], torch.full((h, w, 3), -7.0))
    for x, y, xf in ((xs[0], ys[0], "lab"), (xs[2], ys[2], "sct")):
        ref = M.transform(x.cuda(), xform=xf, gamma="none").cpu()
        assert torch.equal(y, ref)
    srv2 = M.Server(arena_bytes=1 << 24, max_batch=4, compute_streams=1)
    assert M.lib().mact_server_cancel(srv2._h, 12345) == A.E_INVALID
    srv2.close()
