"""Benchmark of the MACT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms all|none]

Headline workload: RGB->CIELAB by MACT (the default (4,4) minimax rational in
place of the cube root) over a batch of 64 synthetic 1920x1080 8-bit images
(smooth random low-frequency gradients plus Gaussian noise sigma 8, clipped;
seeds 1000..1063), packed HWC uint8 in, packed HWC float32 out, inputs
resident in HBM.  One step = one mact_transform over the whole batch; `value`
is Mpixel/s over the K timed steps (wall clock, synchronised on both sides).
Before the W untimed warm-up steps (default 20) come untimed settling steps,
at least 150 of them and at least 250 ms, whatever W is: in a fresh process
the first launch loads the code object (about 11 ms) and the next few dozen
run 3-8% slower while the memory system settles.

The JSON line also carries
  roofline      the hot kernel's achieved HBM bandwidth: 15 algorithmic bytes
                per pixel (3 read, 12 written) x pixels per launch / the mean
                launch duration from HIP events around each step on the
                launch stream (a step's launches and the gaps between them);
                the same for the 32 x 4K batch;
  cpu_baseline  the oracle timed on the host: the scalar FP64 C oracle
                (MACT CIELAB, exact CIELAB, tetrahedral LUTs at 17^3 and 33^3)
                on the first pixels of the batch, on one thread and on a pool
                of up to 16 threads; median of 10 runs after 3 warm-ups;
  accuracy      Delta E*ab of the GPU output against the exact transform on that
                sample, and the oracle's exhaustive-cube figures;
  forms         (--forms all) HSI, SCT, CIELUV, float16 output, the 4K
                batch, other layouts, the inverses and the on-device error
                statistics, MACT's gain over the exact float32 transforms, the
                LUT interpolators, the backward pass, the batched form (1000
                uneven images in one graph in the autotuned shape, and single
                persistent launches, vs 1000 plain launches) and the served form
                (Poisson arrivals: p50/p99 latency and throughput vs the plain
                per-request path; a load sweep; a small-request sweep).
"""
import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_IMG, H, W = 64, 1080, 1920


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


def time_kernel(fn, steps, warmup=20, spread=None):
    """Mean and median duration (ms) of fn() over `steps` launches after
    `warmup` untimed ones, HIP events recorded around each launch on torch's
    current stream, which is the stream the library launches on.  With a dict
    `spread`, also its 10th and 90th percentiles there."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    if spread is not None:
        spread["p10"], spread["p90"] = float(np.percentile(per, 10)), float(np.percentile(per, 90))
    return float(np.mean(per)), float(np.median(per))


def settle(fn, min_steps, min_ms):
    """Untimed launches of fn() until at least `min_steps` have run and at
    least `min_ms` of wall time has passed since the first: in a fresh
    process, and on freshly allocated buffers, the first few dozen launches of
    a streaming kernel run several per cent slower while the memory system
    settles.  Returns (steps, ms)."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while True:
        for _ in range(10):
            fn()
        n += 10
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if n >= min_steps and ms >= min_ms:
            return n, ms


def _median_rate(fn, n_px, warmup=3, runs=10):
    """Median Mpixel/s of fn() over `runs` timed calls after `warmup` untimed ones."""
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    med = float(np.median(ts))
    return {"Mpx_s": n_px / med / 1e6, "median_s": med, "min_s": float(min(ts)), "max_s": float(max(ts))}


def cpu_baseline(batch_np, y, sample_px):
    """The oracle timed on the host: the scalar FP64 C oracle (oracle/cbase.c,
    gcc -O2, one pixel at a time) on the first pixels of the 64 x 1080p batch,
    for the MACT CIELAB transform (the default (4,4) rational, coefficients
    rounded to float32 as the GPU uses them; the headline's CPU counterpart),
    the exact transform, and tetrahedral LUTs of 17^3 and 33^3 nodes (built
    once, untimed); each on one thread (sample_px / 8 pixels) and on all
    threads of the pool (sample_px pixels, equal ranges per thread); 3
    warm-ups and the median of 10 runs each.  Also the GPU output's
    Delta E*ab against the oracle's exact transform, and its largest
    difference from the oracle's MACT values, on the sample."""
    from oracle import cbase, colour
    import paper_1009_0854_amd as M
    p = M.default_params(0)
    pc = np.float32(p.f[0].p_list).astype(np.float64)
    qc = np.float32(p.f[0].q_list).astype(np.float64)
    flat = np.ascontiguousarray(batch_np.reshape(-1, 3)[:sample_px])
    one = flat[: max(1, sample_px // 8)]
    n_thr = max(1, min(16, os.cpu_count() or 1))
    lut17, lut33 = cbase.lut_build_lab(17), cbase.lut_build_lab(33)
    legs = {"mact_lab": lambda v, t: cbase.lab_mact_u8(v, pc, qc, threads=t),
            "exact_lab": lambda v, t: cbase.lab_exact_u8(v, threads=t),
            "lut_tetrahedral_17": lambda v, t: cbase.lut_tetra_u8(lut17, v, threads=t),
            "lut_tetrahedral_33": lambda v, t: cbase.lut_tetra_u8(lut33, v, threads=t)}
    res = {}
    for name, fn in legs.items():
        res[name] = {"one_thread": _median_rate(lambda: fn(one, 1), len(one)),
                     "all_threads": _median_rate(lambda: fn(flat, n_thr), len(flat))}
    # accuracy of the GPU output on the sample
    gpu = y.reshape(-1, 3)[:sample_px].double().cpu().numpy()
    exact = cbase.lab_exact_u8(flat, threads=n_thr)
    ref = cbase.lab_mact_u8(flat, pc, qc, threads=n_thr)
    de = colour.delta_e(gpu, exact)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return ({"value": res["mact_lab"]["all_threads"]["Mpx_s"], "unit": "Mpixel/s", "cores": n_thr, "kind": "oracle",
             "impl": "scalar FP64 C (oracle/cbase.c, gcc -O2), ctypes calls on a thread pool",
             "nproc": os.cpu_count(), "cpu_model": model,
             "sample": "first %d pixels of the 64x1080p batch on %d threads (%d on one thread); MACT CIELAB "
                       "(4,4); 3 warm-ups, median of 10 runs" % (len(flat), n_thr, len(one)),
             "legs": res},
            {"sample_px": len(flat), "gpu_max_dE": float(de.max()), "gpu_mean_dE": float(de.mean()),
             "max_abs_gpu_minus_oracle": float(np.abs(gpu - ref).max())})


def bench_4k(M, p, steps):
    """RGB->CIELAB on 32 x 3840x2160 uint8 (i.i.d. uniform bytes from a seeded
    device generator): 265 Mpx, 3.98 GB moved per step (four launches of 8
    images)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randint(0, 256, (32, 2160, 3840, 3), dtype=torch.uint8, device="cuda", generator=g)
    y = torch.empty((32, 2160, 3840, 3), dtype=torch.float32, device="cuda")
    n_px = 32 * 2160 * 3840
    # fresh buffers settle like a fresh process: untimed steps for at least 60 steps (240 launches)
    # and 200 ms before time_kernel's own 20 warm-up steps
    s_steps, s_ms = settle(lambda: M.transform(x, params=p, out=y), 60, 200.0)
    spread = {}
    ms, med = time_kernel(lambda: M.transform(x, params=p, out=y), steps, spread=spread)
    res = {"Mpx_s": n_px / ms / 1e3, "GBs": 15.0 * n_px / ms / 1e6, "frac_of_8TBs": 15.0 * n_px / ms / 8e9,
           "ms": ms, "ms_median": med, "ms_p10": spread["p10"], "ms_p90": spread["p90"], "pixels": n_px,
           "launches_per_step": 4, "launch_ms": ms / 4, "settle_steps": s_steps, "settle_ms": s_ms,
           **batch_stats(M, x, p)}
    del x, y
    torch.cuda.empty_cache()
    return res


def bench_general(M, x, y, p, n_px, steps):
    """CIELAB on layouts other than packed HWC, float32 (15 bytes per pixel)
    and float16 output (9): the 8-bit batch as a row-padded view (rows 8
    pixels apart beyond their width; the row-strided kernel) into packed HWC,
    as CHW planes into HWC and into CHW, and packed HWC into CHW (the plane
    kernels); row-strided CHW planes into HWC and a row-padded float32 view
    into HWC, float32 out; the packed batch into output views whose rows are
    8 pixels wider (HWC float32 and float16, CHW float32); and shapes no
    4-pixel kernel takes, 64 x 1081 x 1921: odd CHW planes into CHW and HWC,
    and HWC rows of that odd width (a row-padded view) into HWC."""
    import torch
    out = {}
    n, h, w, _ = x.shape
    y16 = y.view(-1).view(torch.float16)[: n_px * 3].view(n, h, w, 3)  # float16 output in y's memory

    def rec(name, ms, bpp):
        out[name] = {"Mpx_s": n_px / ms / 1e3, "GBs": bpp * n_px / ms / 1e6, "ms": ms}

    pad = torch.empty((n, h, w + 8, 3), dtype=torch.uint8, device="cuda")
    pad[:, :, :w] = x
    view = pad[:, :, :w]
    for tag, o, bpp in (("", y, 15.0), ("_f16", y16, 9.0)):
        ms, _ = time_kernel(lambda: M.transform(view, params=p, out=o), steps)
        rec("u8_row_padded_view" + tag, ms, bpp)
    del pad, view
    chw = x.permute(0, 3, 1, 2).contiguous()
    for tag, o, bpp in (("", y, 15.0), ("_f16", y16, 9.0)):
        ochw = o.view(n, 3, h, w)
        ms, _ = time_kernel(lambda: M.transform(chw, params=p, layout="chw", out=o, out_layout="hwc"), steps)
        rec("u8_chw_to_hwc" + tag, ms, bpp)
        ms, _ = time_kernel(lambda: M.transform(chw, params=p, layout="chw", out=ochw, out_layout="chw"), steps)
        rec("u8_chw_to_chw" + tag, ms, bpp)
        ms, _ = time_kernel(lambda: M.transform(x, params=p, out=ochw, out_layout="chw"), steps)
        rec("u8_hwc_to_chw" + tag, ms, bpp)
    # row-strided CHW (each plane's rows 8 pixels apart beyond their width) into packed HWC; float32
    # HWC rows 8 pixels apart into packed HWC (24 bytes per pixel)
    cpad = torch.empty((n, 3, h, w + 8), dtype=torch.uint8, device="cuda")
    cpad[..., :w] = chw
    cview = cpad[..., :w]
    ms, _ = time_kernel(lambda: M.transform(cview, params=p, layout="chw", out=y, out_layout="hwc"), steps)
    rec("u8_chw_row_view_to_hwc", ms, 15.0)
    del cpad, cview, chw
    fpad = torch.empty((n, h, w + 8, 3), dtype=torch.float32, device="cuda")
    fpad[:, :, :w] = x.float().div_(255.0)
    fview = fpad[:, :, :w]
    ms, _ = time_kernel(lambda: M.transform(fview, params=p, out=y), steps)
    rec("f32_row_padded_view", ms, 24.0)
    del fpad, fview
    # output views: rows 8 pixels wider than the image
    big = torch.empty((n, h, w + 8, 3), dtype=torch.float32, device="cuda")
    ms, _ = time_kernel(lambda: M.transform(x, params=p, out=big[:, :, :w]), steps)
    rec("u8_to_hwc_out_view", ms, 15.0)
    big16 = big.view(-1).view(torch.float16)[: n * h * (w + 8) * 3].view(n, h, w + 8, 3)
    ms, _ = time_kernel(lambda: M.transform(x, params=p, out=big16[:, :, :w]), steps)
    rec("u8_to_hwc_out_view_f16", ms, 9.0)
    del big16
    bigc = big.view(-1)[: n * 3 * h * (w + 8)].view(n, 3, h, w + 8)
    ms, _ = time_kernel(lambda: M.transform(x, params=p, out=bigc[..., :w], out_layout="chw"), steps)
    rec("u8_to_chw_out_view", ms, 15.0)
    del bigc, big
    # odd shapes, 64 x 1081 x 1921 uniform bytes (their own pixel count; 64 images, so that the input,
    # 399 MB, does not stay in the 256 MB Infinity Cache from one step to the next)
    on, oh, ow = 64, 1081, 1921
    o_px = on * oh * ow
    g = torch.Generator(device="cuda").manual_seed(11)
    ochw = torch.randint(0, 256, (on, 3, oh, ow), dtype=torch.uint8, device="cuda", generator=g)
    oy = torch.empty(o_px * 3, dtype=torch.float32, device="cuda")
    for name, fn in (("odd_chw_to_chw", lambda: M.transform(ochw, params=p, layout="chw", out=oy.view(on, 3, oh, ow),
                                                           out_layout="chw")),
                     ("odd_chw_to_hwc", lambda: M.transform(ochw, params=p, layout="chw", out=oy.view(on, oh, ow, 3),
                                                           out_layout="hwc"))):
        ms, _ = time_kernel(fn, steps)
        out[name] = {"Mpx_s": o_px / ms / 1e3, "GBs": 15.0 * o_px / ms / 1e6, "ms": ms, "shape": [on, oh, ow]}
    del ochw
    opad = torch.randint(0, 256, (on, oh, ow + 7, 3), dtype=torch.uint8, device="cuda", generator=g)
    ms, _ = time_kernel(lambda: M.transform(opad[:, :, :ow], params=p, out=oy.view(on, oh, ow, 3)), steps)
    out["odd_hwc_rows_view"] = {"Mpx_s": o_px / ms / 1e3, "GBs": 15.0 * o_px / ms / 1e6, "ms": ms, "shape": [on, oh, ow]}
    del opad, oy
    torch.cuda.empty_cache()
    return out


def bench_inverse(M, x, y, n_px, steps):
    """Inverse MACT (L*a*b* / HSI / SCT / L*u*v* float32 -> R'G'B' float32, 24 bytes per
    pixel; CIELAB also to float16) on the forward output of the batch, and the on-device error
    statistics of each forward transform over all 2^24 8-bit colours."""
    import torch
    import synth
    out = {}
    back = torch.empty_like(y)
    for name in ("lab", "hsi", "sct", "luv"):
        M.transform(x, xform=name, out=y)
        gm = "bt709" if name in ("lab", "luv") else "none"
        ms, _ = time_kernel(lambda: M.inverse(y, xform=name, gamma=gm, out=back), steps)
        # forward then inverse MACT against the 8-bit input, on the [0, 1] scale
        rt = max(float((back[i].float() - x[i].float() / 255.0).abs().max()) for i in range(x.shape[0]))
        out["%s_inverse" % name] = {"Mpx_s": n_px / ms / 1e3, "GBs": 24.0 * n_px / ms / 1e6, "ms": ms,
                                    "round_trip_max_abs": rt}
    # CIELAB inverse to float16 R'G'B' (18 bytes per pixel)
    back16 = back.view(-1).view(torch.float16)[: n_px * 3].view(back.shape)
    M.transform(x, xform="lab", out=y)
    ms, _ = time_kernel(lambda: M.inverse(y, xform="lab", out=back16), steps)
    out["lab_inverse_f16_out"] = {"Mpx_s": n_px / ms / 1e3, "GBs": 18.0 * n_px / ms / 1e6, "ms": ms}
    del back, back16
    cube = torch.from_numpy(synth.cube_u8()).cuda()
    for name in ("lab", "hsi", "sct", "luv"):
        M.error_stats(cube, xform=name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = M.error_stats(cube, xform=name)
        dt = time.perf_counter() - t0
        out["%s_error_stats_all_colours" % name] = {"ms": dt * 1e3, "mean": st["mean"], "max": st["max"],
                                                    "max_abs": st["max_abs"]}
    return out


def bench_weighted_fits(M, x, y, n_px, steps):
    """CIELAB cube-root fits of degree (4, 4): the plain minimax, the paper's
    printed row and weighted minimax fits under the dark-end damped weight
    ((t - t0 + delta) / (1 - t0 + delta))^beta.  For each: the on-device
    Delta E*ab mean and max over all 2^24 8-bit colours, the host time of the
    fit, and the transform's rate on the batch (the same kernel)."""
    import torch
    import synth
    cube = torch.from_numpy(synth.cube_u8()).cuda()
    out = {}
    cases = [("minimax", None), ("paper_row", "paper")] + \
        [("weighted_b%.2f_d%.3f" % bd, bd) for bd in ((0.25, 0.01), (0.5, 0.01), (0.5, 0.005), (0.75, 0.02), (1.0, 0.05))]
    for name, arg in cases:
        t0 = time.perf_counter()
        if arg is None:
            ap = M.fit(M.FN_CBRT, 4, 4, 0.008856, 1.0)
        elif arg == "paper":
            ap = M.paper_approx(M.FN_CBRT, 4, 4)
        else:
            ap = M.fit(M.FN_CBRT, 4, 4, 0.008856, 1.0, weight=M.dark_end_weight(*arg))
        fit_s = time.perf_counter() - t0
        p = M.make_params("lab", [ap])
        st = M.error_stats(cube, params=p)
        ms, _ = time_kernel(lambda: M.transform(x, params=p, out=y), max(10, steps // 4))
        out[name] = {"dE_mean": st["mean"], "dE_max": st["max"], "eps": ap.eps, "fit_s": fit_s,
                     "Mpx_s": n_px / ms / 1e3}
    return out


def bench_exact_gain(M, x, y, n_px, steps):
    """MACT's gain over the exact transforms in float32 with the device's
    elementary functions (the paper's Table 11 comparison, on the GPU): the
    same batch, the same access pattern, float32 and float16 output."""
    import torch
    out = {}
    y16 = torch.empty(y.shape, dtype=torch.float16, device="cuda")
    for name, xf in (("lab", 0), ("hsi", 1), ("sct", 2), ("luv", 3)):
        p = M.default_params(xf)
        r = {}
        for tag, o in (("f32_out", y), ("f16_out", y16)):
            # two rounds, MACT and exact alternating, the faster of each kept: the kernel timed second
            # would otherwise run on a memory system the first one has settled
            m_ms = e_ms = float("inf")
            for _ in range(2):
                m_ms = min(m_ms, time_kernel(lambda: M.transform(x, params=p, out=o), steps)[0])
                e_ms = min(e_ms, time_kernel(lambda: M.transform_exact(x, xform=xf, out=o), steps)[0])
            r[tag] = {"mact_ms": m_ms, "exact_ms": e_ms, "gain": e_ms / m_ms,
                      "mact_Mpx_s": n_px / m_ms / 1e3, "exact_Mpx_s": n_px / e_ms / 1e3}
        out[name] = r
    del y16
    return out


def batch_stats(M, xin, params, gamma="bt709"):
    """Accuracy of the MACT transform over the whole input batch against the
    exact transform in float64, on the device (mact_error_stats): mean and max
    Delta E*ab for CIELAB."""
    st = M.error_stats(xin, params=params, gamma=gamma)
    return {"dE_mean_batch": st["mean"], "dE_max_batch": st["max"]}


def lut_error(xf, out, ref):
    """Deviation of a LUT's output from `ref`, the exact float32 transform of
    the same pixels (mact_transform_exact), over the whole batch, in the
    transform's own measure: CIELAB Delta E*ab; HSI's D_HSI with the hue
    difference wrapped to [0, pi]; SCT's angle errors, wrapped."""
    import torch
    o, r = out.reshape(-1, 3), ref.reshape(-1, 3)
    if xf == "lab":
        d = (o - r).square().sum(-1).sqrt()
        return {"dE_mean_batch": float(d.mean()), "dE_max_batch": float(d.max())}

    def wrap(a):
        a = a.abs().remainder(2 * math.pi)
        return torch.minimum(a, 2 * math.pi - a)

    if xf == "hsi":
        th = wrap(o[:, 0] - r[:, 0])
        v = o[:, 1].square() + r[:, 1].square() - 2 * o[:, 1] * r[:, 1] * th.cos() + (o[:, 2] - r[:, 2]).square()
        d = v.clamp_min(0).sqrt()
        return {"D_HSI_mean_batch": float(d.mean()), "D_HSI_max_batch": float(d.max())}
    da, db = wrap(o[:, 1] - r[:, 1]), wrap(o[:, 2] - r[:, 2])
    return {"dA_mean_batch": float(da.mean()), "dA_max_batch": float(da.max()),
            "dB_mean_batch": float(db.mean()), "dB_max_batch": float(db.max()),
            "dL_max_batch": float((o[:, 0] - r[:, 0]).abs().max())}


def bench_lut(M, x, y, n_px, steps):
    """Every LUT interpolator on the 8-bit batch, each rate beside its error
    against the exact float32 transform over the same batch."""
    import torch
    out = {}

    def rec(name, xf, ms, ref):
        out[name] = {"Mpx_s": n_px / ms / 1e3, "GBs": 15 * n_px / ms / 1e6, "ms": ms, **lut_error(xf, y, ref)}

    ref = M.transform_exact(x, xform="lab")
    for N in (9, 17, 33):
        L = M.lut_build("lab", N)
        for method in ("trilinear", "prism", "pyramidal", "tetrahedral"):
            ms, _ = time_kernel(lambda: M.lut_interp(L, N, "lab", method, x, out=y), steps)
            rec("lab_%s_%d" % (method, N), "lab", ms, ref)
        # the cell-major form: one pixel's corners in one contiguous run
        C = M.lut_cells_build(L, N, "lab")
        for method in ("trilinear", "prism", "pyramidal", "tetrahedral"):
            ms, _ = time_kernel(lambda: M.lut_cells_interp(C, N, "lab", method, x, out=y), steps)
            rec("lab_cells_%s_%d" % (method, N), "lab", ms, ref)
        del C
        # the caching form: per-cell node value and edge differences
        Cc = M.lut_cache_build("lab", N)
        for method in ("trilinear", "prism", "pyramidal", "tetrahedral"):
            ms, _ = time_kernel(lambda: M.lut_cache_interp(Cc, N, "lab", method, x, out=y), steps)
            rec("lab_cache_%s_%d" % (method, N), "lab", ms, ref)
        del Cc
        out["storage_bytes_lab_%d" % N] = {"packed": M.lut_bytes("lab", N), "cells": M.lut_cells_bytes("lab", N),
                                           "cache": M.lut_cache_bytes("lab", N),
                                           # the paper's caching storage: N^3 nodes x 3 x 13 values in FP64
                                           "paper_cache_fp64": N ** 3 * 3 * 13 * 8}
    for xf in ("hsi", "sct"):
        ref = M.transform_exact(x, xform=xf)
        for N in (17, 33):
            L = M.lut_build(xf, N)
            for method in ("trilinear", "prism", "pyramidal", "tetrahedral"):
                ms, _ = time_kernel(lambda: M.lut_interp(L, N, xf, method, x, out=y), steps)
                rec("%s_%s_%d" % (xf, method, N), xf, ms, ref)
            C = M.lut_cells_build(L, N, xf)
            ms, _ = time_kernel(lambda: M.lut_cells_interp(C, N, xf, "trilinear", x, out=y), steps)
            rec("%s_cells_trilinear_%d" % (xf, N), xf, ms, ref)
            del C
            Cc = M.lut_cache_build(xf, N)
            for method in ("trilinear", "tetrahedral"):
                ms, _ = time_kernel(lambda: M.lut_cache_interp(Cc, N, xf, method, x, out=y), steps)
                rec("%s_cache_%s_%d" % (xf, method, N), xf, ms, ref)
            del Cc
    del ref
    torch.cuda.synchronize()
    return out


def bench_backward(M, steps, sets=4):
    """Forward and backward of the minimax CIELAB on 32x3x512x512 float32 CHW
    (linear input).  The timed launches rotate over `sets` independent buffer
    sets (x, g, out, dx: 403 MB per set, 1.6 GB in all), so that no launch
    re-reads data an earlier launch left in the 256 MB Infinity Cache."""
    import torch
    import synth
    p = M.default_params(0)
    n_px = 32 * 512 * 512
    xs = [torch.from_numpy(synth.uniform_f32((32, 3, 512, 512), seed=4 + 10 * i)).cuda() for i in range(sets)]
    gs = [torch.randn(xs[0].shape, generator=torch.Generator(device="cuda").manual_seed(5 + 10 * i), device="cuda")
          for i in range(sets)]
    labs = [torch.empty_like(xs[0]) for _ in range(sets)]
    dxs = [torch.empty_like(xs[0]) for _ in range(sets)]
    it = {"f": 0, "b": 0}

    def fwd():
        i = it["f"] % sets
        it["f"] += 1
        M.transform(xs[i], params=p, layout="chw", gamma="none", out=labs[i])

    def bwd():
        i = it["b"] % sets
        it["b"] += 1
        M.transform_backward(xs[i], gs[i], params=p, layout="chw", grad_in=dxs[i])

    fms, _ = time_kernel(fwd, steps)
    bms, _ = time_kernel(bwd, steps)
    del xs, gs, labs, dxs
    torch.cuda.empty_cache()
    return {"shape": "32x3x512x512 float32 CHW", "buffer_sets": sets,
            "forward": {"Mpx_s": n_px / fms / 1e3, "GBs": 24 * n_px / fms / 1e6, "ms": fms},
            "backward": {"Mpx_s": n_px / bms / 1e3, "GBs": 36 * n_px / bms / 1e6, "ms": bms}}


def bench_batch(M, steps):
    """1000 images, width and height log-uniform in 64..4096 (seed 3); uint8
    encoded (p = 0.5) or float16 linear; transform drawn per image."""
    import torch
    import synth
    sizes, g = synth.uneven_sizes(1000, 3, 64, 4096)
    gen = torch.Generator(device="cuda").manual_seed(3)
    params, ins, outs, gams = [], [], [], []
    in_bytes = out_bytes = px = 0
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
        px += h * w
        in_bytes += x.numel() * x.element_size()
        out_bytes += 12 * h * w
    t0 = time.perf_counter()
    plan = M.BatchPlan(params, ins, outs, None, gams)
    plan_s = time.perf_counter() - t0
    gms, _ = time_kernel(lambda: plan.launch(use_graph=True), steps)

    def plain():
        for p, x, o, gm in zip(params, ins, outs, gams):
            M.transform(x, params=p, gamma=gm, out=o)

    pms, _ = time_kernel(plain, max(3, steps // 4), warmup=1)
    t = plan.tune
    plan.close()

    def launches_of(t):
        # the library's split: equal launches of at most 2^26 pixels of tiles, or one
        tiles = sum(-(-(h * w) // t.tile) for (h, w) in sizes)
        return 1 if t.one_launch else max(1, -(-(tiles * t.tile) // (1 << 26)))

    def shape(t):
        return {"block": t.block, "tile": t.tile, "vec": t.vec, "waves_per_cu": t.waves_per_cu,
                "one_launch": t.one_launch, "persistent": t.waves_per_cu > 0, "launches_per_graph": launches_of(t)}

    # the single persistent launch (a grid sized to the GPU walking the whole tile list, one kernel
    # node in the graph) for a few fixed shapes, beside the tuned choice
    single = []
    for tt in ((256, 8192, 4, 16, 1), (512, 32768, 4, 32, 1), (1024, 131072, 4, 32, 1)):
        sp = M.BatchPlan(params, ins, outs, None, gams, tune=M.Tune(*tt))
        sms, _ = time_kernel(lambda: sp.launch(use_graph=True), steps)
        single.append({**shape(sp.tune), "Mpx_s": px / sms / 1e3, "GBs": (in_bytes + out_bytes) / sms / 1e6, "ms": sms})
        sp.close()
    res = {"images": 1000, "pixels": px, "bytes": in_bytes + out_bytes,
           "batched": {"Mpx_s": px / gms / 1e3, "GBs": (in_bytes + out_bytes) / gms / 1e6, "ms": gms,
                       "frac_of_8TBs": (in_bytes + out_bytes) / gms / 8e9},
           "plain_1000_launches": {"Mpx_s": px / pms / 1e3, "GBs": (in_bytes + out_bytes) / pms / 1e6, "ms": pms},
           "tune": shape(t), "single_persistent_launch": single,
           "plan_create_s": plan_s}
    del ins, outs
    torch.cuda.empty_cache()
    return res


def _requests(n, seed, pool, rate=2000.0, w_range=(256, 3840), h_range=(256, 2160)):
    """Request stream: exponential gaps at `rate` per second (all at time 0 for
    rate None); width and height log-uniform in w_range and h_range (default
    256..3840 by 256..2160); uint8 or float16 input (50/50); transform uniform
    over CIELAB, HSI, SCT.  Buffers cycle through `pool` pinned slots."""
    import torch
    import synth
    arr, g = synth.poisson_arrivals(n, 2000.0, seed)
    arr = np.zeros(n) if rate is None else arr * (2000.0 / rate)
    sizes, g2 = synth.uneven_sizes(n, seed + 1, w_range[0], w_range[1], h_range[0], h_range[1])
    kinds = g2.integers(0, 2, n)
    xfs = g2.integers(0, 3, n)
    # one pinned buffer pair per slot, large enough for any request of that slot
    slots = []
    for s in range(pool):
        idx = range(s, n, pool)
        mx = max(sizes[i][0] * sizes[i][1] for i in idx)
        slots.append((torch.randint(0, 256, (mx * 3,), dtype=torch.uint8).pin_memory(),
                      torch.rand((mx * 3,), dtype=torch.float32).half().pin_memory(),
                      torch.empty((mx * 3,), dtype=torch.float32).pin_memory()))
    reqs = []
    for i in range(n):
        h, w = sizes[i]
        u8, f16, out = slots[i % pool]
        x = (u8 if kinds[i] == 0 else f16)[:h * w * 3].view(h, w, 3)
        y = out[:h * w * 3].view(h, w, 3)
        reqs.append((float(arr[i]), x, y, int(xfs[i]), "bt709" if kinds[i] == 0 else "none"))
    return reqs


def _serve_stream(M, srv, rs, pool):
    """Submits rs at their arrival times (a pinned slot is reused only after
    its previous request completed) and waits for all; (arrival -> submit lag
    ms, submit -> done latency ms, wall s)."""
    ids = [None] * len(rs)
    lag = [0.0] * len(rs)
    t0 = time.perf_counter()
    for i, (ta, x, y, xf, gm) in enumerate(rs):
        if i >= pool:
            srv.wait(ids[i - pool], 120000)
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        lag[i] = (time.perf_counter() - t0 - ta) * 1e3  # arrival -> submit
        ids[i] = srv.submit(x, y, xf, gm)
    for i in ids:
        srv.wait(i, 120000)
    wall = time.perf_counter() - t0
    lib = np.array([srv.latency_ms(i) for i in ids])
    return np.array(lag), lib, wall


def _served_stats(M, srv, rs, pool, px, rate, warm):
    if warm:
        _serve_stream(M, srv, warm, pool)
    st0 = srv.stats()
    lag, lib, wall = _serve_stream(M, srv, rs, pool)
    st = srv.stats()
    lat = lag + lib
    nb = st.batches - st0.batches
    return {"requests": len(rs), "Mpx_s": px / wall / 1e6, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()), "mean_ms": float(lat.mean()),
            "p50_ms_from_submit": float(np.percentile(lib, 50)), "p99_ms_from_submit": float(np.percentile(lib, 99)),
            "p99_arrival_to_submit_ms": float(np.percentile(lag, 99)),
            "batches": nb, "mean_batch": len(rs) / max(1, nb), "compute_streams": 2,
            "device_busy_ms": st.device_busy_ms - st0.device_busy_ms, "wall_s": wall,
            "offered_req_s": rate if rate is not None else "all at t=0",
            "warmup_requests": len(warm) if warm else 0, "slots": pool}


def _plain_stats(M, rs, px):
    """The plain per-request path: one stream, copy in, transform, copy out,
    synchronise, in arrival order."""
    import torch
    lat = []
    s = torch.cuda.Stream()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for ta, x, y, xf, gm in rs:
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            xd = x.to("cuda", non_blocking=True)
            yd = M.transform(xd, xform=xf, gamma=gm)
            y.copy_(yd, non_blocking=True)
            s.synchronize()
            lat.append((time.perf_counter() - t0 - ta) * 1e3)
    wall = time.perf_counter() - t0
    lat = np.sort(np.array(lat))
    return {"requests": len(rs), "Mpx_s": px / wall / 1e6, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()), "wall_s": wall}


def bench_serve(M, n_req=2000, pool=16):
    """The served form at 2000 requests/s (the first 400 requests of the stream
    run once untimed on the same server, then the whole stream is timed)
    beside the plain per-request path; then a load sweep of the same request
    sizes (1000 requests at 4000 and 8000 requests/s and all at once, 32 pinned
    slots), which the PCIe copies bound (a request's kernel takes microseconds,
    its copies milliseconds, so a free compute slot finds one ready request and
    batches hold one); and a sweep of small requests (4000 of 32..256 pixels a
    side at 20000 and 50000 requests/s and all at once, 256 slots), where
    several inputs land while the slots are busy and join one batch."""
    reqs = _requests(n_req, 6, pool)
    px = sum(r[1].shape[0] * r[1].shape[1] for r in reqs)
    srv = M.Server(arena_bytes=8 << 30, max_batch=64, compute_streams=2, max_queue=1 << 20)
    served = _served_stats(M, srv, reqs, pool, px, 2000.0, reqs[:400])
    plain = _plain_stats(M, reqs, px)
    del reqs
    sweep = []
    for rate in (4000.0, 8000.0, None):
        rs = _requests(1000, 7, 32, rate)
        rpx = sum(r[1].shape[0] * r[1].shape[1] for r in rs)
        sweep.append({"offered_req_s": rate if rate is not None else "all at t=0",
                      "served": _served_stats(M, srv, rs, 32, rpx, rate, rs[:100]),
                      "plain_per_request": _plain_stats(M, rs, rpx)})
        del rs
    small = []
    for rate in (20000.0, 50000.0, None):
        rs = _requests(4000, 11, 256, rate, (32, 256), (32, 256))
        rpx = sum(r[1].shape[0] * r[1].shape[1] for r in rs)
        small.append({"offered_req_s": rate if rate is not None else "all at t=0", "sizes": "32..256 a side",
                      "served": _served_stats(M, srv, rs, 256, rpx, rate, rs[:400]),
                      "plain_per_request": _plain_stats(M, rs, rpx)})
        del rs
    srv.close()
    return {"served": served, "plain_per_request": plain, "load_sweep": sweep, "small_requests": small,
            "workload": "Poisson 2000 req/s, %d requests, W~logU[256,3840], H~logU[256,2160], uint8/fp16, "
                        "CIELAB/HSI/SCT; pinned host buffers; latency = arrival -> output on host" % n_req}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--forms", default="all", choices=["all", "none", "lut"],
                    help="all: every form; none: the headline and its ceilings only; lut: the headline and the LUTs")
    ap.add_argument("--cpu-px", type=int, default=1 << 23)
    ap.add_argument("--serve-requests", type=int, default=2000)
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: only one GPU is measured here: the transform is per pixel with no cross-GPU step, "
              "and the multi-GPU layout is a design note; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1009_0854_amd as M
    import synth

    log("generating %d x %dx%d synthetic images" % (N_IMG, W, H))
    batch_np = synth.smooth_batch_u8(N_IMG, H, W, 1000)
    x = torch.from_numpy(batch_np).cuda()
    y = torch.empty((N_IMG, H, W, 3), dtype=torch.float32, device="cuda")
    n_px = N_IMG * H * W
    p_lab = M.default_params(0)

    def step():
        M.transform(x, params=p_lab, out=y)

    # untimed settling (at least 150 steps and 250 ms, whatever --warmup says), then the W counted
    # warm-up steps, then the K timed ones
    settle_steps, settle_ms = settle(step, 150, 250.0)
    log("CIELAB: %d settling + %d warmup + %d timed steps" % (settle_steps, a.warmup, a.steps))
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = n_px * a.steps / wall / 1e6

    k_spread = {}
    k_ms, k_med = time_kernel(step, a.steps, spread=k_spread)
    # launches per step under the library's split (equal launches of whole images, at most 2^26 pixels)
    n_launch = -(-n_px // (1 << 26))
    per_img = -(-N_IMG // n_launch)
    launches = -(-N_IMG // per_img)
    # one launch averages step_ms / launches (the short gap between a step's launches included)
    l_ms, l_med = k_ms / launches, k_med / launches
    achieved = 15.0 * (n_px // launches) / (l_ms * 1e-3) / 1e9

    forms = {}
    c_ms, _ = time_kernel(lambda: M.stream_u8_to_f32(x, y, n_px), a.steps)
    forms["stream_u8_to_f32"] = {"GBs": 15.0 * n_px / (c_ms * 1e-3) / 1e9, "ms": c_ms,
                                 "what": "same access pattern, no arithmetic"}
    nb = n_px * 12 // 2 // 16 * 16
    yb = y.view(-1).view(torch.uint8)
    src16, dst16 = yb[:nb], yb[nb:2 * nb]
    cc_ms, _ = time_kernel(lambda: M.copy(src16, dst16, nb), a.steps)
    forms["copy16"] = {"GBs": 2.0 * nb / (cc_ms * 1e-3) / 1e9, "ms": cc_ms, "bytes_each_way": nb}

    if a.forms == "all":
        y16 = torch.empty((N_IMG, H, W, 3), dtype=torch.float16, device="cuda")
        h_ms, h_med = time_kernel(lambda: M.transform(x, params=p_lab, out=y16), a.steps)
        M.transform(x, params=p_lab, out=y)
        forms["lab_f16_out"] = {"Mpx_s": n_px / h_ms / 1e3, "GBs": 9.0 * n_px / h_ms / 1e6, "ms": h_ms,
                                "ms_median": h_med, "what": "same batch, float16 output: 9 bytes per pixel",
                                # the float16 rounding of the float32 result, per channel (L*, a*, b*)
                                "max_abs_vs_f32": [float((y16[..., c].float() - y[..., c]).abs().max()) for c in range(3)]}
        del y16
        # float16 R'G'B' in (BT.709): the exact decoding power vs its minimax polynomial
        x16 = (x.to(torch.float16) / 255.0).contiguous()
        for tag, pp in (("exact", p_lab), ("minimax", M.default_params(0, decode=True))):
            ms, _ = time_kernel(lambda: M.transform(x16, params=pp, out=y), a.steps)
            forms["lab_f16_in_decode_%s" % tag] = {"Mpx_s": n_px / ms / 1e3, "GBs": 18.0 * n_px / ms / 1e6, "ms": ms,
                                                   **batch_stats(M, x16, pp)}
        del x16
        # 16-bit codes (the 8-bit batch times 257), BT.709: exact power vs minimax decoding
        x16u = torch.from_numpy(batch_np.astype(np.uint16) * np.uint16(257)).cuda()
        for tag, pp in (("exact", p_lab), ("minimax", M.default_params(0, decode=True))):
            ms, _ = time_kernel(lambda: M.transform(x16u, params=pp, out=y), a.steps)
            forms["lab_u16_in_decode_%s" % tag] = {"Mpx_s": n_px / ms / 1e3, "GBs": 18.0 * n_px / ms / 1e6, "ms": ms,
                                                   **batch_stats(M, x16u, pp)}
        del x16u
        # float32 HWC input (BT.709-encoded values in [0, 1]): 24 B/px; the exact decoding power, the
        # minimax decoding, and linear input (no decoding)
        x32 = x.float().div_(255.0)
        for tag, pp, gm in (("decode_exact", p_lab, "bt709"), ("decode_minimax", M.default_params(0, decode=True), "bt709"),
                            ("linear", p_lab, "none")):
            ms, _ = time_kernel(lambda: M.transform(x32, params=pp, gamma=gm, out=y), a.steps)
            forms["lab_f32_hwc_in_" + tag] = {"Mpx_s": n_px / ms / 1e3, "GBs": 24.0 * n_px / ms / 1e6, "ms": ms,
                                              **batch_stats(M, x32, pp, gm)}
        del x32
        log("4K batch")
        forms["lab_32x4k"] = bench_4k(M, p_lab, a.steps)
        log("general path")
        forms["general_path"] = bench_general(M, x, y, p_lab, n_px, a.steps)
        # each rate beside its accuracy: the paper's metric (D_HSI for HSI, the inverse-SCT Delta E*ab
        # for SCT, Delta E*uv for CIELUV) over all 2^24 8-bit colours, on the device
        cube = torch.from_numpy(synth.cube_u8()).cuda()
        for name, xf in (("hsi", 1), ("sct", 2), ("luv", 3)):
            p = M.default_params(xf)
            ms, _ = time_kernel(lambda: M.transform(x, params=p, out=y), a.steps)
            st = M.error_stats(cube, params=p)
            forms[name] = {"Mpx_s": n_px / ms / 1e3, "GBs": 15.0 * n_px / ms / 1e6, "ms": ms,
                           "metric_mean_all_colours": st["mean"], "metric_max_all_colours": st["max"],
                           "max_abs_per_channel": st["max_abs"]}
        del cube
        log("inverses and on-device error statistics")
        forms["inverse"] = bench_inverse(M, x, y, n_px, a.steps)
        log("gain over the exact float32 transforms")
        forms["exact_gain"] = bench_exact_gain(M, x, y, n_px, a.steps)
        log("weighted cube-root fits")
        forms["weighted_fits"] = bench_weighted_fits(M, x, y, n_px, a.steps)
    if a.forms in ("all", "lut"):
        log("LUT interpolators")
        forms["lut"] = bench_lut(M, x, y, n_px, a.steps)
    if a.forms == "all":
        log("backward")
        forms["differentiation"] = bench_backward(M, a.steps)
        log("batched form")
        forms["batched"] = bench_batch(M, a.steps)
        log("served form")
        forms["serving"] = bench_serve(M, a.serve_requests)

    step()
    torch.cuda.synchronize()
    log("cpu baseline (oracle)")
    cpu, acc = cpu_baseline(batch_np, y, a.cpu_px)
    # the headline's Delta E*ab over the whole batch against the device's float64 exact transform
    acc["whole_batch_device_reference"] = batch_stats(M, x, p_lab)
    gold = os.path.join(ROOT, "tests", "golden", "mact_accuracy.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        acc["exhaustive_cube_oracle"] = {k: g[k] for k in ("lab", "hsi", "hsi_dH", "sct", "sct_dA", "sct_dB", "luv")
                                         if k in g}
        acc["exhaustive_cube_lut_dE"] = {k: v for k, v in g.items() if k.startswith("lut_")}

    traffic = None
    tfile = os.path.join(ROOT, "profiles", "lab_u8_64x1080p_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            t = json.load(f)
        if t.get("kernel_source_hash") == kernel_hash():
            traffic = t.get("bytes_per_launch")

    line = {
        "metric": "Mpixel/s RGB->CIELAB (MACT) at stated max dE*ab; % HBM peak; served p50/p99",
        "value": value, "unit": "Mpixel/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "RGB->CIELAB MACT, default (4,4) minimax rational; 64 x 1920x1080 uint8 HWC -> float32 HWC",
                   "images": N_IMG, "height": H, "width": W, "pixels_per_step": n_px,
                   "max_dE_exhaustive_cube": acc.get("exhaustive_cube_oracle", {}).get("lab", {}).get("max"),
                   "settle_steps": settle_steps, "settle_ms": settle_ms, "served": served_summary(forms)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_hwc4<U8,F32,4,LAB>",
                     # achieved: 15 B/px x pixels_per_launch / launch_ms.  HIP events around each
                     # step on the launch stream (step_ms); the library splits the batch into equal
                     # launches of at most 2^26 pixels (two of 32 images here), so one launch
                     # averages step_ms / launches_per_step, the gap between the launches included
                     "launch_ms": l_ms, "launch_ms_median": l_med,
                     "algorithmic_bytes_per_px": 15, "launches_per_step": launches,
                     "pixels_per_launch": n_px // launches,
                     "step_ms": k_ms, "step_ms_median": k_med, "step_ms_p10": k_spread["p10"],
                     "step_ms_p90": k_spread["p90"],
                     # the same run's 16-byte copy (equal reads and writes, a grid covering the copy once):
                     # the practical ceiling of this machine's HBM for a streaming kernel
                     "copy16_GBs": forms["copy16"]["GBs"],
                     "frac_of_copy16": achieved / forms["copy16"]["GBs"],
                     # the same kernel on the 32 x 3840x2160 uint8 batch (four launches of 8 images)
                     "r_32x4k": r4k_summary(forms)},
        "cpu_baseline": cpu,
        "accuracy": acc,
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


def r4k_summary(forms):
    """The 32 x 4K leg's roofline figures (None without --forms all)."""
    r = forms.get("lab_32x4k")
    if not r:
        return None
    per = r["pixels"] // r["launches_per_step"]
    return {"frac": r["frac_of_8TBs"], "achieved": r["GBs"], "launch_ms": r["launch_ms"],
            "frac_median": 15.0 * r["pixels"] / r["ms_median"] / 8e9, "launches_per_step": r["launches_per_step"],
            "pixels_per_launch": per, "step_ms": r["ms"], "Mpx_s": r["Mpx_s"]}


def served_summary(forms):
    """The served form's latency and throughput beside the plain per-request
    path (None without --forms all)."""
    sv = forms.get("serving")
    if not sv:
        return None
    a, b = sv["served"], sv["plain_per_request"]
    out = {"p50_ms": a["p50_ms"], "p99_ms": a["p99_ms"], "Mpx_s": a["Mpx_s"], "mean_batch": a["mean_batch"],
           "plain_p50_ms": b["p50_ms"], "plain_p99_ms": b["p99_ms"], "plain_Mpx_s": b["Mpx_s"],
           "offered_req_s": a["offered_req_s"]}
    # small requests at 50000 requests/s, where batches form
    sm = [x for x in sv.get("small_requests", []) if x["offered_req_s"] == 50000.0]
    if sm:
        c, d = sm[0]["served"], sm[0]["plain_per_request"]
        out["small_50k_req_s"] = {"mean_batch": c["mean_batch"], "Mpx_s": c["Mpx_s"], "p50_ms": c["p50_ms"],
                                  "p99_ms": c["p99_ms"], "plain_Mpx_s": d["Mpx_s"], "plain_p50_ms": d["p50_ms"],
                                  "plain_p99_ms": d["p99_ms"]}
    return out


def kernel_hash():
    """Hash of the hot kernel's sources, to tell whether stored counters are
    stale: the per-pixel code and constants (pixel.h, common.h), the
    streaming stores (stream.h) and, from
    xform.hip, the hot kernel with its launch constants, grid, launcher and
    the split of a batch into launches."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1009_0854_amd", "csrc")
    h = hashlib.sha256()
    for f in ("pixel.h", "common.h", "stream.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "xform.hip")) as fh:
        src = fh.read()
    # from the launch constants to the end of k_hwc4, and the launcher template
    a = src.index("constexpr int kHotBlock")
    b = src.index("\n}\n", src.index("void k_hwc4(")) + 3
    h.update(src[a:b].encode())
    for pat in (r"static unsigned hot_grid\(.*?\n}\n", r"static void launch_hwc4\(.*?\n}\n",
                r"int64_t images_per_stream_launch\(.*?\n}\n"):
        h.update(re.search(pat, src, re.S).group(0).encode())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
