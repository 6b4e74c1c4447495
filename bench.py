"""Benchmark of the MACT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms all|none]

Workload (the headline): RGB->CIELAB by MACT (default (4,4) minimax rational
cube root) over a batch of 64 synthetic 1920x1080 8-bit images (smooth random
low-frequency gradients plus Gaussian noise sigma 8, seeds 1000..1063), packed
HWC uint8 in, packed HWC float32 out, inputs resident in HBM.  One step = one
mact_transform over the whole batch.  `value` is Mpixel/s over the K timed
steps.  The JSON line also carries the roofline of that kernel (15 algorithmic
bytes per pixel, timed with HIP events on the launch stream), the oracle timed
on a bounded sample on the host (cpu_baseline), the accuracy against the exact
transform, and (with --forms all) the other transforms, the LUT
interpolators, the batched and the served forms.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_IMG, H, W = 64, 1080, 1920
BYTES_PER_PX = {"u8_to_f32": 15}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_batch(n=N_IMG):
    import synth
    return synth.smooth_batch_u8(n, H, W, 1000)


def time_kernel(fn, steps, warmup):
    """Average duration (ms) of fn() over `steps` launches, HIP events around
    each launch on torch's current stream (the stream the library launches on)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in ev]
    return float(np.mean(per)), float(np.median(per)), wall


def cpu_baseline(batch_np, gpu_out_sample_fn, budget_px=1 << 21):
    """The oracle (FP64 numpy) timed on a bounded sample of the workload: the
    first `budget_px` pixels of the batch, single thread."""
    from threadpoolctl import threadpool_limits
    from oracle import colour, mact
    import paper_1009_0854_amd as M
    p = M.default_params(0)
    pc = np.float32(p.f[0].p_list).astype(np.float64)
    qc = np.float32(p.f[0].q_list).astype(np.float64)
    flat = batch_np.reshape(-1, 3)[:budget_px]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ref = mact.mact_lab(flat / 255.0, pc, qc)
        dt = time.perf_counter() - t0
        exact = colour.rgb_to_lab(flat / 255.0)
    gpu = gpu_out_sample_fn(len(flat))
    de_gpu = colour.delta_e(gpu, exact)
    de_orc = colour.delta_e(ref, exact)
    return {
        "value": len(flat) / dt / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
        "sample": "first %d pixels of the 64x1080p batch, FP64 numpy MACT CIELAB, 1 thread" % len(flat),
        "seconds": dt,
    }, {"sample_px": len(flat), "gpu_max_dE": float(de_gpu.max()), "gpu_mean_dE": float(de_gpu.mean()),
        "oracle_max_dE": float(de_orc.max()), "max_abs_gpu_minus_oracle": float(np.abs(gpu - ref).max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="all", choices=["all", "none"])
    ap.add_argument("--cpu-px", type=int, default=1 << 21)
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: this build measures one GPU only (the transform has no cross-GPU step); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1009_0854_amd as M

    log("bench: generating %d x %dx%d synthetic images" % (N_IMG, W, H))
    batch_np = make_batch()
    x = torch.from_numpy(batch_np).cuda()
    y = torch.empty((N_IMG, H, W, 3), dtype=torch.float32, device="cuda")
    n_px = N_IMG * H * W
    p_lab = M.default_params(0)

    def step():
        M.transform(x, params=p_lab, out=y)

    log("bench: timing CIELAB, %d warmup + %d steps" % (a.warmup, a.steps))
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / a.steps * 1e3
    value = n_px * a.steps / wall / 1e6

    k_ms, k_med, _ = time_kernel(step, a.steps, 2)
    achieved = BYTES_PER_PX["u8_to_f32"] * n_px / (k_ms * 1e-3) / 1e9

    traffic = None
    tfile = os.path.join(ROOT, "profiles", "lab_u8_64x1080p_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            traffic = json.load(f).get("bytes_per_launch")

    extra = {}
    # practical ceilings of the access pattern
    def copy_pat():
        M.stream_u8_to_f32(x, y, n_px)
    c_ms, _, _ = time_kernel(copy_pat, a.steps, 2)
    extra["stream_u8_to_f32_GBs"] = BYTES_PER_PX["u8_to_f32"] * n_px / (c_ms * 1e-3) / 1e9
    nb = (n_px * 12) // 16 * 16
    src16 = y.view(-1)[: nb // 4]
    dst16 = torch.empty_like(src16)
    def copy16():
        M.copy(src16, dst16, nb)
    cc_ms, _, _ = time_kernel(copy16, a.steps, 2)
    extra["copy16_GBs"] = 2 * nb / (cc_ms * 1e-3) / 1e9

    if a.forms == "all":
        for name, xf in (("hsi", 1), ("sct", 2)):
            p = M.default_params(xf)
            ms, _, _ = time_kernel(lambda: M.transform(x, params=p, out=y), a.steps, 2)
            extra[name + "_Mpx_s"] = n_px / (ms * 1e-3) / 1e6
            extra[name + "_GBs"] = 15 * n_px / (ms * 1e-3) / 1e9
        M.transform(x, params=p_lab, out=y)
        torch.cuda.synchronize()

    log("bench: cpu baseline (oracle)")
    def gpu_sample(k):
        return y.reshape(-1, 3)[:k].double().cpu().numpy()
    cpu, acc = cpu_baseline(batch_np, gpu_sample, a.cpu_px)

    gold = os.path.join(ROOT, "tests", "golden", "mact_accuracy.json")
    if os.path.exists(gold):
        with open(gold) as f:
            acc["exhaustive_cube"] = json.load(f)

    line = {
        "metric": "Mpixel/s RGB->CIELAB (MACT) at stated max dE*ab; % HBM peak; served p50/p99",
        "value": value, "unit": "Mpixel/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "RGB->CIELAB MACT (4,4) rational, 64 x 1920x1080 uint8 HWC -> float32 HWC",
                   "images": N_IMG, "height": H, "width": W, "pixels_per_step": n_px},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_u8_hwc<5,LAB>", "kernel_ms": k_ms, "kernel_ms_median": k_med,
                     "algorithmic_bytes_per_px": 15},
        "cpu_baseline": cpu,
        "accuracy": acc,
        "forms": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
