"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  Nothing in here computes any part of a colour transform: it only
makes pixels, image sizes and request streams.

Workloads (all from numpy's PCG64 with the stated seeds):
  * ``uniform_u8``: 8-bit RGB, each channel i.i.d. uniform on 0..255.
  * ``cube_u8``: all 2^24 8-bit colours as one 4096 x 4096 image, pixel p
    holding (p >> 16, (p >> 8) & 255, p & 255).  It has the colour set of the
    paper's RGB16Million test image (every 24-bit colour once), in a fixed
    order of our own.
  * ``smooth_u8``: smooth random low-frequency images: per channel
    127.5 + sum of four plane waves A cos(2 pi (u x/W + v y/H) + phi) with
    A ~ U(20, 60), u, v ~ U(0, 3) cycles per image, phi ~ U(0, 2 pi), plus a
    linear ramp 60 (g_x x/W + g_y y/H) with g ~ U(-1, 1), plus N(0, 8^2)
    noise, rounded and clipped to 0..255.
  * ``uniform_f32``: float32 values i.i.d. uniform on [0, 1).
  * ``uneven_sizes``: image sizes with width and height log-uniform in a
    range.
  * ``poisson_requests``: an arrival process with exponential gaps.
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_u8(h, w, seed=1):
    return rng(seed).integers(0, 256, size=(h, w, 3), dtype=np.uint8)


def cube_u8():
    p = np.arange(1 << 24, dtype=np.uint32)
    img = np.empty((1 << 24, 3), dtype=np.uint8)
    img[:, 0] = (p >> 16) & 255
    img[:, 1] = (p >> 8) & 255
    img[:, 2] = p & 255
    return img.reshape(4096, 4096, 3)


def cube_slice(start, count):
    """Pixels start .. start+count-1 of the cube, as an (count, 3) uint8 array."""
    p = np.arange(start, start + count, dtype=np.uint32)
    return np.stack([(p >> 16) & 255, (p >> 8) & 255, p & 255], axis=-1).astype(np.uint8)


def smooth_f32(h, w, seed):
    """The smooth image before noise and rounding, float32 on the 0..255 scale."""
    g = rng(seed)
    x = (np.arange(w, dtype=np.float64) / w)
    y = (np.arange(h, dtype=np.float64) / h)
    out = np.empty((h, w, 3), dtype=np.float32)
    for c in range(3):
        A = g.uniform(20.0, 60.0, 4)
        u = g.uniform(0.0, 3.0, 4)
        v = g.uniform(0.0, 3.0, 4)
        phi = g.uniform(0.0, 2.0 * np.pi, 4)
        gx, gy = g.uniform(-1.0, 1.0, 2)
        # cos(a + b) = cos a cos b - sin a sin b keeps each wave a sum of outer products
        cols = [np.full(w, 1.0), 60.0 * gx * x]
        rows = [127.5 + 60.0 * gy * y, np.full(h, 1.0)]
        for k in range(4):
            a = 2.0 * np.pi * u[k] * x + phi[k]
            b = 2.0 * np.pi * v[k] * y
            cols += [A[k] * np.cos(a), -A[k] * np.sin(a)]
            rows += [np.cos(b), np.sin(b)]
        out[..., c] = (np.stack(rows, 1).astype(np.float32) @ np.stack(cols, 0).astype(np.float32))
    return out, g


def smooth_u8(h, w, seed):
    base, g = smooth_f32(h, w, seed)
    noise = g.standard_normal(size=base.shape, dtype=np.float32)
    noise *= np.float32(8.0)
    base += noise
    np.rint(base, out=base)
    np.clip(base, 0, 255, out=base)
    return base.astype(np.uint8)


def smooth_batch_u8(n, h, w, seed0, threads=8):
    """n smooth images with seeds seed0 .. seed0 + n - 1, generated on threads."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty((n, h, w, 3), dtype=np.uint8)

    def one(i):
        out[i] = smooth_u8(h, w, seed0 + i)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(n)))
    return out


def uniform_f32(shape, seed):
    return rng(seed).random(size=shape, dtype=np.float32)


def uneven_sizes(n, seed, lo=64, hi=4096, lo_h=None, hi_h=None):
    """n (height, width) pairs; width log-uniform in [lo, hi], height in
    [lo_h, hi_h] (default the same range), rounded to integers."""
    g = rng(seed)
    lo_h = lo if lo_h is None else lo_h
    hi_h = hi if hi_h is None else hi_h
    w = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), n))).astype(np.int64)
    h = np.rint(np.exp(g.uniform(np.log(lo_h), np.log(hi_h), n))).astype(np.int64)
    return list(zip(h.tolist(), w.tolist())), g


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds) of n requests with exponential gaps of mean 1/rate."""
    g = rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, n)), g
