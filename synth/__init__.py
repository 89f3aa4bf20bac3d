"""Seeded synthetic workloads shaped like the paper's inputs.

This module holds no arithmetic of the decolorization or the tone map: it only
draws images (numpy PCG64 streams spawned from ``SeedSequence``) so that the
oracle, the GPU path, the tests and the benchmark all see the same pixels.

The paper's own test images (the Cadik set and color250) are not available, so
these generators stand in for them with the shapes, sizes and value
distributions of the five workloads:

1. ``gradient_rects`` - one 512x512 8-bit image: a full hue circle left to
   right, saturation rising top to bottom, value 1, overpainted by 64 random
   axis-aligned rectangles of uniform random colour.
2. ``video_frames`` - 32 frames at 1920x1080 and 32 at 3840x2160, 8-bit, i.i.d.
   pixels with hue uniform, saturation Beta(2,2), value uniform [0.05, 1].
3. ``hdr_images`` - 16 images of 4096x4096 linear RGB stored as binary16:
   log10 radiance normal(0, 1.2) clipped to [-3, 2], each channel the radiance
   times an independent factor uniform in [0.7, 1.3].
4. ``uneven_batch`` - 256 images, width and height log-uniform in [64, 4096]
   with aspect ratio in [0.5, 2], even index 8-bit (distribution 2), odd index
   binary16 (distribution 3).
5. ``serving_trace`` - Poisson arrivals, sizes log-uniform from 256x256 to
   7680x4320, 70 % 8-bit SDR and 30 % binary16 HDR.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GRADIENT_SEED = 1
VIDEO_SEED = 2
HDR_SEED = 3
UNEVEN_SEED = 4
SERVING_SEED = 5


def _map(fn, items, workers):
    """fn over items, in order; numpy releases the GIL, so threads overlap."""
    if workers <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def _rng(seed, *spawn_path):
    ss = np.random.SeedSequence(seed)
    for k in spawn_path:
        ss = ss.spawn(k + 1)[k]
    return np.random.Generator(np.random.PCG64(ss))


def hsv_to_rgb8(h_deg, s, v):
    """Hexcone HSV -> RGB in [0, 1], then 8-bit code = floor(255 x + 0.5).

    h_deg in degrees [0, 360), s and v in [0, 1]; arrays of equal shape.
    Uses the closed form of the hexcone model: channel n in {5, 3, 1} (R, G, B)
    is v - v s max(0, min(k, 4 - k, 1)) with k = (n + h / 60) mod 6.
    Returns uint8 with a trailing axis of 3.
    """
    h6 = np.mod(np.asarray(h_deg, np.float64), 360.0) / 60.0
    vs = np.asarray(v, np.float64) * np.asarray(s, np.float64)
    v = np.asarray(v, np.float64)
    out = np.empty(h6.shape + (3,), np.uint8)
    for c, n in enumerate((5.0, 3.0, 1.0)):
        k = np.mod(n + h6, 6.0)
        ramp = np.clip(np.minimum(k, 4.0 - k), 0.0, 1.0)
        x = v - vs * ramp
        out[..., c] = np.minimum(np.floor(x * 255.0 + 0.5), 255.0)
    return out


# --------------------------------------------------------------- workload 1

def gradient_rects(seed=GRADIENT_SEED, size=512, n_rects=64):
    """512x512 8-bit hue/saturation gradient plus 64 uniform-colour rectangles."""
    rng = _rng(seed)
    y, x = np.mgrid[0:size, 0:size]
    img = hsv_to_rgb8(360.0 * (x + 0.5) / size, (y + 0.5) / size, np.ones((size, size)))
    for _ in range(n_rects):
        x0, y0 = rng.integers(0, size, 2)
        w, h = rng.integers(8, 129, 2)
        colour = rng.integers(0, 256, 3).astype(np.uint8)
        img[y0:min(size, y0 + h), x0:min(size, x0 + w)] = colour
    return img


# --------------------------------------------------------------- workload 2

def sdr_pixels(rng, h, w):
    """h x w x 3 uint8: hue U[0,360), saturation Beta(2,2), value U[0.05,1].

    Beta(2,2) is drawn as the median of three uniforms (the second order
    statistic of three U(0,1) draws has exactly that law).
    """
    n = h * w
    hue = rng.random(n, dtype=np.float64) * 360.0
    u = rng.random((3, n), dtype=np.float64)
    sat = np.maximum(np.minimum(u[0], u[1]), np.minimum(np.maximum(u[0], u[1]), u[2]))
    val = 0.05 + 0.95 * rng.random(n, dtype=np.float64)
    return hsv_to_rgb8(hue, sat, val).reshape(h, w, 3)


VIDEO_SHAPES = [(1080, 1920)] * 32 + [(2160, 3840)] * 32


def video_frame(index, seed=VIDEO_SEED):
    """Frame `index` (0..63) of the 64-frame batch: 0..31 are 1080p, 32..63 2160p."""
    h, w = VIDEO_SHAPES[index]
    return sdr_pixels(_rng(seed, index), h, w)


def video_frames(seed=VIDEO_SEED, count=64, workers=1):
    return _map(lambda i: video_frame(i, seed), range(count), workers)


# --------------------------------------------------------------- workload 3

def hdr_pixels(rng, h, w, exact=False):
    """h x w x 3 float16 linear radiance: log10 Y ~ N(0, 1.2) clipped to
    [-3, 2]; each channel Y * U[0.7, 1.3]; rounded to nearest binary16. With
    exact=True the same draws are returned unrounded, as float64 (the radiance
    the binary16 image stores)."""
    n = h * w
    log_y = np.clip(rng.normal(0.0, 1.2, n), -3.0, 2.0)
    y = np.power(10.0, log_y)
    jitter = 0.7 + 0.6 * rng.random((n, 3), dtype=np.float64)
    rad = (y[:, None] * jitter).reshape(h, w, 3)
    return rad if exact else rad.astype(np.float16)


HDR_SHAPE = (4096, 4096)


def hdr_image(index, seed=HDR_SEED, shape=HDR_SHAPE, exact=False):
    h, w = shape
    return hdr_pixels(_rng(seed, index), h, w, exact)


def hdr_images(seed=HDR_SEED, count=16, shape=HDR_SHAPE, workers=1):
    return _map(lambda i: hdr_image(i, seed, shape), range(count), workers)


# --------------------------------------------------------------- workload 4

def uneven_shapes(seed=UNEVEN_SEED, count=256, lo=64, hi=4096):
    """(h, w) pairs, each side log-uniform in [lo, hi], aspect w/h in [0.5, 2]."""
    rng = _rng(seed, 0)
    shapes = []
    while len(shapes) < count:
        w, h = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), 2))).astype(int)
        if 0.5 <= w / h <= 2.0:
            shapes.append((int(h), int(w)))
    return shapes


def uneven_image(i, shape, seed=UNEVEN_SEED):
    """Image i of the uneven batch: even index 8-bit SDR, odd index binary16 HDR."""
    h, w = shape
    rng = _rng(seed, 1, i)
    return sdr_pixels(rng, h, w) if i % 2 == 0 else hdr_pixels(rng, h, w)


def uneven_batch(seed=UNEVEN_SEED, count=256, lo=64, hi=4096, workers=1):
    """List of images: even index 8-bit SDR, odd index binary16 HDR."""
    shapes = uneven_shapes(seed, count, lo, hi)
    return _map(lambda i: uneven_image(i, shapes[i], seed), range(count), workers)


# --------------------------------------------------------------- workload 5

def serving_trace(n_requests=10000, rate_per_s=1000.0, seed=SERVING_SEED,
                  w_range=(256, 7680), h_range=(256, 4320), hdr_fraction=0.3):
    """Request list: dicts with arrival time (s), h, w and format ('u8'/'f16').

    Inter-arrival times are exponential with the given rate; width and height
    are independently log-uniform over their ranges.
    """
    rng = _rng(seed, 0)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    ws = np.rint(np.exp(rng.uniform(np.log(w_range[0]), np.log(w_range[1]), n_requests)))
    hs = np.rint(np.exp(rng.uniform(np.log(h_range[0]), np.log(h_range[1]), n_requests)))
    fmt = np.where(rng.random(n_requests) < hdr_fraction, "f16", "u8")
    return [{"id": i, "arrival": float(arrivals[i]), "h": int(hs[i]), "w": int(ws[i]),
             "fmt": str(fmt[i])} for i in range(n_requests)]


# ------------------------------------------------------------- test images

def all_colours_image():
    """4096x4096 uint8 image holding every 24-bit colour exactly once: pixel p
    (row-major) has R = p >> 16, G = (p >> 8) & 255, B = p & 255."""
    p = np.arange(1 << 24, dtype=np.uint32)
    img = np.empty((1 << 24, 3), np.uint8)
    img[:, 0] = p >> 16
    img[:, 1] = (p >> 8) & 255
    img[:, 2] = p & 255
    return img.reshape(4096, 4096, 3)


def random_image(seed, h, w, dtype, scale=1.0):
    """Small random test image: u8 uniform codes, float uniform [0, scale)."""
    rng = _rng(seed, 7)
    if np.dtype(dtype) == np.uint8:
        return rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    return (rng.random((h, w, 3)) * scale).astype(dtype)


def colour_ramps(n=256):
    """The three colour ramps of the weight-sweep figure (Fig. 4), as 1 x n
    8-bit images: pure green to pure red, pure blue to pure red, pure blue to
    pure green, each a straight line in code values (round half up)."""
    t = np.arange(n, dtype=np.float64) / max(1, n - 1)
    g, r, b = np.eye(3)[[1, 0, 2]] * 255.0
    out = {}
    for name, a, z in (("g_to_r", g, r), ("b_to_r", b, r), ("b_to_g", b, g)):
        px = np.floor((1.0 - t)[:, None] * a + t[:, None] * z + 0.5)
        out[name] = px.astype(np.uint8).reshape(1, n, 3)
    return out
