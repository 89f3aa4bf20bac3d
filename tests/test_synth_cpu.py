"""The seeded input generators against the recipes they state (the stand-ins
for the paper's image sets): colour conversion against Python's colorsys,
value and saturation laws of the SDR pixels, the HDR radiance law and channel
jitter, the shapes of the video, uneven and serving workloads, determinism,
and the exhaustive all-colours image."""
import colorsys
import math

import numpy as np
import pytest

import synth


def test_hsv_to_rgb8_matches_colorsys():
    rng = np.random.default_rng(0)
    h, s, v = rng.random(2000) * 360.0, rng.random(2000), rng.random(2000)
    got = synth.hsv_to_rgb8(h, s, v)
    for i in range(len(h)):
        want = [min(255.0, math.floor(255.0 * c + 0.5)) for c in colorsys.hsv_to_rgb(h[i] / 360.0, s[i], v[i])]
        assert np.max(np.abs(got[i].astype(int) - np.array(want, int))) <= 1, (h[i], s[i], v[i])
    prim = synth.hsv_to_rgb8(np.array([0.0, 120.0, 240.0]), np.ones(3), np.ones(3))
    assert prim.tolist() == [[255, 0, 0], [0, 255, 0], [0, 0, 255]]
    grey = synth.hsv_to_rgb8(np.array([77.0]), np.zeros(1), np.array([0.5]))
    assert grey.tolist() == [[128, 128, 128]]


def test_sdr_value_and_saturation_laws():
    img = synth.sdr_pixels(np.random.default_rng(1), 300, 300).reshape(-1, 3).astype(np.float64)
    mx, mn = img.max(axis=1), img.min(axis=1)
    v = mx / 255.0
    s = (mx - mn) / np.maximum(mx, 1.0)
    assert abs(v.mean() - 0.525) < 0.005 and abs(v.std() - 0.95 / math.sqrt(12)) < 0.005
    assert v.min() >= 0.05 - 1 / 255 and v.max() <= 1.0
    # Beta(2, 2): mean 1/2, variance 1/20 (8-bit rounding adds a little)
    assert abs(s.mean() - 0.5) < 0.01 and abs(s.var() - 0.05) < 0.005


def test_hdr_radiance_law_and_jitter():
    rad = synth.hdr_pixels(np.random.default_rng(2), 300, 300, exact=True).reshape(-1, 3)
    ratio = rad.max(axis=1) / rad.min(axis=1)
    assert ratio.max() <= 1.3 / 0.7 + 1e-12
    assert rad.min() >= 1e-3 * 0.7 and rad.max() <= 1e2 * 1.3
    # log10 of the channel mean: the clipped normal(0, 1.2) of the radiance
    # plus the log of a mean of three U[0.7, 1.3] factors (mean ~ -0.002)
    ly = np.log10(rad.mean(axis=1))
    assert abs(np.median(ly)) < 0.02
    assert ly.max() <= 2.0 + math.log10(1.3) and ly.min() >= -3.0 + math.log10(0.7)
    # share above 1.9: P(Z > 1.9 / 1.2) = 0.057 (the clip at 2 holds 0.048 of it),
    # blurred a little by the jitter
    assert abs(np.mean(ly > 1.9) - 0.057) < 0.015
    half = synth.hdr_pixels(np.random.default_rng(2), 300, 300)
    assert half.dtype == np.float16
    assert np.array_equal(half, rad.reshape(300, 300, 3).astype(np.float16))


def test_workload_shapes_and_determinism():
    assert synth.VIDEO_SHAPES[:32] == [(1080, 1920)] * 32 and synth.VIDEO_SHAPES[32:] == [(2160, 3840)] * 32
    a, b = synth.video_frame(5), synth.video_frame(5)
    assert a.shape == (1080, 1920, 3) and np.array_equal(a, b)
    assert not np.array_equal(a, synth.video_frame(6))
    shapes = synth.uneven_shapes()
    assert len(shapes) == 256 and shapes == synth.uneven_shapes()
    for h, w in shapes:
        assert 64 <= h <= 4096 and 64 <= w <= 4096 and 0.5 <= w / h <= 2.0
    img = synth.uneven_image(3, (70, 90))
    assert img.dtype == np.float16 and synth.uneven_image(2, (70, 90)).dtype == np.uint8
    g = synth.gradient_rects()
    assert g.shape == (512, 512, 3) and np.array_equal(g, synth.gradient_rects())


def test_serving_trace_recipe():
    tr = synth.serving_trace(10000, rate_per_s=2000.0)
    arr = np.array([r["arrival"] for r in tr])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0.0)
    assert abs(np.diff(arr).mean() - 1 / 2000.0) < 0.05 / 2000.0
    assert abs(np.mean([r["fmt"] == "f16" for r in tr]) - 0.3) < 0.015
    ws, hs = np.array([r["w"] for r in tr]), np.array([r["h"] for r in tr])
    assert ws.min() >= 256 and ws.max() <= 7680 and hs.min() >= 256 and hs.max() <= 4320
    # log-uniform: the log of the side is uniform, so its median is mid-range
    assert abs(np.median(np.log(ws)) - 0.5 * (math.log(256) + math.log(7680))) < 0.1


@pytest.mark.slow
def test_all_colours_image_holds_every_colour_once():
    img = synth.all_colours_image().reshape(-1, 3).astype(np.uint32)
    codes = (img[:, 0] << 16) | (img[:, 1] << 8) | img[:, 2]
    assert np.array_equal(codes, np.arange(1 << 24, dtype=np.uint32))


def test_colour_ramps_end_points():
    r = synth.colour_ramps(256)
    assert r["g_to_r"][0, 0].tolist() == [0, 255, 0] and r["g_to_r"][0, -1].tolist() == [255, 0, 0]
    assert r["b_to_r"][0, 0].tolist() == [0, 0, 255] and r["b_to_r"][0, -1].tolist() == [255, 0, 0]
    assert r["b_to_g"][0, 0].tolist() == [0, 0, 255] and r["b_to_g"][0, -1].tolist() == [0, 255, 0]
    # each channel moves monotonically along a ramp
    for img in r.values():
        d = np.diff(img[0].astype(int), axis=0)
        assert np.all((d >= 0).all(axis=0) | (d <= 0).all(axis=0))
