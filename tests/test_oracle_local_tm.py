"""Pins of the oracle's local tone map (Sec. III-B.2: smoothed local histogram
equalisation; the reading is stated in the oracle's header). Each test checks
it against something other than its own code path:

- a constant image has the closed form T_l = 1/2 + f/2 - 3 f^2/2 + f^3 (f the
  fractional bin position): the cumulative distribution at u of masses 1 - f
  and f at the two bin centres around u, each spread by the unit triangle;
- strength 0 reduces to the global tone map (separately pinned);
- one tile: the curve is the whole image's triangle-smoothed cumulative
  distribution, computed here by brute force over pixel pairs;
- mirror and transpose symmetry on tile-aligned images (catches swapped axes,
  wrong tile centres or off-by-one interpolation);
- range, monotonicity of the one-tile curve, and the pure-Python twin.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ref as twin

TM = dict(eps=1e-4, contrast=2.0, sigma_floor=1e-3)


def _u(lhat, eps=1e-4):
    return np.clip(2.0 * np.log2((lhat + eps) / eps) - 0.5, 0.0, 63.0)


def _ramp(x):
    return np.where(x <= -1, 0.0, np.where(x <= 0, 0.5 * (1 + x) ** 2,
                                           np.where(x <= 1, 1 - 0.5 * (1 - x) ** 2, 1.0)))


@pytest.mark.parametrize("code", [0, 1, 37, 100, 200, 255])
@pytest.mark.parametrize("shape", [(5, 7), (70, 150), (128, 64)])
def test_constant_image_closed_form(oracle_mod, code, shape):
    img = np.full(shape + (3,), code, np.uint8)
    t, _ = oracle_mod.tonemap_local(img, strength=1.0, **TM)
    u = float(_u(np.array(code / 255.0)))
    k = min(math.floor(u), 62)
    f = u - k
    want = 0.5 + f / 2 - 1.5 * f * f + f ** 3
    np.testing.assert_allclose(t, want, rtol=0, atol=1e-13)
    half, _ = oracle_mod.tonemap_local(img, strength=0.5, **TM)
    # the global half is the global tone map's T (1/2 up to the FP64 rounding of
    # the flat image's mean, amplified by c / sigma_floor)
    tg = oracle_mod.tonemap(img, **TM)[0]
    assert np.max(np.abs(tg - 0.5)) < 1e-8
    np.testing.assert_allclose(half, 0.5 * tg + 0.5 * want, rtol=0, atol=1e-13)


def test_zero_strength_is_global(oracle_mod):
    img = synth.hdr_pixels(np.random.default_rng(41), 90, 130)
    t, st = oracle_mod.tonemap_local(img, strength=0.0, **TM)
    tg, _, st_g = oracle_mod.tonemap(img, **TM)
    np.testing.assert_array_equal(t, tg)
    assert st == st_g


@pytest.mark.parametrize("shape", [(1, 1), (3, 50), (64, 64), (40, 17)])
def test_single_tile_is_smoothed_global_cdf(oracle_mod, shape):
    img = synth.sdr_pixels(np.random.default_rng(42), *shape)
    t, _ = oracle_mod.tonemap_local(img, strength=1.0, **TM)
    u = _u(oracle_mod.decolorize(img)).ravel()
    k = np.minimum(np.floor(u), 62)
    f = u - k
    # each pixel q: mass 1 - f at k_q, f at k_q + 1; CDF at u_p, brute force
    want = ((1 - f)[None, :] * _ramp(u[:, None] - k[None, :]) +
            f[None, :] * _ramp(u[:, None] - k[None, :] - 1)).sum(axis=1) / u.size
    np.testing.assert_allclose(t.ravel(), want, rtol=0, atol=1e-12)


def test_single_tile_curve_is_monotone(oracle_mod):
    img = synth.hdr_pixels(np.random.default_rng(43), 50, 60)
    t, _ = oracle_mod.tonemap_local(img, strength=1.0, **TM)
    u = _u(oracle_mod.decolorize(img)).ravel()
    order = np.argsort(u, kind="stable")
    assert np.all(np.diff(t.ravel()[order]) >= -1e-15)
    assert t.min() >= 0.0 and t.max() <= 1.0


@pytest.mark.parametrize("kind", ["u8", "f16"])
def test_mirror_and_transpose_symmetry(oracle_mod, kind):
    rng = np.random.default_rng(44)
    img = synth.sdr_pixels(rng, 128, 192) if kind == "u8" else synth.hdr_pixels(rng, 128, 192)
    t, _ = oracle_mod.tonemap_local(img, strength=1.0, **TM)
    np.testing.assert_allclose(oracle_mod.tonemap_local(img[:, ::-1], strength=1.0, **TM)[0],
                               t[:, ::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle_mod.tonemap_local(img[::-1], strength=1.0, **TM)[0],
                               t[::-1], rtol=0, atol=1e-12)
    sq = np.ascontiguousarray(img[:, :128])
    ts, _ = oracle_mod.tonemap_local(sq, strength=1.0, **TM)
    tt, _ = oracle_mod.tonemap_local(np.ascontiguousarray(sq.transpose(1, 0, 2)), strength=1.0,
                                     **TM)
    np.testing.assert_allclose(tt, ts.T, rtol=0, atol=1e-12)


def test_dark_tiles_brighten_bright_tiles_darken(oracle_mod):
    """Local equalisation: the same mid-grey pixel maps higher in a dark
    surround than in a bright one."""
    img = np.full((64, 512, 3), 20, np.uint8)
    img[:, 256:] = 235
    img[32, 40] = img[32, 424] = 120  # both two tiles away from the boundary
    t, _ = oracle_mod.tonemap_local(img, strength=1.0, **TM)
    assert t[32, 40] > 0.95 and t[32, 424] < 0.05


@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32])
def test_twin_agrees(oracle_mod, dtype):
    img = synth.random_image(45, 9, 70, dtype, scale=3.0)
    img[0, 0] = 0
    t, _ = oracle_mod.tonemap_local(img, strength=0.7, eps=1e-3, contrast=1.5, sigma_floor=1e-3)
    if dtype == np.float16:
        px, kind = img.view(np.uint16).tolist(), "f16"
    else:
        px, kind = img.astype(np.float64).tolist(), ("u8" if dtype == np.uint8 else "f32")
    want = np.array(twin.tonemap_local(px, kind, 1e-3, 1.5, 1e-3, 0.7))
    np.testing.assert_allclose(t, want, rtol=0, atol=1e-12)


def test_rejects_bad_strength(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.tonemap_local(synth.random_image(46, 2, 2, np.uint8), strength=1.5)


def test_sampled_evaluation_matches_full(oracle_mod):
    img = synth.hdr_pixels(np.random.default_rng(47), 150, 230)
    full, st = oracle_mod.tonemap_local(img, strength=0.6, nthreads=3, **TM)
    idx = np.random.default_rng(48).integers(0, full.size, 500)
    part, st2 = oracle_mod.tonemap_local(img, strength=0.6, sample=idx, **TM)
    np.testing.assert_array_equal(part, full.ravel()[idx])
    assert st == st2


def test_local_colour_output_keeps_ratios_and_luminance(oracle_mod):
    """The local map's colour output is the same re-colouring as the global
    one: at s = 1 every unclamped pixel keeps its channel ratios and has
    Eqs. (1)-(6) luminance equal to its local T (degree-1 homogeneity)."""
    img = synth.sdr_pixels(np.random.default_rng(49), 70, 90)
    rgb, t = oracle_mod.tonemap_local_colour(img, strength=0.7, saturation=1.0, **TM)
    free = rgb.max(axis=2) < 1.0
    assert free.sum() > 1000
    ys, xs = np.nonzero(free)
    for y, x in zip(ys[::37], xs[::37]):
        assert abs(oracle_mod.luminance(*rgb[y, x]) - t[y, x]) <= 1e-12
    src = img.astype(np.float64)
    np.testing.assert_allclose((rgb[..., 0] * src[..., 1])[free], (rgb[..., 1] * src[..., 0])[free],
                               rtol=1e-12, atol=1e-15)


def test_recolour_matches_global_colour(oracle_mod):
    img = synth.hdr_pixels(np.random.default_rng(50), 20, 30)
    rgb, t, lhat, _ = oracle_mod.tonemap_colour(img, saturation=0.6, **TM)
    np.testing.assert_array_equal(oracle_mod.recolour(img, lhat, t, 0.6), rgb)
