"""Pins of the oracle's colour output of the global tone map (Sec. III-B.1 shows
colour results; the re-colouring read here is C_out = min(1, T (C / Lhat)^s)).

Each test checks the oracle against something other than its own formula: the
degree-1 homogeneity of Eqs. (1)-(6) (the luminance of an s = 1 output is T),
ratio preservation, the special cases s = 0 and grey pixels, a two-pixel image
whose T and L have closed forms, and the independent pure-Python twin.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ref as twin

C = 2.0
T_HI = 1.0 / (1.0 + math.exp(-C))  # two-pixel image, brighter pixel
T_LO = 1.0 / (1.0 + math.exp(C))


def _sdr(seed, h, w):
    return synth.sdr_pixels(np.random.default_rng(seed), h, w)


def test_unit_saturation_output_has_luminance_t(oracle_mod):
    """s = 1: L(T C / Lhat) = T L(C) / Lhat = T by homogeneity of Eqs. (1)-(6),
    wherever no channel was clamped."""
    img = _sdr(11, 9, 23)
    rgb, t, lhat, _ = oracle_mod.tonemap_colour(img, saturation=1.0)
    checked = 0
    for y in range(img.shape[0]):
        for x in range(img.shape[1]):
            if rgb[y, x].max() >= 1.0 or lhat[y, x] == 0.0:
                continue
            lum = oracle_mod.luminance(*rgb[y, x])
            assert abs(lum - t[y, x]) <= 1e-12, (y, x)
            checked += 1
    assert checked > 100


def test_unit_saturation_keeps_channel_ratios(oracle_mod):
    img = synth.hdr_pixels(np.random.default_rng(12), 8, 16)
    rgb, t, lhat, _ = oracle_mod.tonemap_colour(img, saturation=1.0)
    src = img.astype(np.float64)
    ok = (rgb.max(axis=2) < 1.0) & (lhat > 0)
    assert ok.sum() > 50
    for a, b in ((0, 1), (1, 2), (0, 2)):
        lhs = rgb[..., a] * src[..., b]
        rhs = rgb[..., b] * src[..., a]
        np.testing.assert_allclose(lhs[ok], rhs[ok], rtol=1e-13, atol=0)


def test_zero_saturation_is_grey_t(oracle_mod):
    img = _sdr(13, 7, 11)
    img[0, 0] = 0
    rgb, t, _, _ = oracle_mod.tonemap_colour(img, saturation=0.0)
    for c in range(3):
        np.testing.assert_array_equal(rgb[..., c], t)


@pytest.mark.parametrize("s", [0.0, 0.4, 1.0, 1.7])
def test_grey_and_black_pixels_stay_grey(oracle_mod, s):
    """Achromatic pixels have L equal to their value (Eqs. (1)-(6) all reduce to
    it), so C / Lhat = 1 and every channel is T; black (Lhat = 0) is grey T."""
    img = _sdr(14, 6, 10)
    img[1, 2] = (90, 90, 90)
    img[3, 4] = (255, 255, 255)
    img[2, 7] = (0, 0, 0)
    rgb, t, _, _ = oracle_mod.tonemap_colour(img, saturation=s)
    for y, x in ((1, 2), (3, 4), (2, 7)):
        for c in range(3):
            assert abs(rgb[y, x, c] - min(t[y, x], 1.0)) <= 1e-14


@pytest.mark.parametrize("s", [0.25, 1.0])
def test_two_pixel_closed_form(oracle_mod, s):
    """Pure red (200, 0, 0) and pure blue (0, 0, 90), default betas. From Eqs.
    (1)-(6): L_red = sqrt(beta_R beta_k) R and L_blue = B / sqrt(3), so red is
    the brighter pixel (T = 1/(1+e^-c)) and blue the darker (T = 1/(1+e^c));
    their ratios C / Lhat are 1/sqrt(beta_R beta_k) and sqrt(3)."""
    img = np.array([[[200, 0, 0], [0, 0, 90]]], np.uint8)
    rgb, t, _, _ = oracle_mod.tonemap_colour(img, contrast=C, saturation=s)
    assert abs(t[0, 0] - T_HI) < 1e-15 and abs(t[0, 1] - T_LO) < 1e-15
    red = min(1.0, T_HI * (1.0 / math.sqrt(0.55 * 0.8)) ** s)
    blue = min(1.0, T_LO * math.sqrt(3.0) ** s)
    np.testing.assert_allclose(rgb[0, 0], [red, 0.0, 0.0], rtol=1e-14, atol=0)
    np.testing.assert_allclose(rgb[0, 1], [0.0, 0.0, blue], rtol=1e-14, atol=0)
    if s == 1.0:
        assert rgb[0, 0, 0] == 1.0  # 0.8808 * 1.5076 is clamped


def test_saturation_orders_channels(oracle_mod):
    """For a channel above the luminance (C / Lhat > 1) the output grows with s;
    below it, the output shrinks."""
    img = _sdr(15, 5, 9)
    outs = [oracle_mod.tonemap_colour(img, saturation=s) for s in (0.3, 0.6, 0.9)]
    lhat = outs[0][2]
    src = img.astype(np.float64) / 255.0
    for c in range(3):
        ratio = np.where(lhat > 0, src[..., c] / np.where(lhat > 0, lhat, 1), 1.0)
        a, b, d = (o[0][..., c] for o in outs)
        up = ratio > 1
        assert np.all(a[up] <= b[up]) and np.all(b[up] <= d[up])
        down = ratio < 1
        assert np.all(a[down] >= b[down]) and np.all(b[down] >= d[down])


def test_nan_and_negative_channels(oracle_mod):
    assert oracle_mod.colour_channel(float("nan"), 0.5, 0.3, 0.7) == 0.0
    assert oracle_mod.colour_channel(-2.0, 0.5, 0.3, 0.7) == 0.0
    assert oracle_mod.colour_channel(-2.0, 0.5, 0.3, 0.0) == 0.3  # 0^0 = 1
    assert oracle_mod.colour_channel(0.4, 0.0, 0.3, 0.7) == 0.3


@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32])
@pytest.mark.parametrize("s", [0.0, 0.55, 1.0, 1.8])
def test_twin_agrees(oracle_mod, dtype, s):
    img = synth.random_image(16, 5, 7, dtype, scale=3.0)
    img[0, 0] = 0
    img[2, 3] = img[2, 3, 1]
    rgb, t, _, _ = oracle_mod.tonemap_colour(img, eps=1e-4, contrast=1.5, sigma_floor=1e-3,
                                             saturation=s)
    if dtype == np.float16:
        px, kind = img.view(np.uint16).tolist(), "f16"
    else:
        px, kind = img.astype(np.float64).tolist(), ("u8" if dtype == np.uint8 else "f32")
    want_rgb, want_t = twin.tonemap_colour(px, kind, 1e-4, 1.5, 1e-3, s)
    np.testing.assert_allclose(t, np.array(want_t), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rgb, np.array(want_rgb), rtol=1e-12, atol=1e-14)


def test_pitched_view_matches_packed(oracle_mod):
    big = synth.random_image(17, 12, 20, np.float16, scale=2.0)
    view = big[1:10, 2:19]
    a = oracle_mod.tonemap_colour(view, saturation=0.6)[0]
    b = oracle_mod.tonemap_colour(np.ascontiguousarray(view), saturation=0.6)[0]
    np.testing.assert_array_equal(a, b)


def test_rejects_negative_saturation(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.tonemap_colour(synth.random_image(18, 2, 2, np.uint8), saturation=-0.1)
