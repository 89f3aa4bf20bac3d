"""Pins of the oracle's comparator channels (rgb2gray weighted sum quoted in
Sec. I, V of HSV of Sec. III-B.1, CIE 1976 L* built on that Y)."""
import math

import numpy as np
import pytest

import synth
from oracle import ref as twin


@pytest.mark.parametrize("rgb,want", [((1, 0, 0), 0.2989), ((0, 1, 0), 0.5870), ((0, 0, 1), 0.1140),
                                      ((1, 1, 1), 0.9999), ((0, 0, 0), 0.0),
                                      ((0.5, 0.25, 0.125), 0.2989 * 0.5 + 0.5870 * 0.25 + 0.1140 * 0.125)])
def test_y601_weights(oracle_mod, rgb, want):
    assert oracle_mod.comparator(*rgb, "y601") == pytest.approx(want, abs=1e-15)


def test_hsv_value_is_max(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(200):
        r, g, b = rng.random(3)
        assert oracle_mod.comparator(r, g, b, "hsv_v") == max(r, g, b)
    assert oracle_mod.comparator(float("nan"), -2.0, 0.25, "hsv_v") == 0.25


def test_cielab_lightness_textbook_points(oracle_mod):
    # L* of Y: white 100, black 0, 18 % grey ~ 49.5 (textbook value), and the
    # linear segment 24389/27 * Y below the knee (6/29)^3.
    def lstar_of_gray(y):
        # a neutral pixel with rgb2gray Y = y: r = g = b = y / 0.9999
        v = y / 0.9999
        return 100.0 * oracle_mod.comparator(v, v, v, "cielab_l")
    assert lstar_of_gray(1.0) == pytest.approx(100.0, abs=1e-9)
    assert lstar_of_gray(0.0) == pytest.approx(0.0, abs=1e-12)
    assert lstar_of_gray(0.18) == pytest.approx(49.4961, abs=1e-3)
    assert lstar_of_gray(0.005) == pytest.approx(24389.0 / 27.0 * 0.005, rel=1e-12)
    knee = (6.0 / 29.0) ** 3
    assert lstar_of_gray(knee * (1 + 1e-12)) == pytest.approx(lstar_of_gray(knee * (1 - 1e-12)),
                                                               abs=1e-8)
    assert lstar_of_gray(knee) == pytest.approx(8.0, abs=1e-9)


def test_comparators_monotone_in_gray(oracle_mod):
    ys = np.linspace(0, 1, 2001)
    ls = [oracle_mod.comparator(y, y, y, "cielab_l") for y in ys]
    assert np.all(np.diff(ls) > 0)


@pytest.mark.parametrize("kind", ["y601", "hsv_v", "cielab_l"])
@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32])
def test_comparator_image_matches_twin(oracle_mod, kind, dtype):
    img = synth.random_image(20, 5, 7, dtype, scale=1.5)
    got = oracle_mod.comparator_image(img, kind)
    unit = 255.0 if dtype == np.uint8 else 1.0
    for y in range(5):
        for x in range(7):
            r, g, b = (float(v) / unit for v in img[y, x].astype(np.float64))
            assert got[y, x] == pytest.approx(twin.comparator(r, g, b, kind), abs=1e-15)


def test_paper_table_ordering_claims(oracle_mod):
    """Sec. I: rgb2gray weights green most; the paper's L exceeds it for red."""
    assert oracle_mod.comparator(0, 1, 0, "y601") > oracle_mod.comparator(1, 0, 0, "y601")
    assert oracle_mod.luminance(1, 0, 0) > oracle_mod.comparator(1, 0, 0, "y601")
    assert math.isclose(oracle_mod.comparator(0.3, 0.6, 0.1, "hsv_v"), 0.6)
