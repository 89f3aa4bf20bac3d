"""Pins of the luminance as a function of the two weights (Fig. 4 plots L along
colour ramps for several beta_R and beta_k; its data is not in the paper's
text, so these pins come from Eqs. (3)-(6) themselves):

- beta_R enters only through L_gr^2 = beta_R R^2 + (1 - beta_R) G^2, whose slope
  is R^2 - G^2; L_warm grows with L_gr (weight R/S >= 0) and L with L_warm, so
  L rises with beta_R exactly where R > G and falls where R < G;
- d(L^2)/d(beta_k) = L_warm^2 - L_cool^2 (Eq. (6)), so L rises with beta_k exactly
  where L_warm > L_cool;
- the ramps' end points have closed forms: pure red sqrt(beta_R beta_k) R, pure
  green sqrt(beta_k / 3) G, pure blue B / sqrt(3) for every weight pair.
"""
import math

import numpy as np
import pytest

import synth

GRID = [0.0, 0.3, 0.5, 0.55, 0.7, 0.8, 0.95, 1.0]


def _pixels():
    ramps = synth.colour_ramps(129)
    rnd = synth.random_image(21, 16, 16, np.uint8).reshape(-1, 3)
    return np.concatenate([r.reshape(-1, 3) for r in ramps.values()] + [rnd]).astype(np.float64)


@pytest.mark.parametrize("beta_k", [0.2, 0.8, 1.0])
def test_beta_r_direction(oracle_mod, beta_k):
    px = _pixels()
    for b1, b2 in zip(GRID[:-1], GRID[1:]):
        for r, g, b in px:
            d = oracle_mod.luminance(r, g, b, b2, beta_k) - oracle_mod.luminance(r, g, b, b1, beta_k)
            if r > g and r > 0:
                assert d > 0, (r, g, b, b1, b2)
            elif r < g and r > 0:
                assert d < 0, (r, g, b, b1, b2)
            else:
                assert abs(d) <= 1e-12 * (1 + abs(r + g + b)), (r, g, b, b1, b2)


@pytest.mark.parametrize("beta_r", [0.0, 0.55, 0.9])
def test_beta_k_direction(oracle_mod, beta_r):
    px = _pixels()
    for b1, b2 in zip(GRID[:-1], GRID[1:]):
        for r, g, b in px:
            _, _, warm, cool, _ = oracle_mod.luminance_terms(r, g, b, beta_r, 0.5)
            d = oracle_mod.luminance(r, g, b, beta_r, b2) - oracle_mod.luminance(r, g, b, beta_r, b1)
            gap = warm - cool
            if abs(gap) <= 1e-9 * (1 + warm):
                assert abs(d) <= 1e-9 * (1 + warm)
            else:
                assert np.sign(d) == np.sign(gap), (r, g, b, b1, b2)


@pytest.mark.parametrize("beta_r", GRID)
@pytest.mark.parametrize("beta_k", GRID)
def test_ramp_end_points(oracle_mod, beta_r, beta_k):
    ramps = synth.colour_ramps(17)
    got = {k: oracle_mod.decolorize(v, beta_r, beta_k)[0] for k, v in ramps.items()}
    red = math.sqrt(beta_r * beta_k)
    green = math.sqrt(beta_k / 3.0)
    blue = 1.0 / math.sqrt(3.0)
    for name, start, end in (("g_to_r", green, red), ("b_to_r", blue, red), ("b_to_g", blue, green)):
        assert got[name][0] == pytest.approx(start, abs=1e-14)
        assert got[name][-1] == pytest.approx(end, abs=1e-14)


def test_ramps_are_straight_lines():
    ramps = synth.colour_ramps(256)
    for img in ramps.values():
        assert img.shape == (1, 256, 3) and img.dtype == np.uint8
        s = img[0].astype(np.int32).sum(axis=1)
        assert np.all(np.abs(s - 255) <= 1)  # the two endpoints' channels trade off
