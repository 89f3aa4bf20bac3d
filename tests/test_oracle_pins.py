"""Pins of the FP64 oracle against what the paper and the mathematics fix.

The oracle is never checked against itself here: each test compares it with a
hand-derived closed form, an invariant implied by Eqs. (1)-(6), an independent
library routine (numpy's binary16 codec, Python's statistics/fsum), the
independent pure-Python twin, or a qualitative property the paper states.
"""
import math
import os
import statistics

import numpy as np
import pytest

import synth
from oracle import ref as twin

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BETAS = [(0.55, 0.8), (0.7, 0.6), (0.51, 0.99), (0.0, 1.0), (1.0, 0.0), (0.9, 0.5)]


def _closed_forms():
    rows = []
    with open(os.path.join(GOLDEN, "closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            cols = [c.strip() for c in line.split("|")]
            rows.append((tuple(float(v) for v in cols[0].split()), cols[1:]))
    return rows


def _eval(expr, br, bk):
    return eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt, "br": br, "bk": bk})


CLOSED = _closed_forms()


@pytest.mark.parametrize("beta_r,beta_k", BETAS)
@pytest.mark.parametrize("idx", range(len(CLOSED)))
def test_closed_forms(oracle_mod, idx, beta_r, beta_k):
    rgb, exprs = CLOSED[idx]
    want = [_eval(e, beta_r, beta_k) for e in exprs]
    got = oracle_mod.luminance_terms(*rgb, beta_r, beta_k)
    # terms: L_white, L_gr, L_warm, L_cool, L
    for g, w in zip(got, want):
        assert g == pytest.approx(w, rel=1e-13, abs=1e-15)
    # Scale invariance of the closed form: the pixel times 255 scales L by 255.
    assert oracle_mod.luminance(*(255 * c for c in rgb), beta_r, beta_k) == pytest.approx(
        255 * want[4], rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("beta_r,beta_k", BETAS)
def test_twin_matches_closed_forms(beta_r, beta_k):
    for rgb, exprs in CLOSED:
        t = twin.luminance_terms(*rgb, beta_r, beta_k)
        want = [_eval(e, beta_r, beta_k) for e in exprs]
        got = (t[0], t[2], t[3], t[4], t[5])
        for g, w in zip(got, want):
            assert g == pytest.approx(w, rel=1e-13, abs=1e-15)


def test_paper_claims_vs_ycbcr(oracle_mod):
    """Qualitative statements of Sec. I, II-A, II-B and III about L versus Y."""
    with open(os.path.join(GOLDEN, "paper_claims.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            parts = line.split()
            r, g, b = (int(v) for v in parts[:3])
            relation = parts[3]
            lum = oracle_mod.luminance(r, g, b)
            y601 = 0.299 * r + 0.587 * g + 0.114 * b
            if relation == "lighter":
                assert lum > y601, line
            else:
                assert lum < y601, line


def test_all_colours_range_invariant(all_colours_lut):
    """min(R,G,B) <= L <= max(R,G,B) for every 24-bit colour: Eq. (6) is a
    weighted RMS of two convex blends of terms that each lie in that range."""
    p = np.arange(1 << 24, dtype=np.int64)
    r, g, b = p >> 16, (p >> 8) & 255, p & 255
    lo = np.minimum(np.minimum(r, g), b)
    hi = np.maximum(np.maximum(r, g), b)
    lum = all_colours_lut
    assert np.all(lum >= lo * (1 - 1e-14) - 1e-12)
    assert np.all(lum <= hi * (1 + 1e-14) + 1e-12)


def test_achromatic_identity(all_colours_lut, oracle_mod):
    """R = G = B = v gives L = v (every term equals v)."""
    k = np.arange(256)
    lum = all_colours_lut[(k << 16) | (k << 8) | k]
    np.testing.assert_allclose(lum, k, rtol=1e-14, atol=1e-13)
    for v in (1e-30, 3.5, 1e6, 65504.0):
        assert oracle_mod.luminance(v, v, v) == pytest.approx(v, rel=1e-14)


def test_homogeneity(all_colours_lut, oracle_mod):
    """L(2R, 2G, 2B) = 2 L(R, G, B): every equation is degree-1 homogeneous."""
    p = np.arange(1 << 24, dtype=np.int64)
    r, g, b = p >> 16, (p >> 8) & 255, p & 255
    m = (r < 128) & (g < 128) & (b < 128)
    src = p[m]
    dbl = (r[m] * 2 << 16) | (g[m] * 2 << 8) | (b[m] * 2)
    np.testing.assert_allclose(all_colours_lut[dbl], 2 * all_colours_lut[src], rtol=1e-14,
                               atol=1e-12)
    rng = np.random.default_rng(5)
    for _ in range(200):
        rgb = rng.random(3) * 10
        s = 2.0 ** rng.integers(-20, 20)
        assert oracle_mod.luminance(*(rgb * s)) == pytest.approx(s * oracle_mod.luminance(*rgb),
                                                                 rel=1e-14)


def test_every_u8_code_reachable(all_colours_lut, oracle_mod):
    codes = oracle_mod.encode_u8(all_colours_lut / 255.0)
    assert len(np.unique(codes)) == 256


def test_beta_special_cases(oracle_mod):
    """beta_k = 1 keeps only L_warm; beta_k = 0 keeps only L_cool; beta_R = 1
    makes L_gr = R and beta_R = 0 makes L_gr = G (Eqs. (3), (6))."""
    rng = np.random.default_rng(11)
    for _ in range(100):
        r, g, b = rng.random(3)
        t = oracle_mod.luminance_terms(r, g, b, 0.55, 1.0)
        assert t[4] == pytest.approx(t[2], rel=1e-14)
        t = oracle_mod.luminance_terms(r, g, b, 0.55, 0.0)
        assert t[4] == pytest.approx(t[3], rel=1e-14)
        assert oracle_mod.luminance_terms(r, g, b, 1.0, 0.8)[1] == pytest.approx(r, rel=1e-14)
        assert oracle_mod.luminance_terms(r, g, b, 0.0, 0.8)[1] == pytest.approx(g, rel=1e-14)


def test_black_nan_negative(oracle_mod):
    assert oracle_mod.luminance(0, 0, 0) == 0.0
    assert oracle_mod.luminance(float("nan"), 0, 0) == 0.0
    assert oracle_mod.luminance(-1.0, 2.0, 0.0) == oracle_mod.luminance(0.0, 2.0, 0.0)
    assert oracle_mod.luminance(float("nan"), 1.0, 1.0) == oracle_mod.luminance(0.0, 1.0, 1.0)


@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32])
def test_twin_agrees_on_tiny_images(oracle_mod, dtype):
    """C oracle and pure-Python twin (independent transcriptions) agree."""
    img = synth.random_image(3, 7, 9, dtype, scale=4.0)
    img[0, 0] = 0  # black pixel
    img[1, 1] = img[1, 1, 0]  # grey pixel
    got = oracle_mod.decolorize(img, 0.55, 0.8)
    if dtype == np.float16:
        px = img.view(np.uint16).tolist()
        want = np.array(twin.decolorize_image(px, "f16"))
    else:
        want = np.array(twin.decolorize_image(img.astype(np.float64).tolist(),
                                              "u8" if dtype == np.uint8 else "f32"))
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)


def test_pitched_image_matches_packed(oracle_mod):
    big = synth.random_image(4, 10, 20, np.uint8)
    view = big[2:9, 3:17]  # row pitch 60 bytes, width 14
    np.testing.assert_array_equal(oracle_mod.decolorize(view),
                                  oracle_mod.decolorize(np.ascontiguousarray(view)))
    img = synth.random_image(5, 33, 17, np.float32)
    np.testing.assert_array_equal(oracle_mod.decolorize(img, nthreads=4),
                                  oracle_mod.decolorize(img, nthreads=1))


def test_f16_decode_all_patterns(oracle_mod):
    """binary16 decoding by definition vs numpy's independent decoder."""
    bits = np.arange(65536, dtype=np.uint16)
    got = oracle_mod.decode_f16(bits)
    want = bits.view(np.float16).astype(np.float64)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    np.testing.assert_array_equal(got[~nan], want[~nan])
    for b in (0x0001, 0x03FF, 0x0400, 0x3C00, 0x7BFF, 0xC000):
        assert twin.half_bits_to_float(b) == float(np.uint16(b).view(np.float16))


def test_f16_encode_rne(oracle_mod):
    """Round-to-nearest-even encoding vs numpy's float64 -> float16 cast."""
    rng = np.random.default_rng(2)
    vals = np.concatenate([
        rng.random(20000) * 2.0,
        np.exp(rng.uniform(-20, 11.2, 20000)),
        # exact midpoints between neighbouring halves (ties)
        (np.arange(0, 4096, dtype=np.float64) + 0.5) * 2.0 ** -24,
        (1024 + np.arange(0, 1024) + 0.5) * 2.0 ** -10,
        [0.0, 65504.0, 65519.99, 65520.0, 1e9, 2.0 ** -25, 2.0 ** -25 * 1.0000001],
    ])
    got = oracle_mod.encode_f16(vals).view(np.uint16)
    with np.errstate(over="ignore"):
        want = vals.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(got, want)


def test_u8_encode(oracle_mod):
    lhat = np.array([0.0, 127.5 / 255, 127.49 / 255, 1.0, 1.2, -0.3, np.nan, 254.5 / 255])
    np.testing.assert_array_equal(oracle_mod.encode_u8(lhat), [0, 128, 127, 255, 255, 0, 0, 255])
    for v in lhat[:-2]:
        assert twin.encode_u8(v) == oracle_mod.encode_u8(np.array([v]))[0]


# ------------------------------------------------------------------ tone map

TM = dict(eps=1e-4, contrast=2.0, sigma_floor=1e-3)


def test_tonemap_two_pixels_closed_form(oracle_mod):
    """Two distinct values: x - mu = +-sigma, so T = 1/(1 + exp(-+c))."""
    img = np.array([[[200, 10, 10], [10, 20, 200]]], np.uint8)
    for c in (1.0, 2.0, 3.5):
        t, _, _ = oracle_mod.tonemap(img, contrast=c, eps=1e-4, sigma_floor=1e-3)
        assert sorted(t.ravel()) == pytest.approx([1 / (1 + math.exp(c)), 1 / (1 + math.exp(-c))],
                                                  abs=1e-14)
    t, _, _ = oracle_mod.tonemap(img, **TM)
    assert sorted(t.ravel()) == pytest.approx([0.1192029220221175, 0.8807970779778823], abs=1e-14)


def test_tonemap_constant_image(oracle_mod):
    img = np.full((5, 6, 3), 77, np.uint8)
    t, lhat, st = oracle_mod.tonemap(img, **TM)
    assert st["sigma"] < 1e-14  # zero up to the rounding of the mean
    np.testing.assert_allclose(t, 0.5, atol=1e-11)
    assert st["mu"] == pytest.approx(math.log(77 / 255 + 1e-4), rel=1e-14)


def test_tonemap_stats_vs_statistics_module(oracle_mod):
    img = synth.random_image(8, 13, 11, np.float32, scale=3.0)
    lhat = oracle_mod.decolorize(img)
    st = oracle_mod.tonemap_stats(lhat, 1e-4)
    xs = [math.log(v + 1e-4) for v in lhat.ravel()]
    assert st["mu"] == pytest.approx(statistics.fmean(xs), rel=1e-13, abs=1e-15)
    assert st["sigma"] == pytest.approx(statistics.pstdev(xs), rel=1e-12)
    assert st["l_min"] == lhat.min() and st["l_max"] == lhat.max()
    mu, sigma, lo, hi = twin.tonemap_stats(list(lhat.ravel()), 1e-4)
    assert (mu, sigma) == pytest.approx((st["mu"], st["sigma"]), rel=1e-13)


def test_tonemap_stats_counted_vs_statistics_module(oracle_mod):
    """Statistics of an image given as a histogram of its values: equal to the
    statistics module's mean and population deviation of the expanded list of
    x = ln(Lhat + eps), and to the per-pixel oracle on that list; zero counts
    take no part, also not in the extremes."""
    rng = np.random.default_rng(81)
    vals = rng.random(40) * 3.0
    counts = rng.integers(0, 6, 40)
    counts[[0, 7]] = 0
    vals[0], vals[7] = 100.0, 1e-9  # extremes that must not count
    st = oracle_mod.tonemap_stats_counted(vals, counts, 1e-4)
    expanded = np.repeat(vals, counts)
    xs = [math.log(v + 1e-4) for v in expanded]
    assert st["count"] == len(xs)
    assert st["mu"] == pytest.approx(statistics.fmean(xs), rel=1e-13, abs=1e-15)
    assert st["sigma"] == pytest.approx(statistics.pstdev(xs), rel=1e-12)
    assert st["l_min"] == expanded.min() and st["l_max"] == expanded.max()
    ref = oracle_mod.tonemap_stats(expanded, 1e-4)
    assert (st["mu"], st["sigma"]) == pytest.approx((ref["mu"], ref["sigma"]), rel=1e-13)


def test_tonemap_symmetry_monotone_exposure(oracle_mod):
    img = synth.random_image(9, 16, 16, np.float32, scale=5.0) + np.float32(0.01)
    t, lhat, st = oracle_mod.tonemap(img, eps=0.0, contrast=2.0, sigma_floor=1e-3)
    # odd symmetry about mu: T(mu + d) + T(mu - d) = 1
    for d in (0.1, 0.7, 2.0):
        a = oracle_mod.tonemap_curve(np.array([math.exp(st["mu"] + d)]), st["mu"], st["sigma"],
                                     eps=0.0)[0]
        b = oracle_mod.tonemap_curve(np.array([math.exp(st["mu"] - d)]), st["mu"], st["sigma"],
                                     eps=0.0)[0]
        assert a + b == pytest.approx(1.0, abs=1e-14)
    # monotone in L
    order = np.argsort(lhat.ravel(), kind="stable")
    assert np.all(np.diff(t.ravel()[order]) >= -1e-15)
    # exposure invariance with eps = 0 (scale by 2^k is exact in float32)
    t2, _, st2 = oracle_mod.tonemap(img * np.float32(8.0), eps=0.0, contrast=2.0, sigma_floor=1e-3)
    np.testing.assert_allclose(t2, t, atol=1e-13)
    assert st2["sigma"] == pytest.approx(st["sigma"], rel=1e-12)
    assert st2["mu"] == pytest.approx(st["mu"] + math.log(8.0), rel=1e-13)


def test_tonemap_twin_curve(oracle_mod):
    img = synth.random_image(10, 6, 5, np.uint8)
    t, lhat, st = oracle_mod.tonemap(img, **TM)
    for v, tv in zip(lhat.ravel(), t.ravel()):
        assert twin.tonemap_curve(v, 1e-4, 2.0, st["mu"], st["sigma"], 1e-3) == pytest.approx(
            tv, abs=1e-15)


def test_hdr_generator_exact_and_stored_agree():
    """The binary16 image is the round-to-nearest of the exact radiance."""
    a = synth.hdr_pixels(np.random.default_rng(5), 7, 9)
    b = synth.hdr_pixels(np.random.default_rng(5), 7, 9, exact=True)
    assert a.dtype == np.float16 and b.dtype == np.float64
    np.testing.assert_array_equal(a, b.astype(np.float16))


def _hand_table():
    rows = []
    with open(os.path.join(GOLDEN, "hand_table.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            cols = [c.strip() for c in line.split("|")]
            rgb = tuple(eval(v, {"__builtins__": {}}) for v in cols[0].split())
            rows.append((rgb, [float(c) for c in cols[1:7]], int(cols[7])))
    return rows


@pytest.mark.parametrize("row", _hand_table(), ids=lambda r: "%.4g,%.4g,%.4g" % r[0])
def test_hand_table(oracle_mod, row):
    """Pixels evaluated by hand from Eqs. (1)-(6) at beta_R = 0.55, beta_k = 0.8
    (tests/golden/hand_table.txt): the four intermediate terms to their 8
    printed digits, L to its 10, the Sec. I rgb2gray value to 4, and the 8-bit
    code exactly; for the C oracle and the Python twin."""
    rgb, want, code = row
    c_terms = oracle_mod.luminance_terms(*rgb, 0.55, 0.8)
    t = twin.luminance_terms(*rgb, 0.55, 0.8)
    py_terms = (t[0], t[2], t[3], t[4], t[5])
    for got in (c_terms, py_terms):
        for g, w in zip(got[:4], want[:4]):
            assert abs(g - w) <= 5e-9
        assert abs(got[4] - want[4]) <= 1e-10
    assert abs(0.2989 * rgb[0] + 0.5870 * rgb[1] + 0.1140 * rgb[2] - want[5]) <= 5e-5
    assert int(oracle_mod.encode_u8(np.array([c_terms[4]]))[0]) == code
    assert twin.encode_u8(py_terms[4]) == code


def test_infinite_channels_read_as_format_maximum(oracle_mod):
    """+Inf in a binary16 channel reads as 65504 and a binary32 channel above
    1e18 as 1e18 (the reading for values past the input's range): a pure-red
    +Inf pixel gives sqrt(beta_R beta_k) times that value (the red closed form,
    scaled by degree-1 homogeneity), and every pixel with an infinite channel
    equals the same pixel with the cap in its place, in the C oracle and the
    Python twin."""
    inf_h, cap_h = np.float16(np.inf), np.float16(65504.0)
    img = np.array([[[inf_h, 0, 0], [inf_h, 1, 2], [0.5, inf_h, inf_h], [np.nan, -1, inf_h]]],
                   np.float16)
    capped = np.where(np.isinf(img), cap_h, img).astype(np.float16)
    got = oracle_mod.decolorize(img)
    assert got[0, 0] == pytest.approx(math.sqrt(0.55 * 0.8) * 65504.0, rel=1e-14)
    np.testing.assert_array_equal(got, oracle_mod.decolorize(capped))
    bits = img.view(np.uint16)
    tw = twin.decolorize_image([[tuple(int(v) for v in px) for px in bits[0]]], "f16")
    np.testing.assert_allclose(np.array(tw), got, rtol=1e-13)
    f = np.array([[[np.inf, 0, 0], [3e18, 0, 0], [0.25, np.inf, 7.0], [0, 0, 2e20]]], np.float32)
    gf = oracle_mod.decolorize(f)
    red = math.sqrt(0.55 * 0.8) * 1e18  # the red closed form at the cap
    assert gf[0, 0] == pytest.approx(red, rel=1e-14)
    assert gf[0, 1] == gf[0, 0]
    assert gf[0, 3] == pytest.approx(1e18 / math.sqrt(3.0), rel=1e-14)  # blue closed form
    twf = twin.decolorize_image([[tuple(float(v) for v in px) for px in f[0]]], "f32")
    np.testing.assert_allclose(np.array(twf), gf, rtol=1e-13)
    # the tone map of an image with an infinite channel stays finite
    t, _, st = oracle_mod.tonemap(np.concatenate([img, capped], 1))
    assert np.all(np.isfinite(t)) and math.isfinite(st["mu"])
