"""Pure-Python FP64 twin of the C oracle (scalar, slow, for tiny inputs).

TEST INFRASTRUCTURE ONLY: used by the test-suite to cross-check the C oracle
(two independent transcriptions of the same definitions). Nothing on the
product path imports it.

Follows Sec. II-B, Eqs. (1)-(6) of arXiv 2108.13656 for the luminance, and this
project's reading of the centred-sigmoid global tone curve of Sec. III-B.1 (log
domain, centred on the mean of ln(Lhat + eps), slope normalised by the
population standard deviation) and of its colour output (ratio re-colouring
C_out = min(1, T (C / Lhat)^s)).
"""
import math

BETA_R = 0.55  # Sec. II-B, parameter choice after Eq. (6)
BETA_K = 0.80


def _clean(v):
    """NaN and negative channel values read as 0."""
    v = float(v)
    return v if v > 0.0 else 0.0


def luminance_terms(r, g, b, beta_r=BETA_R, beta_k=BETA_K):
    """(L_white, L_b, L_gr, L_warm, L_cool, L) of one pixel, Eqs. (1)-(6).

    A black pixel returns all zeros (limit of Eqs. (4)-(6) as R+G+B -> 0).
    """
    r, g, b = _clean(r), _clean(g), _clean(b)
    total = r + g + b
    # Eq. (1): RMS of the three channels ("Euclidean distance" of RGB, /3).
    l_white = math.sqrt((r * r + g * g + b * b) / 3.0)
    # Eq. (2): the blue channel as it is.
    l_b = b
    # Eq. (3): red and green weighted by beta_R and 1 - beta_R.
    l_gr = math.sqrt(beta_r * r * r + (1.0 - beta_r) * g * g)
    if total == 0.0:
        return (l_white, l_b, l_gr, 0.0, 0.0, 0.0)
    red_share = r / total
    blue_share = b / total
    # Eq. (4): warm blend driven by the red share.
    l_warm = red_share * l_gr + (1.0 - red_share) * l_white
    # Eq. (5): cool blend driven by the inverse blue share.
    l_cool = (1.0 - blue_share) * l_b + blue_share * l_white
    # Eq. (6): weighted RMS of the warm and cool luminances.
    lum = math.sqrt(beta_k * l_warm ** 2 + (1.0 - beta_k) * l_cool ** 2)
    return (l_white, l_b, l_gr, l_warm, l_cool, lum)


def luminance(r, g, b, beta_r=BETA_R, beta_k=BETA_K):
    """L of one pixel in the units of its input, Eqs. (1)-(6)."""
    return luminance_terms(r, g, b, beta_r, beta_k)[5]


def half_bits_to_float(bits):
    """IEEE 754 binary16 bit pattern -> Python float (definition of the format)."""
    sign = -1.0 if (bits >> 15) & 1 else 1.0
    exponent = (bits >> 10) & 0x1F
    fraction = bits & 0x3FF
    if exponent == 0:
        return sign * fraction * 2.0 ** -24
    if exponent == 31:
        return sign * math.inf if fraction == 0 else math.nan
    return sign * (1.0 + fraction / 1024.0) * 2.0 ** (exponent - 15)


def decode(px, dtype):
    """The three channel values of a pixel as the method reads them: binary16
    bit patterns decoded, +Inf in binary16 read as 65504 (its largest finite
    value), binary32 values above 1e18 (the top of the supported range, +Inf
    included) read as 1e18; NaN and negatives are left to _clean."""
    if dtype == "f16":
        return [min(half_bits_to_float(int(v)), 65504.0) for v in px]
    if dtype == "f32":
        return [min(float(v), 1e18) if v == v else float(v) for v in px]
    return [float(v) for v in px]


def decolorize_image(pixels, dtype, beta_r=BETA_R, beta_k=BETA_K):
    """Normalised luminance of a nested-list image [[(r, g, b), ...], ...].

    dtype is "u8" (code values, output divided by 255), "f16" (values given as
    binary16 bit patterns) or "f32" (values as floats).
    """
    out = []
    for row in pixels:
        out_row = []
        for px in row:
            px = decode(px, dtype)
            lum = luminance(px[0], px[1], px[2], beta_r, beta_k)
            out_row.append(lum / 255.0 if dtype == "u8" else lum)
        out.append(out_row)
    return out


def encode_u8(lhat):
    """Round half up and clamp: min(255, floor(255 * Lhat + 0.5))."""
    return min(255, int(math.floor(255.0 * _clean(lhat) + 0.5)))


def tonemap_stats(lhat_values, eps):
    """(mu, sigma, min, max) of x = ln(Lhat + eps) over all pixels (fsum)."""
    xs = [math.log(v + eps) for v in lhat_values]
    n = len(xs)
    mu = math.fsum(xs) / n
    sigma = math.sqrt(math.fsum((x - mu) ** 2 for x in xs) / n)
    return mu, sigma, min(lhat_values), max(lhat_values)


def tonemap_curve(lhat, eps, contrast, mu, sigma, sigma_floor):
    """Centred sigmoid of ln(Lhat + eps) around mu with slope contrast / sigma."""
    scale = max(sigma, sigma_floor)
    x = math.log(lhat + eps)
    return 1.0 / (1.0 + math.exp(-contrast * (x - mu) / scale))


def comparator(r, g, b, kind):
    """Comparator gray channels on normalised RGB: rgb2gray weighted sum, V of
    HSV, CIE L* / 100 built on the rgb2gray Y with white Y_n = 1."""
    r, g, b = _clean(r), _clean(g), _clean(b)
    gray = 0.2989 * r + 0.5870 * g + 0.1140 * b
    if kind == "y601":
        return gray
    if kind == "hsv_v":
        return max(r, g, b)
    knee = (6.0 / 29.0) ** 3
    if gray > knee:
        f = gray ** (1.0 / 3.0)
    else:
        f = gray / (3.0 * (6.0 / 29.0) ** 2) + 4.0 / 29.0
    return (116.0 * f - 16.0) / 100.0


def colour_channel(c, lhat, t, s):
    """One re-coloured channel: min(1, T (C / Lhat)^s), grey T where Lhat == 0,
    0^0 = 1 (normalised units)."""
    c = _clean(c)
    if not lhat > 0.0:
        return t
    ratio = c / lhat
    v = t * (1.0 if s == 0.0 else (0.0 if ratio == 0.0 else ratio ** s))
    return min(v, 1.0)


def tonemap_colour(pixels, dtype, eps, contrast, sigma_floor, saturation,
                   beta_r=BETA_R, beta_k=BETA_K):
    """Colour global tone map of a nested-list image (same conventions as
    decolorize_image): returns (rgb rows of (r, g, b), T rows)."""
    lhat = decolorize_image(pixels, dtype, beta_r, beta_k)
    flat = [v for row in lhat for v in row]
    mu, sigma, _, _ = tonemap_stats(flat, eps)
    unit = 255.0 if dtype == "u8" else 1.0
    rgb, t_rows = [], []
    for row, lrow in zip(pixels, lhat):
        out_row, t_row = [], []
        for px, lh in zip(row, lrow):
            px = decode(px, dtype)
            t = tonemap_curve(lh, eps, contrast, mu, sigma, sigma_floor)
            out_row.append(tuple(colour_channel(float(v) / unit, lh, t, saturation) for v in px))
            t_row.append(t)
        rgb.append(out_row)
        t_rows.append(t_row)
    return rgb, t_rows


def tonemap_local(pixels, dtype, eps, contrast, sigma_floor, strength,
                  beta_r=BETA_R, beta_k=BETA_K, tile=64, bins=64):
    """Local tone map of a nested-list image: smoothed local histogram
    equalisation on a tile grid blended with the global curve (same reading as
    the C oracle, written independently; for tiny images only)."""
    lhat = decolorize_image(pixels, dtype, beta_r, beta_k)
    h, w = len(lhat), len(lhat[0])
    flat = [v for row in lhat for v in row]
    mu, sigma, _, _ = tonemap_stats(flat, eps)
    nx, ny = -(-w // tile), -(-h // tile)

    def pos(v):
        u = 2.0 * math.log((v + eps) / eps, 2) - 0.5
        return min(max(u, 0.0), bins - 1.0)

    hist = {(tx, ty): [0.0] * bins for tx in range(nx) for ty in range(ny)}
    for y in range(h):
        for x in range(w):
            u = pos(lhat[y][x])
            k = min(int(math.floor(u)), bins - 2)
            f = u - k
            hb = hist[(x // tile, y // tile)]
            hb[k] += 1.0 - f
            hb[k + 1] += f
    smooth = {}
    for (tx, ty) in hist:
        acc = [0.0] * bins
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb = hist.get((tx + dx, ty + dy))
                if nb is None:
                    continue
                wgt = (2.0 if dx == 0 else 1.0) * (2.0 if dy == 0 else 1.0)
                for b in range(bins):
                    acc[b] += wgt * nb[b]
        smooth[(tx, ty)] = acc

    def ramp(x):  # integral of the unit triangle
        if x <= -1.0:
            return 0.0
        if x <= 0.0:
            return 0.5 * (1.0 + x) ** 2
        if x <= 1.0:
            return 1.0 - 0.5 * (1.0 - x) ** 2
        return 1.0

    def curve(t, u):
        s = smooth[t]
        return math.fsum(s[b] * ramp(u - b) for b in range(bins)) / math.fsum(s)

    def corners(p, n):
        g = (p + 0.5) / tile - 0.5
        a = math.floor(g)
        fr = g - a
        if a < 0:
            a, fr = 0, 0.0
        if a >= n - 1:
            a, fr = n - 1, 0.0
        return a, min(a + 1, n - 1), fr

    out = []
    for y in range(h):
        y0, y1, fy = corners(y, ny)
        row = []
        for x in range(w):
            x0, x1, fx = corners(x, nx)
            u = pos(lhat[y][x])
            tl = ((1 - fx) * (1 - fy) * curve((x0, y0), u) + fx * (1 - fy) * curve((x1, y0), u) +
                  (1 - fx) * fy * curve((x0, y1), u) + fx * fy * curve((x1, y1), u))
            tg = tonemap_curve(lhat[y][x], eps, contrast, mu, sigma, sigma_floor)
            row.append((1.0 - strength) * tg + strength * tl)
        out.append(row)
    return out
