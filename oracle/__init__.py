"""FP64 CPU oracle: numpy-facing wrapper around ``decolor_ref.c``.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path (the HIP
library and its Python binding) never does, and the two share no code.

Every function here marshals arguments and calls the C oracle, whose header
comment cites the passages of arXiv 2108.13656 it follows (Sec. II-B, Eqs.
(1)-(6); Sec. III-B.1 for the tone curve and its colour output; Sec. III-B.2
for the local tone map).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "decolor_ref.c")
_LIB_PATH = os.path.join(_HERE, "libdecolor_ref.so")

DTYPE_CODES = {np.dtype(np.uint8): 0, np.dtype(np.float16): 1, np.dtype(np.float32): 2}

_lib = None


def build():
    """Compile the oracle with plain IEEE double semantics (no fusion, no fast-math)."""
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-fPIC",
           "-shared", "-pthread", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
    vp = ctypes.c_void_p
    lib.ref_decolor_px.restype = d
    lib.ref_decolor_px.argtypes = [d, d, d, d, d]
    lib.ref_decolor_px_terms.restype = None
    lib.ref_decolor_px_terms.argtypes = [d, d, d, d, d, vp]
    lib.ref_half_to_double.restype = d
    lib.ref_half_to_double.argtypes = [ctypes.c_uint16]
    lib.ref_double_to_half.restype = ctypes.c_uint16
    lib.ref_double_to_half.argtypes = [d]
    lib.ref_encode_u8.restype = ctypes.c_uint8
    lib.ref_encode_u8.argtypes = [d]
    for name in ("ref_encode_u8_array", "ref_encode_f16_array", "ref_decode_f16_array"):
        getattr(lib, name).restype = None
        getattr(lib, name).argtypes = [vp, i64, vp]
    lib.ref_decolorize_image.restype = i32
    lib.ref_decolorize_image.argtypes = [vp, i32, i32, i32, i64, d, d, vp, i32]
    lib.ref_all_colours.restype = None
    lib.ref_all_colours.argtypes = [d, d, vp]
    lib.ref_comparator_px.restype = d
    lib.ref_comparator_px.argtypes = [d, d, d, i32]
    lib.ref_comparator_image.restype = i32
    lib.ref_comparator_image.argtypes = [vp, i32, i32, i32, i64, i32, vp]
    lib.ref_tonemap_stats.restype = None
    lib.ref_tonemap_stats.argtypes = [vp, i64, d, vp]
    lib.ref_tonemap_stats_counted.restype = None
    lib.ref_tonemap_stats_counted.argtypes = [vp, vp, i64, d, vp]
    lib.ref_tonemap_curve.restype = d
    lib.ref_tonemap_curve.argtypes = [d, d, d, d, d, d]
    lib.ref_tonemap_curve_array.restype = None
    lib.ref_tonemap_curve_array.argtypes = [vp, i64, d, d, d, d, d, vp]
    lib.ref_tonemap_image.restype = i32
    lib.ref_tonemap_image.argtypes = [vp, i32, i32, i32, i64, d, d, d, d, d, vp, vp, vp, i32]
    lib.ref_tonemap_local_image.restype = i32
    lib.ref_tonemap_local_image.argtypes = [vp, i32, i32, i32, i64, d, d, d, d, d, d, vp, vp, i32,
                                            vp, i64]
    lib.ref_recolour_image.restype = i32
    lib.ref_recolour_image.argtypes = [vp, i32, i32, i32, i64, vp, vp, d, vp]
    lib.ref_colour_channel.restype = d
    lib.ref_colour_channel.argtypes = [d, d, d, d]
    lib.ref_tonemap_colour_image.restype = i32
    lib.ref_tonemap_colour_image.argtypes = [vp, i32, i32, i32, i64, d, d, d, d, d, d, vp, vp, vp,
                                             vp, i32]
    _lib = lib
    return lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _image_args(img):
    """(array, dtype code, W, H, pitch bytes) for an HxWx3 array whose last two
    axes are packed (a row-strided view is fine)."""
    img = np.asarray(img)
    if img.ndim != 3 or img.shape[2] != 3:
        raise ValueError("expected an HxWx3 image")
    code = DTYPE_CODES.get(img.dtype)
    if code is None:
        raise ValueError("unsupported dtype %s" % img.dtype)
    es = img.dtype.itemsize
    if img.strides[2] != es or img.strides[1] != 3 * es or img.strides[0] < 3 * es * img.shape[1]:
        img = np.ascontiguousarray(img)
    return img, code, img.shape[1], img.shape[0], img.strides[0]


def luminance(r, g, b, beta_r=0.55, beta_k=0.8):
    """L of one pixel (input units), Eqs. (1)-(6)."""
    return _load().ref_decolor_px(r, g, b, beta_r, beta_k)


def luminance_terms(r, g, b, beta_r=0.55, beta_k=0.8):
    """(L_white, L_gr, L_warm, L_cool, L) of one pixel."""
    out = np.zeros(5, np.float64)
    _load().ref_decolor_px_terms(r, g, b, beta_r, beta_k, _ptr(out))
    return tuple(out)


def decolorize(img, beta_r=0.55, beta_k=0.8, nthreads=1):
    """Normalised luminance Lhat (float64, HxW) of an HxWx3 u8/f16/f32 image."""
    img, code, w, h, pitch = _image_args(img)
    out = np.empty((h, w), np.float64)
    rc = _load().ref_decolorize_image(_ptr(img), code, w, h, pitch, beta_r, beta_k, _ptr(out),
                                      int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the image")
    return out


COMPARATORS = {"y601": 1, "hsv_v": 2, "cielab_l": 3}


def comparator(r, g, b, kind):
    """One comparator channel (normalised inputs and output): 'y601', 'hsv_v'
    or 'cielab_l' (L* / 100)."""
    return _load().ref_comparator_px(r, g, b, COMPARATORS[kind])


def comparator_image(img, kind):
    """Comparator channel (float64 HxW, normalised units) of an HxWx3 image."""
    img, code, w, h, pitch = _image_args(img)
    out = np.empty((h, w), np.float64)
    if _load().ref_comparator_image(_ptr(img), code, w, h, pitch, COMPARATORS[kind], _ptr(out)):
        raise ValueError("oracle rejected the image")
    return out


def all_colours(beta_r=0.55, beta_k=0.8):
    """L in code units for every 24-bit colour, indexed (R << 16) | (G << 8) | B."""
    out = np.empty(1 << 24, np.float64)
    _load().ref_all_colours(beta_r, beta_k, _ptr(out))
    return out


def encode_u8(lhat):
    """min(255, floor(255 * Lhat + 0.5)) elementwise."""
    a = np.ascontiguousarray(lhat, np.float64)
    out = np.empty(a.shape, np.uint8)
    _load().ref_encode_u8_array(_ptr(a), a.size, _ptr(out))
    return out


def encode_f16(values):
    """IEEE binary16, round to nearest even, elementwise."""
    a = np.ascontiguousarray(values, np.float64)
    out = np.empty(a.shape, np.uint16)
    _load().ref_encode_f16_array(_ptr(a), a.size, _ptr(out))
    return out.view(np.float16)


def decode_f16(halves):
    """binary16 -> float64 by the format's definition."""
    a = np.ascontiguousarray(halves).view(np.uint16)
    out = np.empty(a.shape, np.float64)
    _load().ref_decode_f16_array(_ptr(a), a.size, _ptr(out))
    return out


def tonemap_stats(lhat, eps=1e-4):
    """dict(mu, sigma, l_min, l_max, count) of x = ln(Lhat + eps) over all pixels."""
    a = np.ascontiguousarray(lhat, np.float64).ravel()
    st = np.zeros(4, np.float64)
    _load().ref_tonemap_stats(_ptr(a), a.size, eps, _ptr(st))
    return {"mu": st[0], "sigma": st[1], "l_min": st[2], "l_max": st[3], "count": a.size}


def tonemap_stats_counted(lhat, counts, eps=1e-4):
    """tonemap_stats of the multiset in which value lhat[i] occurs counts[i]
    times (an image given as the histogram of its colours)."""
    a = np.ascontiguousarray(lhat, np.float64).ravel()
    c = np.ascontiguousarray(counts, np.int64).ravel()
    if a.size != c.size:
        raise ValueError("lhat and counts differ in size")
    st = np.zeros(4, np.float64)
    _load().ref_tonemap_stats_counted(_ptr(a), _ptr(c), a.size, eps, _ptr(st))
    return {"mu": st[0], "sigma": st[1], "l_min": st[2], "l_max": st[3], "count": int(c.sum())}


def tonemap_curve(lhat, mu, sigma, eps=1e-4, contrast=2.0, sigma_floor=1e-3):
    """Centred sigmoid T of every value of lhat, given the image statistics."""
    a = np.ascontiguousarray(lhat, np.float64)
    out = np.empty(a.shape, np.float64)
    _load().ref_tonemap_curve_array(_ptr(a), a.size, eps, contrast, mu, sigma, sigma_floor,
                                    _ptr(out))
    return out


def tonemap(img, beta_r=0.55, beta_k=0.8, eps=1e-4, contrast=2.0, sigma_floor=1e-3,
            nthreads=1):
    """Global tone map of one image: (T float64 HxW, Lhat float64 HxW, stats dict)."""
    img, code, w, h, pitch = _image_args(img)
    t = np.empty((h, w), np.float64)
    lhat = np.empty((h, w), np.float64)
    st = np.zeros(4, np.float64)
    rc = _load().ref_tonemap_image(_ptr(img), code, w, h, pitch, beta_r, beta_k, eps, contrast,
                                   sigma_floor, _ptr(lhat), _ptr(t), _ptr(st), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the image")
    stats = {"mu": st[0], "sigma": st[1], "l_min": st[2], "l_max": st[3], "count": w * h}
    return t, lhat, stats


def colour_channel(c, lhat, t, saturation=1.0):
    """One re-coloured channel min(1, T (C / Lhat)^s); grey T where Lhat == 0."""
    return _load().ref_colour_channel(c, lhat, t, saturation)


def tonemap_colour(img, beta_r=0.55, beta_k=0.8, eps=1e-4, contrast=2.0, sigma_floor=1e-3,
                   saturation=1.0, nthreads=1):
    """Colour global tone map of one image: (rgb float64 HxWx3, T HxW, Lhat HxW,
    stats dict)."""
    img, code, w, h, pitch = _image_args(img)
    t = np.empty((h, w), np.float64)
    lhat = np.empty((h, w), np.float64)
    rgb = np.empty((h, w, 3), np.float64)
    st = np.zeros(4, np.float64)
    rc = _load().ref_tonemap_colour_image(_ptr(img), code, w, h, pitch, beta_r, beta_k, eps,
                                          contrast, sigma_floor, saturation, _ptr(lhat), _ptr(t),
                                          _ptr(rgb), _ptr(st), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the image or the saturation")
    stats = {"mu": st[0], "sigma": st[1], "l_min": st[2], "l_max": st[3], "count": w * h}
    return rgb, t, lhat, stats


LTM_TILE, LTM_BINS = 64, 64


def tonemap_local(img, beta_r=0.55, beta_k=0.8, eps=1e-4, contrast=2.0, sigma_floor=1e-3,
                  strength=0.5, nthreads=1, sample=None):
    """Local tone map of one image (smoothed local histogram equalisation on a
    64-pixel tile grid, blended with the global curve): (T float64 HxW, stats),
    or T at the flat pixel indices ``sample`` only."""
    img, code, w, h, pitch = _image_args(img)
    idx = None if sample is None else np.ascontiguousarray(sample, np.int64)
    t = np.empty((h, w) if idx is None else idx.shape, np.float64)
    st = np.zeros(4, np.float64)
    rc = _load().ref_tonemap_local_image(_ptr(img), code, w, h, pitch, beta_r, beta_k, eps,
                                         contrast, sigma_floor, strength, _ptr(t), _ptr(st),
                                         int(nthreads), None if idx is None else _ptr(idx),
                                         0 if idx is None else idx.size)
    if rc != 0:
        raise ValueError("oracle rejected the image or the strength")
    return t, {"mu": st[0], "sigma": st[1], "l_min": st[2], "l_max": st[3], "count": w * h}


def recolour(img, lhat, t, saturation=1.0):
    """Colour output (float64 HxWx3) of any tone map from the image, its Lhat
    and its T: every channel min(1, T (C / Lhat)^s), grey T where Lhat == 0."""
    img, code, w, h, pitch = _image_args(img)
    lh = np.ascontiguousarray(lhat, np.float64)
    tt = np.ascontiguousarray(t, np.float64)
    if lh.shape != (h, w) or tt.shape != (h, w):
        raise ValueError("lhat and t must be HxW")
    rgb = np.empty((h, w, 3), np.float64)
    if _load().ref_recolour_image(_ptr(img), code, w, h, pitch, _ptr(lh), _ptr(tt), saturation,
                                  _ptr(rgb)):
        raise ValueError("oracle rejected the arguments")
    return rgb


def tonemap_local_colour(img, beta_r=0.55, beta_k=0.8, eps=1e-4, contrast=2.0, sigma_floor=1e-3,
                         strength=0.5, saturation=1.0, nthreads=1):
    """Colour output of the local tone map: (rgb float64 HxWx3, T HxW)."""
    t, _ = tonemap_local(img, beta_r, beta_k, eps, contrast, sigma_floor, strength, nthreads)
    lhat = decolorize(img, beta_r, beta_k, nthreads)
    return recolour(img, lhat, t, saturation), t
