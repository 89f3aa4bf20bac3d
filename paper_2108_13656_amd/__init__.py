"""Python binding of the MI355X decolorization library (``libdecolor.so``).

Argument marshalling only: every step of the path runs in the HIP kernels
behind the C ABI declared in ``include/decolor.h`` (Ambalathankandy et al.,
arXiv 2108.13656, Sec. II-B Eqs. (1)-(6) and the global tone map of
Sec. III-B.1). PyTorch supplies device memory and streams.

There is no CPU fallback: if the library has not been built, or no GPU is
present, every compute call raises.
"""
import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdecolor.so")

DC_OK = 0
DC_ERR_INVALID_ARG = -1
DC_ERR_UNSUPPORTED = -2
DC_ERR_ALIAS = -3
DC_ERR_NO_MEMORY = -4
DC_ERR_HIP = -5
DC_ERR_NO_DEVICE = -6
DC_ERR_CANCELLED = -7

DC_NONE, DC_U8, DC_F16, DC_F32 = -1, 0, 1, 2
_TORCH_TO_DC = {torch.uint8: DC_U8, torch.float16: DC_F16, torch.float32: DC_F32}

BETA_R = 0.55  # Eq. (3) weight chosen after Eq. (6)
BETA_K = 0.80  # Eq. (6) weight
TM_EPS, TM_CONTRAST, TM_SIGMA_FLOOR, TM_SATURATION = 1e-4, 2.0, 1e-3, 1.0
TM_LOCAL_STRENGTH = 0.5
DC_IMG_RGB_OUT = 1  # dc_image.flags: tone-map dst holds re-coloured RGB
DC_IMG_HOST_SRC = 2  # dc_image.flags, server requests: src is pinned host memory


class DcImage(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("dst2", ctypes.c_void_p),
                ("src_pitch", ctypes.c_int64), ("dst_pitch", ctypes.c_int64),
                ("dst2_pitch", ctypes.c_int64), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("src_dtype", ctypes.c_int32),
                ("dst_dtype", ctypes.c_int32), ("dst2_dtype", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class DcParams(ctypes.Structure):
    _fields_ = [("beta_r", ctypes.c_float), ("beta_k", ctypes.c_float)]


class DcTmParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("contrast", ctypes.c_float),
                ("sigma_floor", ctypes.c_float), ("saturation", ctypes.c_float),
                ("local_strength", ctypes.c_float)]


class DcStats(ctypes.Structure):
    _fields_ = [("log_mean", ctypes.c_float), ("log_std", ctypes.c_float),
                ("l_min", ctypes.c_float), ("l_max", ctypes.c_float), ("count", ctypes.c_int64)]


STATS_BYTES = ctypes.sizeof(DcStats)


class DcTuning(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int32 * 3), ("mixed_groups", ctypes.c_int32),
                ("decolor_grid_per_cu", ctypes.c_int32), ("mixed_grid_per_cu", ctypes.c_int32),
                ("pass1_grid_per_cu", ctypes.c_int32),
                ("pass2_grid_per_cu", ctypes.c_int32), ("tonemap_pipeline", ctypes.c_int32)]

    def as_dict(self):
        return {"groups": list(self.groups), "mixed_groups": self.mixed_groups,
                "decolor_grid_per_cu": self.decolor_grid_per_cu,
                "mixed_grid_per_cu": self.mixed_grid_per_cu,
                "pass1_grid_per_cu": self.pass1_grid_per_cu,
                "pass2_grid_per_cu": self.pass2_grid_per_cu,
                "tonemap_pipeline": self.tonemap_pipeline}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for i, g in enumerate(d["groups"]):
            t.groups[i] = g
        t.mixed_groups = d["mixed_groups"]
        t.decolor_grid_per_cu = d["decolor_grid_per_cu"]
        t.mixed_grid_per_cu = d.get("mixed_grid_per_cu", 0)
        t.pass1_grid_per_cu = d["pass1_grid_per_cu"]
        t.pass2_grid_per_cu = d["pass2_grid_per_cu"]
        t.tonemap_pipeline = d.get("tonemap_pipeline", 0)
        return t


PLAN_DECOLORIZE, PLAN_TONEMAP, PLAN_LOCAL, PLAN_GRAPH = 0, 1, 2, 1


class DcServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("params", DcParams), ("tm", DcTmParams)]


class DcRequest(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("img", DcImage)]


class DcCompletion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class DecolorError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (_status_string(status), status, message))
        self.status = status


_lib = None


def lib():
    """The loaded ``libdecolor.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdecolor.so is not built: run `python -m paper_2108_13656_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    img_p = ctypes.POINTER(DcImage)
    par_p = ctypes.POINTER(DcParams)
    tm_p = ctypes.POINTER(DcTmParams)
    L.dc_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    L.dc_destroy.argtypes = [vp]
    L.dc_validate.argtypes = [img_p, i32, par_p, tm_p]
    L.dc_decolorize.argtypes = [vp, img_p, par_p, vp]
    L.dc_decolorize_batch.argtypes = [vp, img_p, i32, par_p, vp]
    L.dc_tonemap_global.argtypes = [vp, img_p, i32, par_p, tm_p, vp, vp]
    L.dc_tonemap_local.argtypes = [vp, img_p, i32, par_p, tm_p, vp, vp]
    L.dc_tonemap_global_noalloc.argtypes = [vp, img_p, i32, par_p, tm_p, vp, vp]
    L.dc_status_string.argtypes = [ctypes.c_int]
    L.dc_status_string.restype = ctypes.c_char_p
    L.dc_last_error_message.argtypes = []
    L.dc_last_error_message.restype = ctypes.c_char_p
    L.dc_version.argtypes = []
    tun_p = ctypes.POINTER(DcTuning)
    L.dc_plan_create.argtypes = [vp, i32, img_p, i32, par_p, tm_p, vp, i32, ctypes.POINTER(vp)]
    L.dc_plan_run.argtypes = [vp, vp]
    L.dc_plan_destroy.argtypes = [vp]
    L.dc_get_tuning.argtypes = [vp, tun_p]
    L.dc_set_tuning.argtypes = [vp, tun_p]
    L.dc_autotune.argtypes = [vp, i32, img_p, i32, par_p, tm_p, vp, tun_p]
    req_p = ctypes.POINTER(DcRequest)
    comp_p = ctypes.POINTER(DcCompletion)
    L.dc_server_create.argtypes = [vp, ctypes.POINTER(DcServerConfig), ctypes.POINTER(vp)]
    L.dc_server_destroy.argtypes = [vp]
    L.dc_server_submit.argtypes = [vp, req_p, i32, ctypes.c_double]
    L.dc_server_step.argtypes = [vp]
    L.dc_server_poll.argtypes = [vp, comp_p, i32]
    L.dc_server_cancel.argtypes = [vp, ctypes.c_int64]
    L.dc_server_clock.argtypes = [vp]
    L.dc_server_clock.restype = ctypes.c_double
    L.dc_server_host_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
    L.dc_server_replay.argtypes = [vp, req_p, ctypes.POINTER(ctypes.c_double), i32, comp_p]
    L.dc_channel_batch.argtypes = [vp, img_p, i32, i32, vp]
    L.dc_decolorize_batch_betas.argtypes = [vp, img_p, i32, par_p, vp]
    L.dc_set_profiling.argtypes = [vp, ctypes.c_int]
    L.dc_last_timings.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
    for name in ("dc_create", "dc_destroy", "dc_validate", "dc_decolorize", "dc_decolorize_batch",
                 "dc_tonemap_global", "dc_version", "dc_set_profiling", "dc_last_timings",
                 "dc_plan_create", "dc_plan_run", "dc_plan_destroy", "dc_get_tuning",
                 "dc_set_tuning", "dc_autotune", "dc_server_create", "dc_server_destroy",
                 "dc_server_submit", "dc_server_step", "dc_server_poll", "dc_server_replay",
                 "dc_server_cancel",
                 "dc_channel_batch", "dc_decolorize_batch_betas", "dc_tonemap_local"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _status_string(status):
    try:
        return lib().dc_status_string(status).decode()
    except Exception:  # library missing while formatting an error
        return "status"


def _check(status):
    if status != DC_OK:
        raise DecolorError(status, lib().dc_last_error_message().decode())


class Context:
    """Owns one ``dc_ctx`` (workspace ring) on one device. A dc_ctx serves one
    host thread at a time and ctypes releases the GIL during a call, so every
    call that uses the context (directly, or through a plan or server made
    from it) holds ``lock``."""

    def __init__(self, device=None):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        self.lock = threading.RLock()
        self._h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(lib().dc_create(ctypes.byref(self._h), dev.index))

    @property
    def handle(self):
        return self._h

    def call(self, fn, *args):
        """fn(handle, *args) under the lock; raises DecolorError on failure."""
        with self.lock:
            _check(fn(self._h, *args))

    def close(self):
        with self.lock:
            if self._h:
                lib().dc_destroy(self._h)
                self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts = {}
_contexts_lock = threading.Lock()


def context(device=None):
    """The shared context of a device (created on first use; a new context
    takes the launch shapes of the tuning file named by ``DC_AUTOTUNE_CACHE``
    when that file was written for this device and library build)."""
    if device is None:
        idx = None
    elif isinstance(device, int):
        idx = device
    else:
        idx = torch.device(device).index
    if idx is None:
        idx = torch.cuda.current_device()
    created = False
    with _contexts_lock:
        if idx not in _contexts:
            _contexts[idx] = Context(idx)
            created = True
        ctx = _contexts[idx]
    if created:
        apply_tuning_cache(idx)
    return ctx


# ------------------------------------------------------------- marshalling

def _dc_dtype(t):
    try:
        return _TORCH_TO_DC[t]
    except KeyError:
        raise TypeError("unsupported dtype %s (uint8, float16, float32)" % t) from None


def _check_rgb(x):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if x.dim() != 3 or x.shape[2] != 3:
        raise ValueError("expected an HxWx3 interleaved RGB tensor, got %s" % (tuple(x.shape),))
    if x.stride(2) != 1 or x.stride(1) != 3 or x.stride(0) < 3 * x.shape[1]:
        raise ValueError("the W and channel axes must be packed (strides (pitch, 3, 1))")


def _check_gray(y, h, w, device):
    if y.dim() != 2 or tuple(y.shape) != (h, w) or y.device != device:
        raise ValueError("output must be an HxW tensor on the input's device")
    if y.stride(1) != 1 or y.stride(0) < w:
        raise ValueError("output rows must be packed (strides (pitch, 1))")


def _check_out(y, h, w, device):
    """HxW gray output, or HxWx3 colour output (tone map only)."""
    if y.dim() == 3:
        if tuple(y.shape) != (h, w, 3) or y.device != device:
            raise ValueError("colour output must be an HxWx3 tensor on the input's device")
        if y.stride(2) != 1 or y.stride(1) != 3 or y.stride(0) < 3 * w:
            raise ValueError("colour output must have strides (pitch, 3, 1)")
        return DC_IMG_RGB_OUT
    _check_gray(y, h, w, device)
    return 0


def _image(x, out, out2):
    h, w = x.shape[0], x.shape[1]
    d = DcImage()
    d.src = x.data_ptr()
    d.src_pitch = x.stride(0) * x.element_size()
    d.width, d.height = w, h
    d.src_dtype = _dc_dtype(x.dtype)
    flags = _check_out(out, h, w, x.device)
    d.dst = out.data_ptr()
    d.dst_pitch = out.stride(0) * out.element_size()
    d.dst_dtype = _dc_dtype(out.dtype)
    if out2 is None:
        d.dst2, d.dst2_pitch, d.dst2_dtype = None, 0, DC_NONE
    else:
        _check_gray(out2, h, w, x.device)
        d.dst2 = out2.data_ptr()
        d.dst2_pitch = out2.stride(0) * out2.element_size()
        d.dst2_dtype = _dc_dtype(out2.dtype)
    d.flags = flags
    return d


def _params(beta_r, beta_k):
    return DcParams(beta_r, beta_k)


def _stream_ptr(stream, device):
    s = torch.cuda.current_stream(device) if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _alloc(x, dtype, h, w, colour=False):
    return torch.empty((h, w, 3) if colour else (h, w), dtype=dtype, device=x.device)


# ------------------------------------------------------------- public API

def decolorize(x, out_dtype=torch.float32, out2_dtype=None, beta_r=BETA_R, beta_k=BETA_K,
               out=None, out2=None, stream=None):
    """Luminance of Eqs. (1)-(6) for one HxWx3 image.

    Returns the HxW output (Lhat as float, or its 8-bit / binary16 encoding),
    or (out, out2) when a second output is requested.
    """
    _check_rgb(x)
    h, w = x.shape[0], x.shape[1]
    out = _alloc(x, out_dtype, h, w) if out is None else out
    if out2 is None and out2_dtype is not None:
        out2 = _alloc(x, out2_dtype, h, w)
    d = _image(x, out, out2)
    p = _params(beta_r, beta_k)
    context(x.device).call(lib().dc_decolorize, ctypes.byref(d), ctypes.byref(p),
                           _stream_ptr(stream, x.device))
    return out if out2 is None else (out, out2)


def _image_array(xs, outs, outs2):
    arr = (DcImage * len(xs))()
    for i, x in enumerate(xs):
        _check_rgb(x)
        arr[i] = _image(x, outs[i], None if outs2 is None else outs2[i])
    return arr


def decolorize_batch(xs, out_dtype=torch.float32, out2_dtype=None, beta_r=BETA_R, beta_k=BETA_K,
                     outs=None, outs2=None, stream=None):
    """Decolorization of a list of images (any sizes, mixed input types) in one
    persistent launch. Returns a list of outputs (or of (out, out2) pairs)."""
    xs = list(xs)
    if not xs:
        return []
    dev = xs[0].device
    if outs is None:
        outs = [_alloc(x, out_dtype, x.shape[0], x.shape[1]) for x in xs]
    if outs2 is None and out2_dtype is not None:
        outs2 = [_alloc(x, out2_dtype, x.shape[0], x.shape[1]) for x in xs]
    arr = _image_array(xs, outs, outs2)
    p = _params(beta_r, beta_k)
    context(dev).call(lib().dc_decolorize_batch, arr, len(xs), ctypes.byref(p),
                      _stream_ptr(stream, dev))
    return outs if outs2 is None else list(zip(outs, outs2))


def decolorize_betas(xs, betas, out_dtype=torch.float32, outs=None, stream=None):
    """Decolorization of a list of images, image i with its own weights
    betas[i] = (beta_r, beta_k), in one persistent launch."""
    xs = list(xs)
    if len(betas) != len(xs):
        raise ValueError("one (beta_r, beta_k) pair per image")
    if not xs:
        return []
    dev = xs[0].device
    if outs is None:
        outs = [_alloc(x, out_dtype, x.shape[0], x.shape[1]) for x in xs]
    arr = _image_array(xs, outs, None)
    pa = (DcParams * len(xs))(*[DcParams(float(a), float(b)) for a, b in betas])
    context(dev).call(lib().dc_decolorize_batch_betas, arr, len(xs), pa, _stream_ptr(stream, dev))
    return outs


def beta_sweep(x, betas, out_dtype=torch.float32, out=None, stream=None):
    """L of one HxWx3 image for every (beta_r, beta_k) pair (the weight sweep of
    Fig. 4): an (n, H, W) tensor, one launch reading the shared input."""
    _check_rgb(x)
    h, w = x.shape[0], x.shape[1]
    if out is None:
        out = torch.empty((len(betas), h, w), dtype=out_dtype, device=x.device)
    decolorize_betas([x] * len(betas), betas, outs=list(out.unbind(0)), stream=stream)
    return out


CHANNELS = {"y601": 1, "hsv_v": 2, "cielab_l": 3}


def channel_batch(xs, channel, out_dtype=torch.float32, out2_dtype=None, outs=None, outs2=None,
                  stream=None):
    """Comparator gray channel ('y601', 'hsv_v' or 'cielab_l' = L*/100) of a
    list of images, on the same data path as the decolorization."""
    xs = list(xs)
    if not xs:
        return []
    dev = xs[0].device
    if outs is None:
        outs = [_alloc(x, out_dtype, x.shape[0], x.shape[1]) for x in xs]
    if outs2 is None and out2_dtype is not None:
        outs2 = [_alloc(x, out2_dtype, x.shape[0], x.shape[1]) for x in xs]
    arr = _image_array(xs, outs, outs2)
    context(dev).call(lib().dc_channel_batch, arr, len(xs), CHANNELS[channel],
                      _stream_ptr(stream, dev))
    return outs if outs2 is None else list(zip(outs, outs2))


def _stats_ptr(stats, n, dev):
    """Device address of a caller's statistics tensor, after checking that the
    kernels can write n entries of STATS_BYTES there: a contiguous tensor on
    the images' device holding at least n * STATS_BYTES bytes. None gives 0
    (no statistics)."""
    if stats is None:
        return ctypes.c_void_p(0)
    if not isinstance(stats, torch.Tensor):
        raise ValueError("stats must be a torch tensor")
    if stats.device != dev:
        raise ValueError("stats must be on %s (the images' device), not %s" % (dev, stats.device))
    if not stats.is_contiguous():
        raise ValueError("stats must be contiguous")
    have = stats.numel() * stats.element_size()
    if have < n * STATS_BYTES:
        raise ValueError("stats holds %d bytes; %d images need %d" % (have, n, n * STATS_BYTES))
    return ctypes.c_void_p(stats.data_ptr())


def tonemap_global(xs, out_dtype=torch.float32, lhat_dtype=None, beta_r=BETA_R, beta_k=BETA_K,
                   eps=TM_EPS, contrast=TM_CONTRAST, sigma_floor=TM_SIGMA_FLOOR, outs=None,
                   lhats=None, stats=None, want_stats=True, stream=None, colour=False,
                   saturation=TM_SATURATION):
    """Global tone map (Sec. III-B.1, centred sigmoid on ln(Lhat + eps)) of a
    list of images. Returns (outputs, Lhat outputs or None, stats) where stats
    is a uint8 device tensor of n x 24 bytes (see ``stats_to_host``). Outputs
    are HxW T, or HxWx3 re-coloured RGB min(1, T (C / Lhat)^saturation) with
    colour=True (given ``outs`` may mix both shapes)."""
    return _tonemap_global(lib().dc_tonemap_global, xs, out_dtype, lhat_dtype, beta_r, beta_k,
                           eps, contrast, sigma_floor, outs, lhats, stats, want_stats, stream,
                           colour, saturation)


def tonemap_global_noalloc(xs, outs, lhats=None, stats=None, beta_r=BETA_R, beta_k=BETA_K,
                           eps=TM_EPS, contrast=TM_CONTRAST, sigma_floor=TM_SIGMA_FLOOR,
                           stream=None, saturation=TM_SATURATION):
    """``tonemap_global`` through dc_tonemap_global_noalloc, the entry point
    that allocates nothing (its workspace is the library's fixed per-device
    scratch array). The caller passes every output (``outs``, optional
    ``lhats`` and ``stats``); nothing is allocated here either. Returns
    (outs, lhats, stats)."""
    xs = list(xs)
    if outs is None or len(outs) != len(xs):
        raise ValueError("tonemap_global_noalloc needs one given output per image")
    if not xs:
        return [], lhats, stats
    return _tonemap_global(lib().dc_tonemap_global_noalloc, xs, None, None, beta_r, beta_k, eps,
                           contrast, sigma_floor, outs, lhats, stats, False, stream, False,
                           saturation)


def _tonemap_global(fn, xs, out_dtype, lhat_dtype, beta_r, beta_k, eps, contrast, sigma_floor,
                    outs, lhats, stats, want_stats, stream, colour, saturation):
    xs = list(xs)
    if not xs:
        return [], None, None
    dev = xs[0].device
    if outs is None:
        outs = [_alloc(x, out_dtype, x.shape[0], x.shape[1], colour) for x in xs]
    if lhats is None and lhat_dtype is not None:
        lhats = [_alloc(x, lhat_dtype, x.shape[0], x.shape[1]) for x in xs]
    if stats is None and want_stats:
        stats = torch.empty((len(xs), STATS_BYTES), dtype=torch.uint8, device=dev)
    arr = _image_array(xs, outs, lhats)
    p = _params(beta_r, beta_k)
    tm = DcTmParams(eps, contrast, sigma_floor, saturation, TM_LOCAL_STRENGTH)
    context(dev).call(fn, arr, len(xs), ctypes.byref(p), ctypes.byref(tm),
                      _stats_ptr(stats, len(xs), dev), _stream_ptr(stream, dev))
    return outs, lhats, stats


def tonemap_local(xs, out_dtype=torch.float32, lhat_dtype=None, beta_r=BETA_R, beta_k=BETA_K,
                  eps=TM_EPS, contrast=TM_CONTRAST, sigma_floor=TM_SIGMA_FLOOR,
                  strength=TM_LOCAL_STRENGTH, outs=None, lhats=None, stats=None, want_stats=True,
                  stream=None, colour=False, saturation=TM_SATURATION):
    """Local tone map (Sec. III-B.2: smoothed local histogram equalisation on
    64-pixel tiles, blended with the global curve by ``strength``) of a list of
    images. Returns (outputs, Lhat outputs or None, stats) as ``tonemap_global``;
    colour=True (or HxWx3 ``outs``) gives the re-coloured RGB."""
    xs = list(xs)
    if not xs:
        return [], None, None
    dev = xs[0].device
    if outs is None:
        outs = [_alloc(x, out_dtype, x.shape[0], x.shape[1], colour) for x in xs]
    if lhats is None and lhat_dtype is not None:
        lhats = [_alloc(x, lhat_dtype, x.shape[0], x.shape[1]) for x in xs]
    if stats is None and want_stats:
        stats = torch.empty((len(xs), STATS_BYTES), dtype=torch.uint8, device=dev)
    arr = _image_array(xs, outs, lhats)
    p = _params(beta_r, beta_k)
    tm = DcTmParams(eps, contrast, sigma_floor, saturation, strength)
    context(dev).call(lib().dc_tonemap_local, arr, len(xs), ctypes.byref(p), ctypes.byref(tm),
                      _stats_ptr(stats, len(xs), dev), _stream_ptr(stream, dev))
    return outs, lhats, stats


def stats_to_host(stats):
    """List of dicts (log_mean, log_std, l_min, l_max, count) from the device
    statistics tensor returned by ``tonemap_global``."""
    raw = stats.cpu().contiguous()
    f = raw[:, :16].contiguous().view(torch.float32)
    c = raw[:, 16:24].contiguous().view(torch.int64)
    return [{"mu": float(f[i, 0]), "sigma": float(f[i, 1]), "l_min": float(f[i, 2]),
             "l_max": float(f[i, 3]), "count": int(c[i, 0])} for i in range(raw.shape[0])]


def validate(images, beta_r=BETA_R, beta_k=BETA_K, tm=None):
    """Host-only check of DcImage descriptors (no GPU needed). Returns the status."""
    arr = (DcImage * len(images))(*images) if images else None
    p = _params(beta_r, beta_k)
    if tm is not None:
        tm = tuple(tm) + (TM_SATURATION, TM_LOCAL_STRENGTH)[len(tm) - 3:]
    tmp = DcTmParams(*tm) if tm is not None else None
    return lib().dc_validate(arr, len(images), ctypes.byref(p),
                             ctypes.byref(tmp) if tmp is not None else None)


class Plan:
    """A frozen batched decolorization or tone map over fixed buffers
    (``dc_plan_*``): the descriptor table is uploaded once, and ``run()``
    enqueues only the kernels (or replays a captured HIP graph)."""

    def __init__(self, kind, xs, outs, outs2=None, beta_r=BETA_R, beta_k=BETA_K, eps=TM_EPS,
                 contrast=TM_CONTRAST, sigma_floor=TM_SIGMA_FLOOR, stats=None, graph=False,
                 saturation=TM_SATURATION, local_strength=TM_LOCAL_STRENGTH):
        xs = list(xs)
        self.device = xs[0].device
        self._keep = (xs, list(outs), None if outs2 is None else list(outs2), stats)
        arr = _image_array(xs, list(outs), None if outs2 is None else list(outs2))
        p = _params(beta_r, beta_k)
        tm = (DcTmParams(eps, contrast, sigma_floor, saturation, local_strength)
              if kind in (PLAN_TONEMAP, PLAN_LOCAL) else None)
        self._h = ctypes.c_void_p()
        self._ctx = context(self.device)
        self._ctx.call(lib().dc_plan_create, kind, arr, len(xs), ctypes.byref(p),
                       ctypes.byref(tm) if tm is not None else None,
                       _stats_ptr(stats, len(xs), self.device),
                       PLAN_GRAPH if graph else 0, ctypes.byref(self._h))

    def run(self, stream=None):
        with self._ctx.lock:
            _check(lib().dc_plan_run(self._h, _stream_ptr(stream, self.device)))

    def close(self):
        if self._h:
            with self._ctx.lock:
                lib().dc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_request(rid, src, src_dtype, width, height, src_pitch, dst_dtype, dst=None, dst_pitch=0,
                 flags=0):
    """A DcRequest for a device image given by raw pointer (dst None: the
    server allocates and frees the output; flags DC_IMG_RGB_OUT asks for the
    re-coloured RGB)."""
    r = DcRequest()
    r.id = rid
    r.img.src = src
    r.img.src_pitch = src_pitch
    r.img.width, r.img.height = width, height
    r.img.src_dtype = src_dtype
    r.img.dst = dst
    r.img.dst_pitch = dst_pitch
    r.img.dst_dtype = dst_dtype
    r.img.dst2, r.img.dst2_pitch, r.img.dst2_dtype, r.img.flags = None, 0, DC_NONE, flags
    return r


def request_for(rid, x, out=None, out_dtype=torch.float32, colour=False):
    """A DcRequest for an HxWx3 tensor (and an optional HxW, or with colour
    HxWx3, device output). x is a device tensor, or a pinned host tensor that
    the server copies to the device itself."""
    host = isinstance(x, torch.Tensor) and not x.is_cuda
    if host:
        if not x.is_pinned():
            raise ValueError("host inputs must be pinned (pin_memory=True)")
        if x.dim() != 3 or x.shape[2] != 3 or x.stride(2) != 1 or x.stride(1) != 3:
            raise ValueError("expected an HxWx3 interleaved RGB tensor")
    else:
        _check_rgb(x)
    flags = (DC_IMG_RGB_OUT if colour else 0) | (DC_IMG_HOST_SRC if host else 0)
    if out is not None:
        flags = _check_out(out, x.shape[0], x.shape[1], out.device) | (
            DC_IMG_HOST_SRC if host else 0)
    return make_request(rid, x.data_ptr(), _dc_dtype(x.dtype), x.shape[1], x.shape[0],
                        x.stride(0) * x.element_size(),
                        _dc_dtype(out.dtype if out is not None else out_dtype),
                        None if out is None else out.data_ptr(),
                        0 if out is None else out.stride(0) * out.element_size(), flags)


class Server:
    """Continuous-batching tone-map server (``dc_server_*``)."""

    def __init__(self, budget_bytes, max_batch=64, max_inflight=4, beta_r=BETA_R, beta_k=BETA_K,
                 eps=TM_EPS, contrast=TM_CONTRAST, sigma_floor=TM_SIGMA_FLOOR, device=None,
                 saturation=TM_SATURATION):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device if isinstance(device, torch.device) else torch.device("cuda", device)
        cfg = DcServerConfig(budget_bytes, max_batch, max_inflight, 0, DcParams(beta_r, beta_k),
                             DcTmParams(eps, contrast, sigma_floor, saturation,
                                        TM_LOCAL_STRENGTH))
        self._h = ctypes.c_void_p()
        self._ctx = context(self.device)
        self._ctx.call(lib().dc_server_create, ctypes.byref(cfg), ctypes.byref(self._h))

    def submit(self, reqs, t_submit=-1.0):
        arr = (DcRequest * len(reqs))(*reqs)
        with self._ctx.lock:
            _check(lib().dc_server_submit(self._h, arr, len(reqs), t_submit))

    def step(self):
        with self._ctx.lock:
            n = lib().dc_server_step(self._h)
            if n < 0:
                _check(n)
        return n

    def poll(self, cap=4096):
        buf = (DcCompletion * cap)()
        with self._ctx.lock:
            n = lib().dc_server_poll(self._h, buf, cap)
            if n < 0:
                _check(n)
        return [buf[i] for i in range(n)]

    def cancel(self, rid):
        """Cancels request rid if it is still queued (not launched); True if
        it was. It then completes with status DC_ERR_CANCELLED."""
        with self._ctx.lock:
            n = lib().dc_server_cancel(self._h, rid)
            if n < 0:
                _check(n)
        return n == 1

    def clock(self):
        return lib().dc_server_clock(self._h)

    def host_stats(self):
        """(seconds of host time spent enqueueing launches, number of launches)
        since the server was created."""
        sec, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().dc_server_host_stats(self._h, ctypes.byref(sec), ctypes.byref(n)))
        return sec.value, n.value

    def replay(self, reqs, arrivals):
        """Replays a trace natively; returns the completions in finishing order."""
        n = len(reqs)
        arr = (DcRequest * n)(*reqs)
        times = (ctypes.c_double * n)(*arrivals)
        out = (DcCompletion * n)()
        with self._ctx.lock:
            _check(lib().dc_server_replay(self._h, arr, times, n, out))
        return [out[i] for i in range(n)]

    def close(self):
        if self._h:
            with self._ctx.lock:
                lib().dc_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def get_tuning(device=None):
    t = DcTuning()
    context(device).call(lib().dc_get_tuning, ctypes.byref(t))
    return t.as_dict()


def set_tuning(d, device=None):
    t = DcTuning.from_dict(d)
    context(device).call(lib().dc_set_tuning, ctypes.byref(t))


# ------------------------------------------------------------- tuning cache
#
# A tuning file records the launch shapes together with what they were
# measured on: the device's name and the SHA-256 of the built library. A file
# from another device or another build is ignored rather than applied.

TUNING_CACHE_VERSION = 1


def library_sha256():
    import hashlib
    with open(LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def tuning_record(tuning, device_name, lib_sha):
    """The JSON-ready record of a tuning dict for a device and library build."""
    return {"version": TUNING_CACHE_VERSION, "device": device_name, "library_sha256": lib_sha,
            "tuning": dict(tuning)}


def tuning_from_record(record, device_name, lib_sha):
    """The tuning dict of a record when it was made for this device and
    library build, else None."""
    try:
        if (record.get("version") == TUNING_CACHE_VERSION and record.get("device") == device_name
                and record.get("library_sha256") == lib_sha):
            t = record["tuning"]
            DcTuning.from_dict(t)  # every field present
            return dict(t)
    except (AttributeError, KeyError, TypeError, ValueError):
        pass
    return None


def save_tuning(path, device=None):
    """Writes the context's current launch shapes to a tuning file."""
    import json
    idx = context(device).device.index
    rec = tuning_record(get_tuning(idx), torch.cuda.get_device_name(idx), library_sha256())
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)


def load_tuning(path, device=None):
    """Applies a tuning file if it was written for this device and library
    build; returns whether it did."""
    import json
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return False
    idx = context(device).device.index
    t = tuning_from_record(rec, torch.cuda.get_device_name(idx), library_sha256())
    if t is None:
        return False
    set_tuning(t, idx)
    return True


TUNING_CACHE_ENV = "DC_AUTOTUNE_CACHE"


def apply_tuning_cache(device=None):
    """Applies the tuning file named by ``DC_AUTOTUNE_CACHE``, if set and made
    for this device and library build; returns whether it did."""
    path = os.environ.get(TUNING_CACHE_ENV)
    return bool(path) and load_tuning(path, device)


def autotune(kind, xs, outs, outs2=None, beta_r=BETA_R, beta_k=BETA_K, eps=TM_EPS,
             contrast=TM_CONTRAST, sigma_floor=TM_SIGMA_FLOOR, stream=None,
             saturation=TM_SATURATION):
    """Runs the library's launch-shape search on these buffers and returns the
    tuning it kept (a dict, see ``get_tuning``). With ``DC_AUTOTUNE_CACHE``
    set, the context's shapes are then written to that file."""
    xs = list(xs)
    dev = xs[0].device
    arr = _image_array(xs, list(outs), None if outs2 is None else list(outs2))
    p = _params(beta_r, beta_k)
    tm = DcTmParams(eps, contrast, sigma_floor, saturation, TM_LOCAL_STRENGTH)
    t = DcTuning()
    context(dev).call(lib().dc_autotune, kind, arr, len(xs), ctypes.byref(p), ctypes.byref(tm),
                      _stream_ptr(stream, dev), ctypes.byref(t))
    path = os.environ.get(TUNING_CACHE_ENV)
    if path:
        save_tuning(path, dev)
    return t.as_dict()


def set_profiling(on, device=None):
    """Records per-kernel timing events on later calls of this device's context."""
    context(device).call(lib().dc_set_profiling, 1 if on else 0)


def last_timings(device=None, cap=8):
    """Per-kernel durations (ms) of the most recent profiled call."""
    buf = (ctypes.c_float * cap)()
    ctx = context(device)
    with ctx.lock:
        n = lib().dc_last_timings(ctx.handle, buf, cap)
        if n < 0:
            _check(n)
    return [float(buf[i]) for i in range(n)]


def last_error():
    return lib().dc_last_error_message().decode()
