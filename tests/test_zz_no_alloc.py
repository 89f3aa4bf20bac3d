"""GPU tests of dc_tonemap_global_noalloc, the global tone map (Sec. III-B.1)
for callers that cannot allocate: its workspace is the library's fixed
per-device scratch array. Every output must equal, bit for bit, what
dc_tonemap_global writes for the same call (the two share their kernels), on
two calls in a row with the second smaller (the scratch keeps the first call's
contents), and calls past the scratch's limits must be rejected before any
work. One image of each call is also checked against the FP64 oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f32, need_gpu, report, to_dev

pytestmark = pytest.mark.gpu
TM = dict(eps=1e-4, contrast=2.0, sigma_floor=1e-3)


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _images(dev, seed, shapes):
    """Mixed inputs: 8-bit, binary16 HDR and binary32, of the given shapes."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (h, w) in enumerate(shapes):
        k = i % 3
        if k == 0:
            img = synth.random_image(seed + i, h, w, np.uint8)
        elif k == 1:
            img = synth.hdr_pixels(rng, h, w)
        else:
            img = synth.random_image(seed + i, h, w, np.float32, scale=5.0)
        out.append(img)
    return out, [to_dev(a, dev) for a in out]


def _outputs(xs, colour_at=None):
    outs = []
    for i, x in enumerate(xs):
        h, w = x.shape[0], x.shape[1]
        shape = (h, w, 3) if i == colour_at else (h, w)
        outs.append(torch.full(shape, float("nan"), dtype=torch.float32, device=x.device))
    return outs


def _same(a, b, what):
    assert a.shape == b.shape, what
    eq = torch.equal(a.view(torch.uint8) if a.dtype == torch.uint8 else a.view(torch.int32),
                     b.view(torch.uint8) if b.dtype == torch.uint8 else b.view(torch.int32))
    assert eq, "%s differs from dc_tonemap_global" % what


def _call_pair(dev, imgs, xs, colour_at=None, saturation=1.0):
    n = len(xs)
    outs_ref = _outputs(xs, colour_at)
    lh_ref = [torch.full(x.shape[:2], float("nan"), dtype=torch.float32, device=dev) for x in xs]
    st_ref = torch.zeros((n, P.STATS_BYTES), dtype=torch.uint8, device=dev)
    P.tonemap_global(xs, outs=outs_ref, lhats=lh_ref, stats=st_ref, saturation=saturation, **TM)
    outs = _outputs(xs, colour_at)
    lh = [torch.full(x.shape[:2], float("nan"), dtype=torch.float32, device=dev) for x in xs]
    st = torch.full((n, P.STATS_BYTES), 0xAB, dtype=torch.uint8, device=dev)
    P.tonemap_global_noalloc(xs, outs, lhats=lh, stats=st, saturation=saturation, **TM)
    torch.cuda.synchronize()
    for i in range(n):
        _same(outs[i], outs_ref[i], "image %d output" % i)
        _same(lh[i], lh_ref[i], "image %d Lhat" % i)
    _same(st, st_ref, "statistics")
    return outs, st


def test_noalloc_equals_tonemap_global_twice(dev):
    shapes1 = [(512, 512), (300, 4099), (97, 131), (1, 1), (2048, 1024), (5, 7), (640, 480)]
    imgs1, xs1 = _images(dev, 11, shapes1)
    report("no-alloc call 1: %d images, %d px" % (len(xs1), sum(h * w for h, w in shapes1)))
    outs1, st1 = _call_pair(dev, imgs1, xs1, colour_at=2)
    t_ref, _, s_ref = oracle.tonemap(imgs1[0], **TM)
    check_f32(outs1[0].cpu().numpy(), t_ref, "no-alloc call 1, image 0 T vs oracle")
    s = P.stats_to_host(st1)[0]
    assert abs(s["mu"] - s_ref["mu"]) <= 2e-5 * (1 + abs(s_ref["mu"]))
    assert s["count"] == s_ref["count"]

    # Second call, smaller in every way: fewer images, fewer tiles, fewer
    # partials. The scratch still holds the first call's table and partials.
    shapes2 = [(64, 64), (33, 250), (256, 128)]
    imgs2, xs2 = _images(dev, 23, shapes2)
    report("no-alloc call 2: %d images, %d px" % (len(xs2), sum(h * w for h, w in shapes2)))
    outs2, st2 = _call_pair(dev, imgs2, xs2)
    t_ref, _, _ = oracle.tonemap(imgs2[1], **TM)
    check_f32(outs2[1].cpu().numpy(), t_ref, "no-alloc call 2, image 1 T vs oracle")


def test_noalloc_colour_power_and_u8(dev):
    imgs, xs = _images(dev, 5, [(200, 300), (128, 96)])
    _call_pair(dev, imgs, xs, colour_at=0, saturation=0.6)
    # 8-bit T outputs through both entry points
    o_ref = [torch.zeros(x.shape[:2], dtype=torch.uint8, device=dev) for x in xs]
    o = [torch.full(x.shape[:2], 7, dtype=torch.uint8, device=dev) for x in xs]
    P.tonemap_global(xs, outs=o_ref, want_stats=False, **TM)
    P.tonemap_global_noalloc(xs, o, **TM)
    torch.cuda.synchronize()
    for a, b in zip(o, o_ref):
        _same(a, b, "8-bit T")


def _status(fn_args):
    L = P.lib()
    ctx = P.context(fn_args[0].device)
    arr = P._image_array(*fn_args[1:])
    p = P._params(P.BETA_R, P.BETA_K)
    tm = P.DcTmParams(1e-4, 2.0, 1e-3, 1.0, 0.5)
    return L.dc_tonemap_global_noalloc(ctx.handle, arr, len(fn_args[1]), ctypes.byref(p),
                                       ctypes.byref(tm), None, None)


def test_noalloc_rejects_beyond_scratch(dev):
    L = P.lib()
    # More images than the scratch's table holds: 1025 one-pixel images
    # sharing one input, each writing its own element of one output buffer.
    x = torch.zeros((1, 1, 3), dtype=torch.uint8, device=dev)
    out = torch.zeros(1025, dtype=torch.float32, device=dev)
    xs = [x] * 1025
    outs = [out[i:i + 1].view(1, 1) for i in range(1025)]
    rc = _status((x, xs, outs, None))
    report("1025 images: status %d (%s)" % (rc, L.dc_last_error_message().decode()))
    assert rc == -1
    # More pixels than the partials fit: 20000 x 20000 8-bit (400 Mpx; the
    # buffers are real, so nothing could be read out of bounds).
    big = torch.zeros((20000, 20000, 3), dtype=torch.uint8, device=dev)
    big_out = torch.zeros((20000, 20000), dtype=torch.uint8, device=dev)
    rc = _status((big, [big], [big_out], None))
    report("400 Mpx: status %d (%s)" % (rc, L.dc_last_error_message().decode()))
    assert rc == -1
    torch.cuda.synchronize()
    assert int(big_out.max()) == 0  # nothing ran
    del big, big_out
    # The context and the scratch still work afterwards.
    imgs, xs2 = _images(dev, 3, [(40, 50)])
    _call_pair(dev, imgs, xs2)


def test_noalloc_headline_size(dev):
    """The largest workload the benchmark times, 16 x 4096^2 binary16, fits
    the scratch and matches dc_tonemap_global bit for bit."""
    rng = np.random.default_rng(99)
    img = synth.hdr_pixels(rng, 4096, 4096)
    x = to_dev(img, dev)
    xs = [x] * 16  # one input read by all 16 (inputs may be shared)
    o_ref = [torch.empty((4096, 4096), dtype=torch.float32, device=dev) for _ in xs]
    o = [torch.empty((4096, 4096), dtype=torch.float32, device=dev) for _ in xs]
    st_ref = torch.zeros((16, P.STATS_BYTES), dtype=torch.uint8, device=dev)
    st = torch.zeros((16, P.STATS_BYTES), dtype=torch.uint8, device=dev)
    P.tonemap_global(xs, outs=o_ref, stats=st_ref, **TM)
    P.tonemap_global_noalloc(xs, o, stats=st, **TM)
    torch.cuda.synchronize()
    for i in range(16):
        _same(o[i], o_ref[i], "4096^2 image %d" % i)
    _same(st, st_ref, "statistics")
    report("16 x 4096^2 binary16: bit-identical to dc_tonemap_global")
