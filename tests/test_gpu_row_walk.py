"""GPU tests of the row walk: a pitched image (rows further apart than their
bytes: crops, padded rows, any element-aligned offset) is tiled like a packed
one over its W x H pixels in row-major order, with the row breaks placed per
unit. Every per-pixel result and every statistic is therefore the same, bit for
bit, as for a packed copy of the same pixels, which these tests assert for the
decolorization (Sec. II-B, Eqs. (1)-(6)), the global tone map (Sec. III-B.1)
with gray and colour output, and the comparator channels; widths that are not
a multiple of a unit's pixels (units split by a row break), tiles that span
many short rows, odd row paddings and unaligned bases are all covered, and the
rows' padding must be left untouched. One image per case is also checked
against the FP64 oracle, and widths past the row walk's range fall back to the
per-pixel walk."""
import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f32, need_gpu, report, to_dev

pytestmark = pytest.mark.gpu
TM = dict(eps=1e-4, contrast=2.0, sigma_floor=1e-3)
SENT = {torch.uint8: 77, torch.float16: -1234.0, torch.float32: -12345.0}


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _pixels(kind, h, w, seed):
    rng = np.random.default_rng(seed)
    if kind == "u8":
        return synth.sdr_pixels(rng, h, w)
    if kind == "f16":
        return synth.hdr_pixels(rng, h, w)
    return synth.random_image(seed, h, w, np.float32, scale=3.0)


def _pitched_input(img, pad, off, dev):
    """The image as an h x w x 3 view whose rows are w + pad pixels apart,
    starting `off` elements into its buffer (pad and off in elements)."""
    h, w, _ = img.shape
    t = torch.from_numpy(img).to(dev)
    pitch = 3 * w + pad
    buf = torch.zeros(off + h * pitch + 16, dtype=t.dtype, device=dev)
    view = buf[off:off + h * pitch].view(h, pitch)[:, :3 * w].view(h, w, 3)
    view.copy_(t)
    return view


def _pitched_output(h, w, ch, dtype, pad, off, dev):
    """An output view with `pad` extra elements per row and `off` leading
    elements, in a buffer full of a sentinel; returns (buf, view, mask)."""
    pitch = ch * w + pad
    n = off + h * pitch + 64
    buf = torch.full((n,), SENT[dtype], dtype=dtype, device=dev)
    body = buf[off:off + h * pitch].view(h, pitch)[:, :ch * w]
    view = body.view(h, w, 3) if ch == 3 else body
    mask = torch.zeros(n, dtype=torch.bool, device=dev)
    mask[off:off + h * pitch].view(h, pitch)[:, :ch * w] = True
    return buf, view, mask


def _untouched(buf, mask, dtype, what):
    assert bool((buf[~mask] == SENT[dtype]).all()), "%s: write outside the view" % what


def _same(a, b, what):
    a = a.contiguous()
    b = b.contiguous()
    if a.dtype == torch.uint8:
        ok = torch.equal(a, b)
    else:
        ok = torch.equal(a.view(torch.int16 if a.element_size() == 2 else torch.int32),
                         b.view(torch.int16 if b.element_size() == 2 else torch.int32))
    assert ok, "%s differs from the packed copy" % what


# (width, height, input pad in elements, input offset in elements)
CASES = [(4, 5, 3, 0), (5, 9, 1, 1), (6, 7, 2, 3), (7, 33, 5, 2), (13, 300, 9, 5),
         (255, 40, 33, 7), (1001, 19, 47, 1), (4097, 3, 12, 4), (5000, 6, 3000, 0)]


@pytest.mark.parametrize("kind", ["u8", "f16", "f32"])
def test_decolorize_pitched_equals_packed(dev, kind):
    for i, (w, h, pad, off) in enumerate(CASES):
        img = _pixels(kind, h, w, 100 + i)
        xp = to_dev(img, dev)
        xv = _pitched_input(img, pad, off, dev)
        for dt in (torch.float32, torch.uint8, torch.float16):
            want = P.decolorize(xp, out_dtype=dt)
            buf, view, mask = _pitched_output(h, w, 1, dt, pad=3 + i, off=i % 3, dev=dev)
            P.decolorize(xv, out=view)
            torch.cuda.synchronize()
            what = "%s %dx%d pad %d off %d -> %s" % (kind, w, h, pad, off, dt)
            _same(view, want, what)
            _untouched(buf, mask, dt, what)
        if i in (3, 6):
            check_f32(P.decolorize(xv).cpu().numpy(), oracle.decolorize(img),
                      "%s %dx%d pitched vs oracle" % (kind, w, h), rel=(kind != "u8"))


@pytest.mark.parametrize("kind", ["u8", "f16", "f32"])
def test_batch_of_pitched_and_packed_images(dev, kind):
    """One batch mixing packed and pitched images (two launches, one per walk):
    every image bit-identical to its packed single call."""
    xs, wants = [], []
    for i, (w, h, pad, off) in enumerate(CASES):
        img = _pixels(kind, h, w, 200 + i)
        xp = to_dev(img, dev)
        wants.append(P.decolorize(xp))
        xs.append(xp if i % 2 else _pitched_input(img, pad, off, dev))
    got = P.decolorize_batch(xs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(got, wants)):
        _same(a, b, "batch image %d" % i)


@pytest.mark.parametrize("kind", ["u8", "f16", "f32"])
def test_tonemap_pitched_equals_packed(dev, kind):
    """Statistics chunks of a pitched image are the packed image's, so T and
    the statistics are bit-identical; gray and colour outputs, and a batch that
    mixes both walks."""
    xs_p, xs_v, imgs = [], [], []
    for i, (w, h, pad, off) in enumerate(CASES):
        img = _pixels(kind, h, w, 300 + i)
        imgs.append(img)
        xs_p.append(to_dev(img, dev))
        xs_v.append(_pitched_input(img, pad, off, dev))
    want, _, want_st = P.tonemap_global(xs_p, **TM)
    outs, bufs = [], []
    for i, x in enumerate(xs_v):
        h, w = x.shape[:2]
        buf, view, mask = _pitched_output(h, w, 1, torch.float32, pad=5 + i, off=1 + i % 2,
                                          dev=dev)
        outs.append(view)
        bufs.append((buf, mask))
    mixed = [xs_v[i] if i % 2 == 0 else xs_p[i] for i in range(len(xs_v))]
    _, _, st = P.tonemap_global(mixed, outs=outs, **TM)
    torch.cuda.synchronize()
    for i in range(len(outs)):
        _same(outs[i], want[i], "%s tone map image %d" % (kind, i))
        _untouched(bufs[i][0], bufs[i][1], torch.float32, "tone map image %d" % i)
    _same(st, want_st, "%s statistics" % kind)
    t_ref, _, _ = oracle.tonemap(imgs[6], **TM)
    check_f32(outs[6].cpu().numpy(), t_ref, "%s pitched tone map vs oracle" % kind)
    # colour output into pitched 8-bit RGB rows
    for sat in (1.0, 0.6):
        want_c, _, _ = P.tonemap_global(xs_p, out_dtype=torch.uint8, colour=True,
                                        saturation=sat, **TM)
        outs_c, bufs_c = [], []
        for i, x in enumerate(xs_v):
            h, w = x.shape[:2]
            buf, view, mask = _pitched_output(h, w, 3, torch.uint8, pad=7, off=i % 4, dev=dev)
            outs_c.append(view)
            bufs_c.append((buf, mask))
        P.tonemap_global(xs_v, outs=outs_c, saturation=sat, **TM)
        torch.cuda.synchronize()
        for i in range(len(outs_c)):
            _same(outs_c[i], want_c[i], "%s colour s=%g image %d" % (kind, sat, i))
            _untouched(bufs_c[i][0], bufs_c[i][1], torch.uint8, "colour image %d" % i)


@pytest.mark.parametrize("channel", ["y601", "hsv_v", "cielab_l"])
def test_channels_pitched_equals_packed(dev, channel):
    for i, (w, h, pad, off) in enumerate(CASES[:7]):
        img = _pixels("u8", h, w, 400 + i)
        want = P.channel_batch([to_dev(img, dev)], channel)[0]
        got = P.channel_batch([_pitched_input(img, pad, off, dev)], channel)[0]
        torch.cuda.synchronize()
        _same(got, want, "%s %dx%d" % (channel, w, h))


def test_weight_sweep_pitched_equals_packed(dev):
    w, h = 1001, 37
    img = _pixels("u8", h, w, 7)
    betas = [(0.55, 0.8), (0.7, 0.5), (0.5, 0.95)]
    want = P.beta_sweep(to_dev(img, dev), betas)
    got = P.beta_sweep(_pitched_input(img, 11, 3, dev), betas)
    torch.cuda.synchronize()
    for k in range(len(betas)):
        _same(got[k], want[k], "sweep pair %d" % k)


def test_wide_rows_take_the_per_pixel_walk(dev):
    """Past the row walk's width (46000 px) a pitched image is walked row by
    row, pixel by pixel: still the packed copy's per-pixel values, and the
    tone map within the tolerance."""
    w, h = 46005, 3
    img = _pixels("u8", h, w, 9)
    xp = to_dev(img, dev)
    xv = _pitched_input(img, 5, 1, dev)
    _same(P.decolorize(xv), P.decolorize(xp), "wide pitched decolorize")
    t_ref, _, _ = oracle.tonemap(img, **TM)
    outs, _, _ = P.tonemap_global([xv], **TM)
    check_f32(outs[0].cpu().numpy(), t_ref, "wide pitched tone map vs oracle")
    report("46005-px rows: per-pixel walk matches")


@pytest.mark.parametrize("kind", ["u8", "f16", "f32"])
def test_packed_rows_at_any_element_offset(dev, kind):
    """Packed rows (pitch = row bytes) whose first byte is not 4-byte aligned
    take the row walk with zero gaps, whose tiles, units and addresses are the
    packed walk's: decolorization, T and the statistics are the aligned copy's
    bits, for every width (below 4 and single rows included)."""
    shapes = [(1, 9), (2, 3), (5, 4), (7, 1001), (3, 4097), (40, 257)]
    for i, (h, w) in enumerate(shapes):
        img = _pixels(kind, h, w, 500 + i)
        xp = to_dev(img, dev)
        for off in (1, 2, 3):
            xv = _pitched_input(img, 0, off, dev)
            what = "%s %dx%d at element offset %d" % (kind, w, h, off)
            _same(P.decolorize(xv), P.decolorize(xp), what)
            _same(P.decolorize(xv, out_dtype=torch.uint8), P.decolorize(xp, out_dtype=torch.uint8),
                  what + " u8")
            tv, _, sv = P.tonemap_global([xv], **TM)
            tp, _, sp = P.tonemap_global([xp], **TM)
            torch.cuda.synchronize()
            _same(tv[0], tp[0], what + " T")
            _same(sv, sp, what + " statistics")
    report("packed rows at element offsets 1-3 match the aligned copies")
