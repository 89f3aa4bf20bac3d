"""Guard bands around every output: each output is a view into a larger buffer
whose bytes before, after and between the rows hold a sentinel; after every
entry point has run on ragged shapes (partial tiles, odd widths, single rows
and columns, both walks), the sentinels must be intact and every float output
element must have been written. Out-of-range writes stay inside the buffer,
so the check is safe to run."""
import numpy as np
import pytest
import torch

import paper_2108_13656_amd as P
import synth
from gpuhelp import need_gpu, to_dev

pytestmark = pytest.mark.gpu
SHAPES = [(1, 1), (1, 4099), (4099, 1), (3, 5), (63, 65), (65, 63), (129, 257), (64, 64)]
GUARD = 4096  # elements of sentinel before and after each view


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _guarded(h, w, ch, dtype, dev, pad):
    """A view of h x w (x ch) with `pad` extra elements per row, inside a
    buffer with GUARD sentinel elements on both sides; returns (buf, view, mask)
    where mask marks the view's elements."""
    row = (w + pad) * ch
    n = GUARD + h * row + GUARD
    sentinel = 77 if dtype == torch.uint8 else -12345.0
    buf = torch.full((n,), sentinel, dtype=dtype, device=dev)
    body = buf[GUARD:GUARD + h * row].view(h, w + pad, ch)[:, :w]
    view = body if ch == 3 else body[..., 0]
    mask = torch.zeros(n, dtype=torch.bool, device=dev)
    mask[GUARD:GUARD + h * row].view(h, w + pad, ch)[:, :w] = True
    return buf, view, mask, sentinel


def _check(buf, mask, sentinel, what):
    outside = buf[~mask]
    assert bool((outside == sentinel).all()), "%s: write outside the output" % what
    if buf.dtype != torch.uint8:  # no output is negative; an 8-bit code may equal the sentinel
        inside = buf[mask]
        assert not bool((inside == sentinel).any()), "%s: output element left unwritten" % what


def _image(kind, h, w, seed):
    rng = np.random.default_rng(seed)
    if kind == "u8":
        return synth.sdr_pixels(rng, h, w)
    return synth.hdr_pixels(rng, h, w)


@pytest.mark.parametrize("kind", ["u8", "f16"])
@pytest.mark.parametrize("pad", [0, 3])
def test_outputs_stay_in_bounds(dev, kind, pad):
    for i, (h, w) in enumerate(SHAPES):
        x = to_dev(_image(kind, h, w, 1000 + i), dev)
        cases = []
        for dt in (torch.uint8, torch.float16, torch.float32):
            b1, o1, m1, s1 = _guarded(h, w, 1, dt, dev, pad)
            b2, o2, m2, s2 = _guarded(h, w, 1, torch.float32, dev, pad)
            P.decolorize(x, out=o1, out2=o2)
            cases += [(b1, m1, s1, "decolorize %s" % dt), (b2, m2, s2, "decolorize lhat")]
            b, o, m, s = _guarded(h, w, 1, dt, dev, pad)
            P.decolorize_betas([x], [(0.7, 0.6)], outs=[o])
            cases.append((b, m, s, "betas %s" % dt))
            sweep = [_guarded(h, w, 1, dt, dev, pad) for _ in range(3)]
            P.decolorize_betas([x] * 3, [(0.7, 0.6), (0.1, 0.9), (1.0, 0.0)],
                               outs=[g[1] for g in sweep])
            cases += [(g[0], g[2], g[3], "sweep %s" % dt) for g in sweep]
            b, o, m, s = _guarded(h, w, 1, dt, dev, pad)
            P.channel_batch([x], "cielab_l", outs=[o])
            cases.append((b, m, s, "channel %s" % dt))
            for colour in (False, True):
                ch = 3 if colour else 1
                b, o, m, s = _guarded(h, w, ch, dt, dev, pad)
                bl, ol, ml, sl = _guarded(h, w, 1, torch.float32, dev, pad)
                P.tonemap_global([x], outs=[o], lhats=[ol], saturation=0.7)
                cases += [(b, m, s, "global %s colour=%s" % (dt, colour)), (bl, ml, sl, "global lhat")]
                b, o, m, s = _guarded(h, w, ch, dt, dev, pad)
                bl, ol, ml, sl = _guarded(h, w, 1, torch.float32, dev, pad)
                P.tonemap_local([x], outs=[o], lhats=[ol], saturation=0.7)
                cases += [(b, m, s, "local %s colour=%s" % (dt, colour)), (bl, ml, sl, "local lhat")]
        torch.cuda.synchronize()
        for b, m, s, what in cases:
            _check(b, m, s, "%s %dx%d %s pad=%d" % (kind, h, w, what, pad))
