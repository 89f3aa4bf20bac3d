"""GPU parity of the local tone map (dc_tonemap_local: smoothed local histogram
equalisation on 64 x 64-pixel tiles blended with the global curve, the reading
of Sec. III-B.2 stated in include/decolor.h) against the FP64 oracle.

Tolerance. T is within 1e-5 of the oracle: the histogram masses are integers of
2^-19 per pixel (each rounded by at most 2^-20, so a tile curve moves by at most
2^-20 ~ 1e-6), the curve tables are rounded once to FP32 (~6e-8), the bin
position u = 2 log2(Lhat + eps) - ... carries the FP32 error of log2 (a few 1e-7
bins), and a tile curve's slope in u is at most 1 per bin, so each of these
moves T by about 1e-6 or less; the global part is bounded as in the global tone
map's tests.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f16, check_f32, check_u8, need_gpu, report, to_dev

pytestmark = pytest.mark.gpu
TM = dict(eps=1e-4, contrast=2.0, sigma_floor=1e-3)


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _image(kind, h, w, seed):
    if kind == "u8":
        return synth.gradient_rects() if (h, w) == (512, 512) else synth.sdr_pixels(
            np.random.default_rng(seed), h, w)
    if kind == "f16":
        return synth.hdr_pixels(np.random.default_rng(seed), h, w)
    return synth.random_image(seed, h, w, np.float32, scale=4.0)


@pytest.mark.parametrize("strength", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("kind,shape", [("u8", (512, 512)), ("u8", (1, 1)), ("u8", (5, 3)),
                                        ("u8", (64, 64)), ("u8", (65, 130)), ("f16", (256, 256)),
                                        ("f16", (130, 1001)), ("f32", (70, 33)),
                                        ("u8", (300, 517))])
def test_local_vs_oracle(dev, kind, shape, strength):
    h, w = shape
    img = _image(kind, h, w, h * w)
    t_ref, st_ref = oracle.tonemap_local(img, strength=strength, **TM)
    outs, _, stats = P.tonemap_local([to_dev(img, dev)], torch.float32, strength=strength, **TM)
    check_f32(outs[0].cpu().numpy(), t_ref, "local %s %dx%d strength %g" % (kind, h, w, strength))
    st = P.stats_to_host(stats)[0]
    assert st["count"] == h * w
    if h * w > 1:
        assert abs(st["mu"] - st_ref["mu"]) <= 2e-5 * (1 + abs(st_ref["mu"]))


@pytest.mark.parametrize("kind", ["u8", "f16"])
def test_local_encodings_and_lhat(dev, kind):
    img = _image(kind, 200, 333, 51)
    t_ref, _ = oracle.tonemap_local(img, strength=0.7, **TM)
    x = to_dev(img, dev)
    o8, l8, _ = P.tonemap_local([x], torch.uint8, torch.float32, strength=0.7, **TM)
    o16 = P.tonemap_local([x], torch.float16, strength=0.7, **TM)[0][0]
    check_u8(o8[0].cpu().numpy(), t_ref, "local %s u8" % kind,
             max_fraction=1e-3)
    check_f16(o16.cpu().numpy(), oracle.encode_f16(t_ref), "local %s f16" % kind)
    check_f32(l8[0].cpu().numpy(), oracle.decolorize(img), "local %s lhat" % kind,
              rel=kind != "u8")


@pytest.mark.parametrize("kind", ["u8", "f16"])
def test_local_pitched_views(dev, kind):
    """Row pitches that allow the unit walk (16-byte multiples, first column
    16-byte aligned) and ones that force the per-pixel walk."""
    img = _image(kind, 150, 200, 52)
    t_ref, _ = oracle.tonemap_local(img, strength=0.5, **TM)
    x = to_dev(img, dev)
    big = torch.zeros((150, 240, 3), dtype=x.dtype, device=dev)
    for c0, pad in ((16, 4), (16, 3), (5, 4)):
        big.zero_()
        big[:, c0:c0 + 200] = x
        o = torch.full((150, 200 + pad), -1.0, device=dev)
        P.tonemap_local([big[:, c0:c0 + 200]], outs=[o[:, :200]], want_stats=False, strength=0.5,
                        **TM)
        check_f32(o[:, :200].cpu().numpy(), t_ref, "local %s view c0=%d pad=%d" % (kind, c0, pad))
        assert bool((o[:, 200:] == -1.0).all())


def test_local_batch_matches_single_calls(dev):
    imgs = [_image("u8", 100, 150, 53), _image("f16", 64, 700, 54), _image("f32", 9, 100, 55),
            _image("u8", 1, 1, 56), _image("f16", 200, 65, 57)]
    xs = [to_dev(a, dev) for a in imgs]
    outs, _, stats = P.tonemap_local(xs, torch.float32, strength=0.8, **TM)
    st = P.stats_to_host(stats)
    for i, x in enumerate(xs):
        one, _, s1 = P.tonemap_local([x], torch.float32, strength=0.8, **TM)
        assert torch.equal(outs[i], one[0]), i
        assert st[i] == P.stats_to_host(s1)[0], i


def test_local_plan_graph_replays(dev):
    imgs = [_image("f16", 256, 300, 58), _image("u8", 128, 640, 59)]
    xs = [to_dev(a, dev) for a in imgs]
    want = [P.tonemap_local([x], torch.float32, strength=0.6, **TM)[0][0] for x in xs]
    outs = [torch.zeros_like(w) for w in want]
    s = torch.cuda.Stream()
    plan = P.Plan(P.PLAN_LOCAL, xs, outs, graph=True, local_strength=0.6, **TM)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            plan.run(s)
        s.synchronize()
        for o, w in zip(outs, want):
            assert torch.equal(o, w), rep
    plan.close()


@pytest.mark.parametrize("s", [1.0, 0.6, 0.0])
@pytest.mark.parametrize("kind,shape", [("u8", (64, 64)), ("f16", (130, 1001)), ("u8", (300, 517)),
                                        ("f32", (70, 33))])
def test_local_colour_vs_oracle(dev, kind, shape, s):
    h, w = shape
    img = _image(kind, h, w, h + w)
    rgb_ref, _ = oracle.tonemap_local_colour(img, strength=0.6, saturation=s, **TM)
    x = to_dev(img, dev)
    got = P.tonemap_local([x], torch.float32, colour=True, strength=0.6, saturation=s, **TM)[0][0]
    assert got.shape == (h, w, 3)
    check_f32(got.cpu().numpy(), rgb_ref, "local colour %s %dx%d s=%g" % (kind, h, w, s))
    g8 = P.tonemap_local([x], torch.uint8, colour=True, strength=0.6, saturation=s, **TM)[0][0]
    check_u8(g8.cpu().numpy(), rgb_ref, "local colour u8", max_fraction=2e-3)


def test_local_gray_and_colour_in_one_call(dev):
    imgs = [_image("u8", 100, 150, 61), _image("f16", 64, 700, 62), _image("u8", 33, 65, 63)]
    xs = [to_dev(a, dev) for a in imgs]
    outs = [torch.empty((100, 150, 3), dtype=torch.uint8, device=dev),
            torch.empty((64, 700), device=dev),
            torch.empty((33, 65, 3), dtype=torch.float16, device=dev)]
    P.tonemap_local(xs, outs=outs, strength=0.8, saturation=0.7, **TM)
    for x, o in zip(xs, outs):
        one = P.tonemap_local([x], o.dtype, colour=o.dim() == 3, strength=0.8, saturation=0.7,
                              **TM)[0][0]
        assert torch.equal(one, o)
