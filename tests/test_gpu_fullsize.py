"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times: autotuned launch shapes and a HIP-graph plan over resident buffers.

- 64-frame video batch (32 x 1920x1080 + 32 x 3840x2160, 8-bit): every pixel of
  both outputs (8-bit and FP32) against the oracle's value of its colour (the
  oracle's table of all 2^24 colours, computed by the FP64 oracle).
- 16 x 4096^2 binary16 tone map: every image's statistics against the FP64
  oracle over all its pixels, and T at 65536 sampled pixels per image against
  the oracle's curve evaluated with the oracle's own statistics; the same for
  the re-coloured 8-bit RGB output (s = 1 and s = 0.6) at 16384 sampled pixels
  per image.
- the same images through the local tone map: T at 8192 sampled pixels per
  image against the oracle (which still builds every tile's histogram).
- uneven batch of 256 images (half 8-bit, half binary16, 64..4096 per side),
  one persistent launch: every pixel against the oracle.
- the weight sweep of a 3840x2160 frame of the video batch under 20 (beta_R,
  beta_k) pairs, as bench.py times it: every output bit-identical to a single
  call, and every pixel of 4 of the outputs against the oracle's table of all
  colours at that pair.
- 8-bit frames of the video batch (8 x 1080p + 8 x 2160p) through the global
  tone map, 8-bit T and FP32 Lhat out (the serving mix's SDR request): every
  image's statistics, and every pixel of both outputs, against the oracle.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f32, check_u8, need_gpu, report, to_dev, u8_mismatches_at_ties

pytestmark = pytest.mark.gpu
WORKERS = min(16, os.cpu_count() or 1)
TM = dict(eps=1e-4, contrast=2.0, sigma_floor=1e-3)


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def lut():
    return oracle.all_colours(0.55, 0.8)


def _run_plan(kind, xs, outs, outs2=None, **kw):
    t0 = P.get_tuning()
    try:
        chosen = P.autotune(kind, xs, outs, outs2,
                             **{k: v for k, v in kw.items() if k in TM or k == "saturation"})
        report("autotuned: %s" % chosen)
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        plan = P.Plan(kind, xs, outs, outs2, graph=True, **kw)
        with torch.cuda.stream(s):
            plan.run(s)
        s.synchronize()
        plan.close()
    finally:
        P.set_tuning(t0)


def _codes(img):
    c = img.astype(np.int64)
    return (c[..., 0] << 16) | (c[..., 1] << 8) | c[..., 2]


@pytest.mark.timeout(600)
def test_video_batch_every_pixel(dev, lut):
    frames = synth.video_frames(workers=WORKERS)
    xs = [to_dev(f, dev) for f in frames]
    o8 = [torch.empty(f.shape[:2], dtype=torch.uint8, device=dev) for f in frames]
    o32 = [torch.empty(f.shape[:2], dtype=torch.float32, device=dev) for f in frames]
    _run_plan(P.PLAN_DECOLORIZE, xs, o8, o32)
    worst, off, total = 0.0, 0, 0
    for f, a, b in zip(frames, o8, o32):
        want = lut[_codes(f)]
        err = np.abs(b.cpu().numpy().astype(np.float64) - want / 255.0)
        worst = max(worst, float(err.max()))
        codes = a.cpu().numpy()
        d = np.abs(codes.astype(np.int32) - oracle.encode_u8(want / 255.0).astype(np.int32))
        assert d.max() <= 1
        u8_mismatches_at_ties(codes, want / 255.0)
        off += int(np.count_nonzero(d))
        total += d.size
    report("video batch: %d px, max |dL| %.3e, u8 codes off by one: %d (fraction %.3e)" %
           (total, worst, off, off / total))
    assert worst <= 1e-5
    assert off / total <= 1e-4


@pytest.mark.timeout(600)
def test_weight_sweep_4k_every_pixel(dev):
    frame = synth.video_frame(63)
    x = to_dev(frame, dev)
    betas = [(br, bk) for br in (0.0, 0.3, 0.55, 0.8, 1.0) for bk in (0.2, 0.5, 0.8, 1.0)]
    sweep = P.beta_sweep(x, betas)
    for i, (br, bk) in enumerate(betas):
        assert torch.equal(sweep[i], P.decolorize(x, beta_r=br, beta_k=bk)), (br, bk)
    codes = _codes(frame)
    worst = 0.0
    for i in (0, 6, 13, 19):
        br, bk = betas[i]
        want = oracle.all_colours(br, bk)[codes] / 255.0
        err = np.abs(sweep[i].cpu().numpy().astype(np.float64) - want)
        worst = max(worst, float(err.max()))
    report("weight sweep 3840x2160 x 20 pairs: max |dL| %.3e over 4 checked pairs" % worst)
    assert worst <= 1e-5


@pytest.mark.timeout(600)
def test_hdr_tonemap_full(dev):
    imgs = synth.hdr_images(workers=WORKERS)
    xs = [to_dev(a, dev) for a in imgs]
    outs = [torch.empty(a.shape[:2], dtype=torch.float32, device=dev) for a in imgs]
    stats = torch.zeros((len(imgs), P.STATS_BYTES), dtype=torch.uint8, device=dev)
    _run_plan(P.PLAN_TONEMAP, xs, outs, stats=stats, **TM)
    st = P.stats_to_host(stats)
    rng = np.random.default_rng(99)
    worst_t, worst_mu, worst_sig = 0.0, 0.0, 0.0
    for i, img in enumerate(imgs):
        lhat = oracle.decolorize(img, nthreads=WORKERS)
        ref = oracle.tonemap_stats(lhat, TM["eps"])
        worst_mu = max(worst_mu, abs(st[i]["mu"] - ref["mu"]))
        worst_sig = max(worst_sig, abs(st[i]["sigma"] - ref["sigma"]) / ref["sigma"])
        assert st[i]["count"] == ref["count"]
        assert st[i]["l_min"] == pytest.approx(ref["l_min"], rel=1e-5)
        assert st[i]["l_max"] == pytest.approx(ref["l_max"], rel=1e-5)
        idx = rng.integers(0, lhat.size, 65536)
        t_ref = oracle.tonemap_curve(lhat.ravel()[idx], ref["mu"], ref["sigma"], **TM)
        t_gpu = outs[i].view(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
        worst_t = max(worst_t, float(np.max(np.abs(t_gpu - t_ref))))
    report("hdr tone map 16x4096^2: max |d mu| %.2e, max |d sigma|/sigma %.2e, max |dT| %.2e "
           "(65536 sampled px per image)" % (worst_mu, worst_sig, worst_t))
    assert worst_mu <= 2e-5 and worst_sig <= 2e-5 and worst_t <= 1e-5


@pytest.mark.timeout(600)
def test_sdr_tonemap_every_pixel(dev, lut):
    frames = [synth.video_frame(i) for i in list(range(8)) + list(range(32, 40))]
    xs = [to_dev(f, dev) for f in frames]
    outs = [torch.empty(f.shape[:2], dtype=torch.uint8, device=dev) for f in frames]
    lh = [torch.empty(f.shape[:2], dtype=torch.float32, device=dev) for f in frames]
    stats = torch.zeros((len(frames), P.STATS_BYTES), dtype=torch.uint8, device=dev)
    _run_plan(P.PLAN_TONEMAP, xs, outs, lh, stats=stats, **TM)
    st = P.stats_to_host(stats)
    worst_l, worst_mu, off, total = 0.0, 0.0, 0, 0
    for i, f in enumerate(frames):
        lhat = lut[_codes(f)] / 255.0
        ref = oracle.tonemap_stats(lhat, TM["eps"])
        worst_mu = max(worst_mu, abs(st[i]["mu"] - ref["mu"]),
                       abs(st[i]["sigma"] - ref["sigma"]) / ref["sigma"])
        assert st[i]["count"] == ref["count"]
        worst_l = max(worst_l, float(np.max(np.abs(lh[i].cpu().numpy() - lhat))))
        t_ref = oracle.tonemap_curve(lhat, ref["mu"], ref["sigma"], **TM)
        codes = outs[i].cpu().numpy()
        d = np.abs(codes.astype(np.int32) - oracle.encode_u8(t_ref).astype(np.int32))
        assert d.max() <= 1, i
        u8_mismatches_at_ties(codes, t_ref)
        off += int(np.count_nonzero(d))
        total += d.size
    report("sdr tone map 8x1080p + 8x2160p: max |d mu|, |d sigma|/sigma %.2e, max |dLhat| %.2e, "
           "u8 T codes off by one: %d of %d (fraction %.3e)" %
           (worst_mu, worst_l, off, total, off / total))
    assert worst_mu <= 2e-5 and worst_l <= 1e-5
    assert off / total <= 1e-3


@pytest.mark.timeout(900)
@pytest.mark.parametrize("s", [1.0, 0.6])
def test_hdr_colour_tonemap_full(dev, s):
    imgs = synth.hdr_images(workers=WORKERS)
    xs = [to_dev(a, dev) for a in imgs]
    outs = [torch.empty(a.shape, dtype=torch.uint8, device=dev) for a in imgs]
    _run_plan(P.PLAN_TONEMAP, xs, outs, saturation=s, **TM)
    rng = np.random.default_rng(98)
    off, total = 0, 0
    for i, img in enumerate(imgs):
        lhat = oracle.decolorize(img, nthreads=WORKERS).ravel()
        ref = oracle.tonemap_stats(lhat, TM["eps"])
        idx = rng.integers(0, lhat.size, 16384)
        t_ref = oracle.tonemap_curve(lhat[idx], ref["mu"], ref["sigma"], **TM)
        rgb = oracle.decode_f16(img.reshape(-1, 3)[idx])
        want = np.array([[oracle.colour_channel(c, lh, t, s) for c in px]
                         for px, lh, t in zip(rgb, lhat[idx], t_ref)])
        got = outs[i].view(-1, 3)[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.int32)
        d = np.abs(got - oracle.encode_u8(want).astype(np.int32))
        assert d.max() <= 1, i
        u8_mismatches_at_ties(got, want)
        off += int(np.count_nonzero(d))
        total += d.size
    report("hdr colour tone map 16x4096^2 -> u8 RGB, s=%g: %d sampled codes, %d off by one "
           "(fraction %.3e)" % (s, total, off, off / total))
    assert off / total <= 2e-3


@pytest.mark.timeout(900)
def test_hdr_local_tonemap_full(dev):
    imgs = synth.hdr_images(workers=WORKERS)
    xs = [to_dev(a, dev) for a in imgs]
    outs = [torch.empty(a.shape[:2], dtype=torch.float32, device=dev) for a in imgs]
    s = torch.cuda.Stream()
    plan = P.Plan(P.PLAN_LOCAL, xs, outs, graph=True, local_strength=0.5, **TM)
    with torch.cuda.stream(s):
        plan.run(s)
    s.synchronize()
    plan.close()
    rng = np.random.default_rng(97)
    worst = 0.0
    for i, img in enumerate(imgs):
        idx = rng.integers(0, img.shape[0] * img.shape[1], 8192)
        want, _ = oracle.tonemap_local(img, strength=0.5, nthreads=WORKERS, sample=idx, **TM)
        got = outs[i].view(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
        worst = max(worst, float(np.max(np.abs(got - want))))
    report("hdr local tone map 16x4096^2: max |dT| %.2e (8192 sampled px per image)" % worst)
    assert worst <= 1e-5


@pytest.mark.timeout(900)
def test_uneven_batch_every_pixel(dev, lut):
    imgs = synth.uneven_batch(workers=WORKERS)
    xs = [to_dev(a, dev) for a in imgs]
    outs = [torch.empty(a.shape[:2], dtype=torch.float32, device=dev) for a in imgs]
    _run_plan(P.PLAN_DECOLORIZE, xs, outs)
    worst8, worst16 = 0.0, 0.0
    for img, o in zip(imgs, outs):
        got = o.cpu().numpy().astype(np.float64)
        if img.dtype == np.uint8:
            worst8 = max(worst8, float(np.max(np.abs(got - lut[_codes(img)] / 255.0))))
        else:
            want = oracle.decolorize(img, nthreads=WORKERS)
            worst16 = max(worst16, check_f32(got, want, "uneven f16 %dx%d" % img.shape[:2],
                                             rel=True))
    report("uneven batch: %d px, max |dL| u8 %.3e, f16 relative %.3e" %
           (sum(a.shape[0] * a.shape[1] for a in imgs), worst8, worst16))
    assert worst8 <= 1e-5 and worst16 <= 1e-5


@pytest.mark.timeout(900)
def test_image_larger_than_2gib(dev):
    """One binary32 image of 14000 x 14000 (2.35 GB of input, byte offsets past
    2^31): decolorization at sampled pixels and at the last row against the
    oracle's per-pixel value, and the global tone map's statistics against the
    oracle over every pixel."""
    h = w = 14000
    rng = np.random.default_rng(96)
    img = rng.random((h, w, 3), dtype=np.float32) * 4.0
    x = to_dev(img, dev)
    out = P.decolorize(x)
    idx = np.concatenate([rng.integers(0, h * w, 4096), np.arange(h * w - w, h * w)])
    got = out.view(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    flat = img.reshape(-1, 3)[idx].astype(np.float64)
    want = np.array([oracle.luminance(*p) for p in flat])
    check_f32(got, want, "14000^2 binary32 decolorize", rel=True)
    del out
    _, _, stats = P.tonemap_global([x], torch.float16, **TM)
    st = P.stats_to_host(stats)[0]
    ref = oracle.tonemap_stats(oracle.decolorize(img, nthreads=WORKERS), TM["eps"])
    report("14000^2 tone map: mu %.7f / %.7f, sigma %.7f / %.7f" %
           (st["mu"], ref["mu"], st["sigma"], ref["sigma"]))
    assert st["count"] == h * w
    assert abs(st["mu"] - ref["mu"]) <= 2e-5 * (1 + abs(ref["mu"]))
    assert abs(st["sigma"] - ref["sigma"]) <= 2e-5 * ref["sigma"]


@pytest.mark.timeout(900)
def test_more_than_2_31_pixels(dev, lut):
    """One 8-bit image of 46400 x 46400 = 2.15e9 pixels (pixel indices past
    2^31, 6.5 GB of input made on the device): decolorization to 8-bit codes at
    a million sampled pixels and along the last row against the oracle's table
    of all colours; the global tone map's statistics over every pixel against
    the oracle's, computed in FP64 from the image's colour histogram (counted
    on the device) and the oracle's value of each colour, and T at the sampled
    pixels against the oracle curve with the oracle's statistics."""
    h = w = 46400
    assert h * w > 2 ** 31
    gen = torch.Generator(device=dev)
    gen.manual_seed(97)
    x = torch.randint(0, 256, (h, w, 3), dtype=torch.uint8, device=dev, generator=gen)
    out = P.decolorize(x, torch.uint8)
    rng = np.random.default_rng(97)
    idx = np.concatenate([rng.integers(0, h * w, 1 << 20), np.arange(h * w - w, h * w)])
    tidx = torch.from_numpy(idx).to(dev)
    px = x.view(-1, 3)[tidx].cpu().numpy()
    codes = (px[:, 0].astype(np.int64) << 16) | (px[:, 1].astype(np.int64) << 8) | px[:, 2]
    lhat = lut[codes] / 255.0
    got = out.view(-1)[tidx].cpu().numpy()
    d = np.abs(got.astype(np.int32) - oracle.encode_u8(lhat).astype(np.int32))
    assert d.max() <= 1
    u8_mismatches_at_ties(got, lhat)
    del out
    # colour histogram on the device, in slabs of rows (int32 codes)
    counts = torch.zeros(1 << 24, dtype=torch.int64, device=dev)
    for r0 in range(0, h, 4096):
        c = x[r0:r0 + 4096].reshape(-1, 3).to(torch.int32)
        code = (c[:, 0] << 16) | (c[:, 1] << 8) | c[:, 2]
        counts += torch.bincount(code, minlength=1 << 24)
        del c, code
    counts = counts.cpu().numpy()
    assert int(counts.sum()) == h * w
    ref = oracle.tonemap_stats_counted(lut / 255.0, counts, TM["eps"])
    t, _, stats = P.tonemap_global([x], torch.float32, **TM)
    st = P.stats_to_host(stats)[0]
    assert st["count"] == h * w
    report("46400^2 tone map: mu %.7f / %.7f, sigma %.7f / %.7f, min %.4g / %.4g, max %.4g / %.4g"
           % (st["mu"], ref["mu"], st["sigma"], ref["sigma"], st["l_min"], ref["l_min"],
              st["l_max"], ref["l_max"]))
    assert abs(st["mu"] - ref["mu"]) <= 2e-5 * (1 + abs(ref["mu"]))
    assert abs(st["sigma"] - ref["sigma"]) <= 2e-5 * ref["sigma"]
    assert st["l_min"] == pytest.approx(ref["l_min"], rel=1e-5, abs=1e-6)
    assert st["l_max"] == pytest.approx(ref["l_max"], rel=1e-5)
    t_ref = oracle.tonemap_curve(lhat, ref["mu"], ref["sigma"], **TM)
    err = float(np.max(np.abs(t[0].view(-1)[tidx].cpu().numpy() - t_ref)))
    report("46400^2 u8: %d px, codes off by one %d, max |dT| %.2e at %d sampled px" %
           (h * w, int(np.count_nonzero(d)), err, idx.size))
    assert err <= 1e-5
