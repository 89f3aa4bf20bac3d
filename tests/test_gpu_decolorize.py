"""GPU parity of the decolorization (Sec. II-B, Eqs. (1)-(6)) against the FP64
oracle, through the C ABI (``paper_2108_13656_amd`` marshals torch tensors
into ``dc_decolorize`` / ``dc_decolorize_batch``)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f16, check_f32, check_u8, need_gpu, report, to_dev

pytestmark = pytest.mark.gpu

TORCH_OF = {np.uint8: torch.uint8, np.float16: torch.float16, np.float32: torch.float32}


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def lut():
    return oracle.all_colours(0.55, 0.8)


def test_all_colours_exhaustive(dev, lut):
    """Every 24-bit colour once (4096 x 4096): FP32 and 8-bit outputs in one pass."""
    img = synth.all_colours_image()
    x = to_dev(img, dev)
    f32, u8 = P.decolorize(x, torch.float32, torch.uint8)
    torch.cuda.synchronize()
    want = lut / 255.0
    check_f32(f32.cpu().numpy().ravel(), want, "all colours single f32")
    check_u8(u8.cpu().numpy().ravel(), want, "all colours single u8")
    # same through the batched launch, bit-identical to the single launch
    bf, bu = P.decolorize_batch([x], torch.float32, torch.uint8)[0]
    torch.cuda.synchronize()
    assert torch.equal(bf, f32) and torch.equal(bu, u8)


def test_gradient_rects_512(dev):
    """The 512 x 512 seeded test image, 8-bit in, FP32 out."""
    img = synth.gradient_rects()
    got = P.decolorize(to_dev(img, dev)).cpu().numpy()
    check_f32(got, oracle.decolorize(img), "gradient+rects 512x512")


def test_f16_channel_sweep(dev):
    """Every non-negative binary16 value in each channel (0 .. 65504 and +Inf,
    which reads as 65504), plus NaN, -Inf, -0 and a negative subnormal (which
    read as 0), crossed with a grid of values of the other two channels; true
    relative error 1e-5 everywhere (the flush floor 1e-30 lies below every
    nonzero binary16 result)."""
    extra = np.array([0x7E00, 0xFC00, 0x8000, 0x8001], np.uint16)
    halves = np.concatenate([np.arange(0, 0x7C01, dtype=np.uint16), extra]).view(np.float16)
    grid = np.array([0.0, 6e-8, 1e-3, 0.5, 1.0, 7.25, 100.0, 65504.0], np.float16)
    for ch in range(3):
        others = [c for c in range(3) if c != ch]
        rows = []
        for a in grid:
            for b in grid[::3]:
                px = np.zeros((halves.size, 3), np.float16)
                px[:, ch] = halves
                px[:, others[0]] = a
                px[:, others[1]] = b
                rows.append(px)
        img = np.concatenate(rows).reshape(-1, 1, 3)  # H x 1 x 3
        got = P.decolorize(to_dev(img, dev)).cpu().numpy().ravel()
        want = oracle.decolorize(img).ravel()
        check_f32(got, want, "f16 sweep channel %d" % ch, rel=True)


def test_f32_special_values(dev):
    """Zero, negatives, NaN, +-Inf, subnormals and values up to and past the
    1e18 ceiling in every combination of channels: relative 1e-5, with values
    below 1e-30 allowed to flush (absolute error < 1e-30); +Inf and 3e18 read as
    1e18."""
    vals = np.array([0.0, -1.0, np.nan, -np.inf, np.inf, 1e-40, 1e-20, 1e-6, 0.3, 1.0, 255.0,
                     1e6, 1e18, 3e18], np.float32)
    r, g, b = np.meshgrid(vals, vals, vals, indexing="ij")
    img = np.stack([r.ravel(), g.ravel(), b.ravel()], -1).reshape(-1, vals.size, 3)
    img = img.astype(np.float32)
    got = P.decolorize(to_dev(img, dev)).cpu().numpy()
    want = oracle.decolorize(img)
    assert np.all(np.isfinite(got))
    check_f32(got, want, "f32 special values", rel=True)


def test_hdr_distribution(dev):
    img = synth.hdr_pixels(np.random.default_rng(12), 301, 257)
    got = P.decolorize(to_dev(img, dev)).cpu().numpy()
    check_f32(got, oracle.decolorize(img), "hdr 301x257 f16", rel=True)


@pytest.mark.parametrize("beta_r,beta_k", [(0.7, 0.6), (0.51, 0.99), (1.0, 0.0), (0.0, 1.0)])
def test_other_betas(dev, beta_r, beta_k):
    img8 = synth.random_image(21, 67, 45, np.uint8)
    got = P.decolorize(to_dev(img8, dev), beta_r=beta_r, beta_k=beta_k).cpu().numpy()
    check_f32(got, oracle.decolorize(img8, beta_r, beta_k), "u8 betas %s %s" % (beta_r, beta_k))
    imgh = synth.hdr_pixels(np.random.default_rng(22), 45, 67)
    got = P.decolorize(to_dev(imgh, dev), beta_r=beta_r, beta_k=beta_k).cpu().numpy()
    check_f32(got, oracle.decolorize(imgh, beta_r, beta_k), "f16 betas", rel=True)


@pytest.mark.parametrize("src", [np.uint8, np.float16, np.float32])
@pytest.mark.parametrize("dst", [torch.uint8, torch.float16, torch.float32])
def test_output_encodings(dev, src, dst):
    if src == np.uint8:
        img = synth.random_image(31, 33, 70, np.uint8)
    else:
        img = synth.random_image(32, 33, 70, src, scale=2.0)  # HDR values above 1 too
    out = P.decolorize(to_dev(img, dev), dst).cpu().numpy()
    lhat = oracle.decolorize(img)
    name = "%s->%s" % (np.dtype(src).name, dst)
    if dst == torch.uint8:
        check_u8(out, lhat, name, max_fraction=1e-3)
    elif dst == torch.float16:
        check_f16(out, oracle.encode_f16(lhat), name)
    else:
        check_f32(out, lhat, name, rel=src != np.uint8)


SHAPES = [(1, 1), (1, 17), (17, 1), (3, 5), (37, 53), (2, 16 * 256 * 2 + 5), (129, 4099)]


def _check_any(out, img, dtype, what):
    lhat = oracle.decolorize(img)
    check_f32(out, lhat, what, rel=dtype != np.uint8)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("src", [np.uint8, np.float16, np.float32])
@pytest.mark.parametrize("walk", ["packed", "rows", "odd"])
def test_shapes_and_walks(dev, shape, src, walk):
    """Ragged sizes through each of the three walks: packed (one segment),
    pitched rows starting 16-byte aligned, and pitched rows starting at an odd
    element (both on the row walk; widths below 4 on the per-pixel walk)."""
    h, w = shape
    seed = hash((h, w, np.dtype(src).name, walk)) & 0xFFFF
    if walk == "packed":
        big = synth.random_image(seed, h, w, src, scale=3.0)
        x = to_dev(big, dev)
        out = torch.empty((h, w), dtype=torch.float32, device=dev)
    else:
        pad = 16 if walk == "rows" else 1
        wbig = ((w + 2 * pad + 15) // 16) * 16
        big = synth.random_image(seed, h, wbig, src, scale=3.0)
        x = to_dev(big, dev)[:, pad:pad + w]
        outbig = torch.empty((h, wbig), dtype=torch.float32, device=dev)
        out = outbig[:, pad:pad + w]
        big = big[:, pad:pad + w]
    P.decolorize(x, out=out)
    _check_any(out.cpu().numpy(), big, src, "%s %dx%d %s" % (walk, h, w, np.dtype(src).name))


def test_batch_mixed_equals_single(dev):
    rng = np.random.default_rng(40)
    imgs = []
    for i in range(24):
        h, w = (int(v) for v in rng.integers(1, 300, 2))
        dt = [np.uint8, np.float16, np.float32][i % 3]
        imgs.append(synth.random_image(100 + i, h, w, dt, scale=4.0))
    xs = [to_dev(a, dev) for a in imgs]
    batch = P.decolorize_batch(xs, torch.float32, torch.uint8)
    single = [P.decolorize(x, torch.float32, torch.uint8) for x in xs]
    torch.cuda.synchronize()
    for i, ((bf, bu), (sf, su)) in enumerate(zip(batch, single)):
        assert torch.equal(bf, sf) and torch.equal(bu, su), i
        _check_any(bf.cpu().numpy(), imgs[i], imgs[i].dtype.type, "batch image %d" % i)
    # one input type only (the non-mixed kernel)
    xs8 = [x for x, a in zip(xs, imgs) if a.dtype == np.uint8]
    b8 = P.decolorize_batch(xs8, torch.float32)
    for x, b in zip(xs8, b8):
        assert torch.equal(b, P.decolorize(x))


def test_non_default_stream(dev):
    img = synth.random_image(50, 200, 300, np.uint8)
    x = to_dev(img, dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = P.decolorize(x, stream=s)
    s.synchronize()
    check_f32(out.cpu().numpy(), oracle.decolorize(img), "side stream")


def test_alias_rejected_on_device(dev):
    x = torch.zeros((8, 8, 3), dtype=torch.float32, device=dev)
    with pytest.raises(P.DecolorError) as e:
        P.decolorize(x, out=x.view(-1)[:64].view(8, 8))
    assert e.value.status == P.DC_ERR_ALIAS


def test_repeatable(dev):
    img = synth.random_image(60, 333, 444, np.float16, scale=10.0)
    x = to_dev(img, dev)
    a = P.decolorize(x)
    for _ in range(5):
        assert torch.equal(P.decolorize(x), a)


def test_plans_match_direct_calls(dev):
    """Frozen plans (direct launches and HIP-graph replays) give the results of
    the direct batched call, bit for bit, on every replay."""
    rng = np.random.default_rng(70)
    imgs = [synth.sdr_pixels(rng, 123, 457), synth.hdr_pixels(rng, 64, 64),
            synth.sdr_pixels(rng, 1, 999)]
    xs = [to_dev(a, dev) for a in imgs]
    want = P.decolorize_batch(xs, torch.float32, torch.uint8)
    for graph in (False, True):
        o32 = [torch.full(x.shape[:2], -1.0, device=dev) for x in xs]
        o8 = [torch.zeros(x.shape[:2], dtype=torch.uint8, device=dev) for x in xs]
        plan = P.Plan(P.PLAN_DECOLORIZE, xs, o32, o8, graph=graph)
        s = torch.cuda.Stream()
        for rep in range(4):
            for o in o32:
                o.fill_(-1.0)  # eager work between replays
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                plan.run(s)
            s.synchronize()
            for (wf, wu), a, b in zip(want, o32, o8):
                assert torch.equal(a, wf) and torch.equal(b, wu), (graph, rep)
        plan.close()


def test_tuning_roundtrip_and_autotune(dev):
    t0 = P.get_tuning()
    try:
        t = dict(t0, groups=[4, 1, 2], decolor_grid_per_cu=8)
        P.set_tuning(t)
        assert P.get_tuning() == t
        with pytest.raises(P.DecolorError):
            P.set_tuning(dict(t0, groups=[3, 1, 2]))
        img = synth.sdr_pixels(np.random.default_rng(71), 1080, 1920)
        x = to_dev(img, dev)
        ref = P.decolorize(x)
        out = torch.empty_like(ref)
        chosen = P.autotune(P.PLAN_DECOLORIZE, [x], [out])
        report("autotune chose %s" % chosen)
        assert chosen["groups"][0] in (1, 2, 4)
        assert torch.equal(P.decolorize(x), ref)  # launch shape never changes results
        assert torch.equal(out, ref)
    finally:
        P.set_tuning(t0)


def test_tuning_env_cache(dev, tmp_path, monkeypatch):
    """DC_AUTOTUNE_CACHE: autotune writes the context's shapes to the named
    file, and apply_tuning_cache (which a new context runs) applies it."""
    import json
    t0 = P.get_tuning()
    try:
        path = str(tmp_path / "cache.json")
        monkeypatch.setenv(P.TUNING_CACHE_ENV, path)
        x = to_dev(synth.sdr_pixels(np.random.default_rng(3), 256, 256), dev)
        o = torch.empty((256, 256), device=dev)
        P.autotune(P.PLAN_DECOLORIZE, [x], [o])
        saved = json.load(open(path))["tuning"]
        assert saved == P.get_tuning()
        P.set_tuning(dict(t0, groups=[4, 4, 4], pass2_grid_per_cu=2))
        assert P.apply_tuning_cache() and P.get_tuning() == saved
        monkeypatch.delenv(P.TUNING_CACHE_ENV)
        assert not P.apply_tuning_cache()
    finally:
        P.set_tuning(t0)


def test_tuning_file(dev, tmp_path):
    """save_tuning / load_tuning: a file written on this device and build is
    applied; one naming another device is not, and leaves the tuning alone."""
    import json
    t0 = P.get_tuning()
    try:
        path = str(tmp_path / "tuning.json")
        P.set_tuning(dict(t0, groups=[2, 1, 4], pass1_grid_per_cu=8))
        P.save_tuning(path)
        want = P.get_tuning()
        P.set_tuning(t0)
        assert P.load_tuning(path) and P.get_tuning() == want
        rec = json.load(open(path))
        rec["device"] = "another device"
        json.dump(rec, open(path, "w"))
        P.set_tuning(t0)
        assert not P.load_tuning(path) and P.get_tuning() == t0
        assert not P.load_tuning(str(tmp_path / "missing.json"))
    finally:
        P.set_tuning(t0)
