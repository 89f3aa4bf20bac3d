"""GPU parity of the global tone map (Sec. III-B.1, centred sigmoid on
ln(Lhat + eps), slope normalised by the image's standard deviation) against the
FP64 oracle, through ``dc_tonemap_global``.

Tolerances. The statistics are FP32 Chan merges of FP32 log2 values: |d mu| and
|d sigma| / sigma stay below 2e-5. T = 1 / (1 + exp(-c z)) moves by at most
c / 4 * |dz| with z = (x - mu) / s, so for images with sigma >= 0.1 the 1e-5
bound on T holds with room to spare; flat images are checked by their closed
form (T = 1/2) instead.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f32, check_u8, need_gpu, report, to_dev

pytestmark = pytest.mark.gpu
TM = dict(eps=1e-4, contrast=2.0, sigma_floor=1e-3)


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _check_stats(st, ref, what):
    report("%s: mu %.7f/%.7f sigma %.7f/%.7f" % (what, st["mu"], ref["mu"], st["sigma"],
                                                  ref["sigma"]))
    assert abs(st["mu"] - ref["mu"]) <= 2e-5 * (1 + abs(ref["mu"])), what
    assert abs(st["sigma"] - ref["sigma"]) <= 2e-5 * max(ref["sigma"], 1e-3), what
    assert st["l_min"] == pytest.approx(ref["l_min"], rel=1e-5, abs=1e-6)
    assert st["l_max"] == pytest.approx(ref["l_max"], rel=1e-5, abs=1e-6)
    assert st["count"] == ref["count"]


@pytest.mark.parametrize("kind,shape", [("u8", (64, 64)), ("u8", (1, 1)), ("u8", (37, 91)),
                                        ("f16", (256, 256)), ("f16", (5, 4099)),
                                        ("f32", (70, 33)), ("u8", (512, 512))])
def test_tonemap_vs_oracle(dev, kind, shape):
    h, w = shape
    if kind == "u8":
        img = synth.gradient_rects() if shape == (512, 512) else synth.random_image(7, h, w, np.uint8)
    elif kind == "f16":
        img = synth.hdr_pixels(np.random.default_rng(h * w), h, w)
    else:
        img = synth.random_image(8, h, w, np.float32, scale=5.0)
    t_ref, lhat_ref, st_ref = oracle.tonemap(img, **TM)
    outs, lhats, stats = P.tonemap_global([to_dev(img, dev)], torch.float32, torch.float32, **TM)
    st = P.stats_to_host(stats)[0]
    name = "%s %dx%d" % (kind, h, w)
    if h * w > 1:
        _check_stats(st, st_ref, name)
        check_f32(outs[0].cpu().numpy(), t_ref, name + " T")
    else:
        assert st["sigma"] == 0.0 and outs[0].item() == 0.5
    check_f32(lhats[0].cpu().numpy(), lhat_ref, name + " Lhat", rel=kind != "u8")


def test_two_pixel_closed_form(dev):
    img = np.array([[[200, 10, 10], [10, 20, 200]]], np.uint8)
    outs, _, _ = P.tonemap_global([to_dev(img, dev)], **TM)
    got = sorted(outs[0].cpu().numpy().ravel())
    want = [1 / (1 + math.exp(2.0)), 1 / (1 + math.exp(-2.0))]
    report("two-pixel T %s vs %s" % (got, want))
    assert got == pytest.approx(want, abs=1e-5)


def test_constant_image_is_one_half(dev):
    for img in (np.full((33, 65, 3), 77, np.uint8), np.full((7, 9, 3), 3.5, np.float16)):
        outs, _, stats = P.tonemap_global([to_dev(img, dev)], **TM)
        assert torch.all(outs[0] == 0.5)
        assert P.stats_to_host(stats)[0]["sigma"] == 0.0


def test_u8_output_codes(dev):
    img = synth.gradient_rects()
    t_ref, _, _ = oracle.tonemap(img, **TM)
    outs, _, _ = P.tonemap_global([to_dev(img, dev)], torch.uint8, **TM)
    check_u8(outs[0].cpu().numpy(), t_ref, "tonemap u8", max_fraction=1e-3)


def test_lhat_matches_decolorize(dev):
    img = synth.hdr_pixels(np.random.default_rng(3), 77, 190)
    x = to_dev(img, dev)
    _, lhats, _ = P.tonemap_global([x], torch.float32, torch.float32, **TM)
    assert torch.equal(lhats[0], P.decolorize(x))


def test_result_independent_of_batch(dev):
    """Each image's T and statistics are bit-identical alone and in a mix."""
    rng = np.random.default_rng(9)
    imgs = []
    for i in range(9):
        h, w = (int(v) for v in rng.integers(1, 400, 2))
        imgs.append(synth.hdr_pixels(rng, h, w) if i % 2 else synth.sdr_pixels(rng, h, w))
    xs = [to_dev(a, dev) for a in imgs]
    mix_t, _, mix_st = P.tonemap_global(xs, torch.float32, **TM)
    mix_st = P.stats_to_host(mix_st)
    for i, x in enumerate(xs):
        t, _, st = P.tonemap_global([x], torch.float32, **TM)
        assert torch.equal(t[0], mix_t[i]), i
        assert P.stats_to_host(st)[0] == mix_st[i], i
    for i in (0, 1):
        t_ref, _, st_ref = oracle.tonemap(imgs[i], **TM)
        _check_stats(mix_st[i], st_ref, "mix image %d" % i)
        check_f32(mix_t[i].cpu().numpy(), t_ref, "mix image %d T" % i)


def test_pitched_and_unaligned_views(dev):
    big = synth.random_image(11, 50, 96, np.uint8)
    for x0, name in ((16, "aligned rows"), (1, "odd-offset rows")):
        view = big[:, x0:x0 + 70]
        t_ref, _, st_ref = oracle.tonemap(view, **TM)
        outs, _, stats = P.tonemap_global([to_dev(big, dev)[:, x0:x0 + 70]], **TM)
        _check_stats(P.stats_to_host(stats)[0], st_ref, name)
        check_f32(outs[0].cpu().numpy(), t_ref, name + " T")


def test_tonemap_plan_and_graph_replays(dev):
    rng = np.random.default_rng(12)
    imgs = [synth.hdr_pixels(rng, 300, 200), synth.sdr_pixels(rng, 77, 1000)]
    xs = [to_dev(a, dev) for a in imgs]
    want, _, want_st = P.tonemap_global(xs, torch.float32, **TM)
    want_st = want_st.clone()
    for graph in (False, True):
        outs = [torch.empty(x.shape[:2], device=dev) for x in xs]
        st = torch.zeros_like(want_st)
        plan = P.Plan(P.PLAN_TONEMAP, xs, outs, stats=st, graph=graph, **TM)
        s = torch.cuda.Stream()
        for rep in range(4):
            for o in outs:
                o.fill_(2.0)
            st.zero_()
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                plan.run(s)
            s.synchronize()
            for a, b in zip(outs, want):
                assert torch.equal(a, b), (graph, rep)
            assert torch.equal(st, want_st), (graph, rep)
        plan.close()


def test_autotune_tonemap_keeps_results(dev):
    t0 = P.get_tuning()
    try:
        img = synth.hdr_pixels(np.random.default_rng(13), 1024, 1024)
        x = to_dev(img, dev)
        ref, _, ref_st = P.tonemap_global([x], **TM)
        out = torch.empty_like(ref[0])
        chosen = P.autotune(P.PLAN_TONEMAP, [x], [out], **TM)
        report("tone-map autotune chose %s" % chosen)
        t, _, st = P.tonemap_global([x], **TM)
        assert torch.equal(t[0], ref[0]) and torch.equal(st, ref_st)
    finally:
        P.set_tuning(t0)


@pytest.mark.parametrize("graph,group", [(False, 1), (True, 1), (False, 2), (True, 3),
                                         (False, 64)])
def test_two_stream_pipeline_matches_batch_schedule(dev, graph, group):
    """The two-stream schedule (groups of `group` images; runs of one input
    type split into chunks) gives the batch schedule's bits, also when captured
    into a graph and replayed."""
    rng = np.random.default_rng(14)
    imgs = [synth.hdr_pixels(rng, 700, 513), synth.sdr_pixels(rng, 64, 64),
            synth.hdr_pixels(rng, 1, 4097), synth.sdr_pixels(rng, 333, 1000),
            synth.hdr_pixels(rng, 90, 91), synth.sdr_pixels(rng, 5, 3000),
            synth.hdr_pixels(rng, 256, 256)]
    xs = [to_dev(a, dev) for a in imgs]
    t0 = P.get_tuning()
    try:
        P.set_tuning(dict(t0, tonemap_pipeline=0))
        want, _, want_st = P.tonemap_global(xs, torch.float32, **TM)
        torch.cuda.synchronize()
        P.set_tuning(dict(t0, tonemap_pipeline=group, pass1_grid_per_cu=2, pass2_grid_per_cu=4))
        got, _, got_st = P.tonemap_global(xs, torch.float32, **TM)
        torch.cuda.synchronize()
        for a, b in zip(got, want):
            assert torch.equal(a, b)
        assert torch.equal(got_st, want_st)
        outs = [torch.empty(x.shape[:2], device=dev) for x in xs]
        st = torch.zeros_like(want_st)
        plan = P.Plan(P.PLAN_TONEMAP, xs, outs, stats=st, graph=graph, **TM)
        s = torch.cuda.Stream()
        for rep in range(3):
            for o in outs:
                o.fill_(-1.0)
            st.zero_()
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                plan.run(s)
            s.synchronize()
            for a, b in zip(outs, want):
                assert torch.equal(a, b), rep
            assert torch.equal(st, want_st), rep
        plan.close()
    finally:
        P.set_tuning(t0)


def test_low_variance_image_within_derived_bound(dev):
    """sigma far below the 0.1 of the other tests: T moves by up to c / (4 s)
    times the FP32 error of x, s = max(sigma, sigma_floor). The bound below is
    that slope times 4e-7 (1 + |x|) (log2, rcp and sqrt rounding of x and of the
    statistics), plus the 1e-5 of well-conditioned images."""
    rng = np.random.default_rng(15)
    base = np.array([0.4, 0.35, 0.3])
    img = (base * (1.0 + 0.002 * rng.standard_normal((96, 80, 3)))).astype(np.float32)
    t_ref, lhat_ref, st_ref = oracle.tonemap(img, **TM)
    outs, _, stats = P.tonemap_global([to_dev(img, dev)], **TM)
    st = P.stats_to_host(stats)[0]
    s = max(st_ref["sigma"], TM["sigma_floor"])
    xmax = float(np.max(np.abs(np.log(lhat_ref + TM["eps"]))))
    bound = 1e-5 + TM["contrast"] / (4 * s) * 4e-7 * (1 + xmax)
    err = float(np.max(np.abs(outs[0].cpu().numpy() - t_ref)))
    report("low-variance image: sigma %.2e, |dT| %.2e, derived bound %.2e" % (st_ref["sigma"], err,
                                                                          bound))
    assert err <= bound


def _t_fp32_bound(st_ref, lhat_ref):
    """The FP32 conditioning term of T: c / (4 s) times 4e-7 (1 + |x|max), with
    s = max(sigma, sigma_floor) (T's slope in x is at most c / (4 s); x and the
    statistics carry log2, rcp and sqrt rounding of about 4e-7 (1 + |x|))."""
    s = max(st_ref["sigma"], TM["sigma_floor"])
    xmax = float(np.max(np.abs(np.log(lhat_ref + TM["eps"]))))
    return TM["contrast"] / (4 * s) * 4e-7 * (1 + xmax), xmax


@pytest.mark.parametrize("sigma", [0.5, 0.2, 0.1, 0.06, 0.04, 0.02, 0.01, 3e-3, 1e-3, 3e-4])
def test_t_tolerance_over_sigma(dev, sigma):
    """Where |dT| <= 1e-5 holds: images whose x = ln(Lhat + eps) has standard
    deviation sigma (a fixed colour scaled by exp(sigma n), n standard normal).
    With sigma_star = c 4e-7 (1 + |x|max) / (4e-5), the sigma at which the FP32
    term of _t_fp32_bound reaches 1e-5 (about 0.045 for c = 2 and |x| <= 1.3),
    T must be within 1e-5 for sigma >= sigma_star and within 1e-5 plus that
    term below it."""
    rng = np.random.default_rng(int(sigma * 1e6))
    base = np.array([0.4, 0.35, 0.3])
    scale = np.exp(sigma * rng.standard_normal((64, 96, 1)))
    img = (base * scale).astype(np.float32)
    t_ref, lhat_ref, st_ref = oracle.tonemap(img, **TM)
    outs, _, _ = P.tonemap_global([to_dev(img, dev)], **TM)
    term, xmax = _t_fp32_bound(st_ref, lhat_ref)
    sigma_star = TM["contrast"] * 4e-7 * (1 + xmax) / (4 * 1e-5)
    err = float(np.max(np.abs(outs[0].cpu().numpy() - t_ref)))
    bound = 1e-5 if st_ref["sigma"] >= sigma_star else 1e-5 + term
    report("sigma %.2e (sigma_star %.3f): |dT| %.2e, bound %.2e" % (st_ref["sigma"], sigma_star,
                                                                    err, bound))
    assert err <= bound


def test_infinite_channels(dev):
    """+Inf channels of a binary16 image read as 65504 and of a binary32 image
    as 1e18 (NaN and -Inf as 0): the tone map stays finite and matches the
    oracle, L-hat included."""
    rng = np.random.default_rng(16)
    for dtype, special in ((np.float16, [np.inf, -np.inf, np.nan]),
                           (np.float32, [np.inf, -np.inf, np.nan, 5e18])):
        img = synth.hdr_pixels(rng, 40, 70).astype(dtype)
        for i, v in enumerate(special):
            img[3 + i, 5:9, i % 3] = v
        img[0, 0, :] = np.inf
        t_ref, lhat_ref, st_ref = oracle.tonemap(img, **TM)
        outs, lhats, stats = P.tonemap_global([to_dev(img, dev)], torch.float32, torch.float32,
                                              **TM)
        name = "inf %s" % np.dtype(dtype).name
        assert np.all(np.isfinite(outs[0].cpu().numpy()))
        _check_stats(P.stats_to_host(stats)[0], st_ref, name)
        check_f32(outs[0].cpu().numpy(), t_ref, name + " T")
        check_f32(lhats[0].cpu().numpy(), lhat_ref, name + " Lhat", rel=True)


def test_hdr_storage_error_against_exact_radiance(dev):
    """The HDR error stated a second way: the GPU result from the binary16
    image against the FP64 oracle on the radiance it stores before rounding
    (passed as FP32, 2^-24 relative). Each binary16 channel is within 2^-11
    relative of that radiance, and L is degree-1 homogeneous and monotone in
    every channel, so L moves by at most 2^-11 relative (plus the kernel's
    1e-5). Then x = ln(Lhat + eps) and mu move by at most 2^-11 and sigma by at
    most 2 * 2^-11; with z = (x - mu) / sigma, dT = T (1 - T) c dz, and since
    T (1 - T) <= 1/4 and T (1 - T) |c z| <= 0.224 (the logistic's largest
    u sigma'(u)), |dT| <= (c / 4) (2 * 2^-11) / sigma + 0.224 (2 * 2^-11) / sigma,
    plus the kernel's 1e-5."""
    img = synth.hdr_pixels(np.random.default_rng(123), 256, 256)
    exact = synth.hdr_pixels(np.random.default_rng(123), 256, 256, exact=True).astype(np.float32)
    outs, lhats, _ = P.tonemap_global([to_dev(img, dev)], torch.float32, torch.float32, **TM)
    lhat_ref = oracle.decolorize(exact)
    rel = float(np.max(np.abs(lhats[0].cpu().numpy() - lhat_ref) / lhat_ref))
    t_ref, _, st = oracle.tonemap(exact, **TM)
    dt = float(np.max(np.abs(outs[0].cpu().numpy() - t_ref)))
    half = 2.0 ** -11
    bound_t = (TM["contrast"] / 4 + 0.224) * (2 * half) / st["sigma"] + 1e-5
    report("binary16 storage: max rel |dL| %.3e (bound %.3e), max |dT| %.3e (bound %.3e)" %
           (rel, half + 1e-5, dt, bound_t))
    assert rel <= half + 1e-5
    assert dt <= bound_t


def test_combine_publication_across_workgroups(dev):
    """The one-launch combine publishes each group partial for the workgroup
    that completes its image. Two batches of different shapes alternate 24
    times through the same context (its workspace slots hold the other
    batch's partials and counters in between); every run's statistics and T
    must repeat the first run's bits, and match the oracle."""
    rng = np.random.default_rng(31)
    a = [synth.hdr_pixels(rng, 1100, 900), synth.sdr_pixels(rng, 2000, 1500),
         synth.hdr_pixels(rng, 64, 64)]
    b = [synth.sdr_pixels(rng, 517, 3001), synth.hdr_pixels(rng, 2048, 2048)]
    batches = [[to_dev(x, dev) for x in a], [to_dev(x, dev) for x in b]]
    first = [None, None]
    for rep in range(24):
        k = rep % 2
        outs, _, st = P.tonemap_global(batches[k], **TM)
        torch.cuda.synchronize()
        if first[k] is None:
            first[k] = (outs, st)
            for img, s in zip(a if k == 0 else b, P.stats_to_host(st)):
                _, _, ref = oracle.tonemap(img, **TM)
                _check_stats(s, ref, "batch %d" % k)
        else:
            assert torch.equal(st, first[k][1]), rep
            for o, w in zip(outs, first[k][0]):
                assert torch.equal(o, w), rep
