"""GPU parity of the weight-sweep explorer (dc_decolorize_batch_betas: every
image of a batch with its own beta_R, beta_k, as in Fig. 4) against the FP64
oracle, and bit-identity with single calls at the same weights."""
import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f32, need_gpu, to_dev

pytestmark = pytest.mark.gpu
BETAS = [(br, bk) for br in (0.0, 0.3, 0.55, 0.8, 1.0) for bk in (0.2, 0.5, 0.8, 1.0)]


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def test_colour_ramps_sweep(dev):
    ramps = synth.colour_ramps(256)
    for name, img in ramps.items():
        got = P.beta_sweep(to_dev(img, dev), BETAS).cpu().numpy()
        for i, (br, bk) in enumerate(BETAS):
            check_f32(got[i], oracle.decolorize(img, br, bk), "%s beta (%g, %g)" % (name, br, bk))


# (input, height, width, output type). The planes of an (n, H, W) output start
# wherever H * W * (output bytes) puts them (123 x 517 FP32 planes, for one,
# are not 16-byte aligned); every image of the call has the same walk either
# way, so the call runs as one pass over the input (the shared-input sweep
# kernel), and must equal single calls bit for bit.
SWEEP_CASES = [("u8", 123, 517, torch.float32), ("u8", 128, 517, torch.float32),
               ("u8", 64, 250, torch.uint8), ("u8", 96, 130, torch.float16),
               ("f16", 64, 1000, torch.float32), ("f16", 64, 1000, torch.float16),
               ("f32", 40, 77, torch.float32), ("f32", 33, 48, torch.uint8)]


def _sweep_image(kind, h, w, seed):
    rng = np.random.default_rng(seed)
    if kind == "u8":
        return synth.sdr_pixels(rng, h, w)
    if kind == "f16":
        return synth.hdr_pixels(rng, h, w)
    return synth.random_image(seed, h, w, np.float32, scale=8.0)


@pytest.mark.parametrize("kind,h,w,odt", SWEEP_CASES)
def test_sweep_equals_single_calls(dev, kind, h, w, odt):
    img = _sweep_image(kind, h, w, 31 + h)
    x = to_dev(img, dev)
    sweep = P.beta_sweep(x, BETAS, out_dtype=odt)
    for i, (br, bk) in enumerate(BETAS):
        one = P.decolorize(x, odt, beta_r=br, beta_k=bk)
        assert torch.equal(sweep[i], one), (br, bk)
    if odt != torch.float32:
        return
    got = sweep.cpu().numpy()
    for i in (0, 7, len(BETAS) - 1):
        br, bk = BETAS[i]
        check_f32(got[i], oracle.decolorize(img, br, bk), "%s (%g, %g)" % (kind, br, bk),
                  rel=kind != "u8")


@pytest.mark.parametrize("kind", ["u8", "f16"])
@pytest.mark.parametrize("npairs", [2, 7, 20, 45])
def test_sweep_pair_chunks(dev, npairs, kind):
    """More pairs than the image has tiles to spread over: the pairs split into
    chunks (the last one short) and every output still equals a single call."""
    rng = np.random.default_rng(40 + npairs)
    img = synth.sdr_pixels(rng, 300, 400) if kind == "u8" else synth.hdr_pixels(rng, 300, 400)
    betas = [(float(a), float(b)) for a, b in rng.uniform(0.0, 1.0, (npairs, 2))]
    x = to_dev(img, dev)
    sweep = P.beta_sweep(x, betas)
    for i, (br, bk) in enumerate(betas):
        assert torch.equal(sweep[i], P.decolorize(x, beta_r=br, beta_k=bk)), (i, br, bk)
    got = sweep.cpu().numpy()
    for i in (0, npairs - 1):
        check_f32(got[i], oracle.decolorize(img, *betas[i]), "pair %d of %d" % (i, npairs),
                  rel=kind != "u8")


def test_sweep_row_walk(dev):
    """A sweep into padded output rows (input rows of 624 bytes), 16-byte
    aligned (output rows of 848 bytes) and not (844 bytes)."""
    img = synth.sdr_pixels(np.random.default_rng(47), 70, 208)
    x = to_dev(img, dev)
    for pad in (4, 3):
        bufs = [torch.full((70, 208 + pad), -1.0, device=dev) for _ in BETAS[:6]]
        P.decolorize_betas([x] * 6, BETAS[:6], outs=[b[:, :208] for b in bufs])
        for buf, (br, bk) in zip(bufs, BETAS[:6]):
            assert torch.equal(buf[:, :208], P.decolorize(x, beta_r=br, beta_k=bk)), (pad, br, bk)
            assert bool((buf[:, 208:] == -1.0).all())


def test_mixed_images_and_weights(dev):
    imgs = [synth.sdr_pixels(np.random.default_rng(34), 50, 60),
            synth.hdr_pixels(np.random.default_rng(35), 30, 700),
            synth.random_image(36, 3, 5, np.float32)]
    betas = [(0.9, 0.6), (0.55, 0.8), (0.1, 0.95)]
    xs = [to_dev(a, dev) for a in imgs]
    outs = P.decolorize_betas(xs, betas, torch.float16)
    for x, o, (br, bk) in zip(xs, outs, betas):
        assert torch.equal(o, P.decolorize(x, torch.float16, beta_r=br, beta_k=bk))


def test_rejects_bad_weights(dev):
    x = to_dev(synth.random_image(37, 4, 4, np.uint8), dev)
    with pytest.raises(P.DecolorError) as e:
        P.decolorize_betas([x, x], [(0.5, 0.5), (1.5, 0.5)])
    assert e.value.status == P.DC_ERR_INVALID_ARG
