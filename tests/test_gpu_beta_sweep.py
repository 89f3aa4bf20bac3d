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


@pytest.mark.parametrize("kind", ["u8", "f16", "f32"])
def test_sweep_equals_single_calls(dev, kind):
    if kind == "u8":
        img = synth.sdr_pixels(np.random.default_rng(31), 123, 517)
    elif kind == "f16":
        img = synth.hdr_pixels(np.random.default_rng(32), 64, 1000)
    else:
        img = synth.random_image(33, 40, 77, np.float32, scale=8.0)
    x = to_dev(img, dev)
    sweep = P.beta_sweep(x, BETAS)
    for i, (br, bk) in enumerate(BETAS):
        one = P.decolorize(x, beta_r=br, beta_k=bk)
        assert torch.equal(sweep[i], one), (br, bk)
    got = sweep.cpu().numpy()
    for i in (0, 7, len(BETAS) - 1):
        br, bk = BETAS[i]
        check_f32(got[i], oracle.decolorize(img, br, bk), "%s (%g, %g)" % (kind, br, bk),
                  rel=kind != "u8")


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
