"""GPU parity of the comparator gray channels (rgb2gray Y of Sec. I, V of HSV,
CIE L* on that Y) against the FP64 oracle, through dc_channel_batch."""
import numpy as np
import pytest
import torch

import oracle
import paper_2108_13656_amd as P
import synth
from gpuhelp import check_f32, check_u8, need_gpu, to_dev

pytestmark = pytest.mark.gpu
KINDS = ["y601", "hsv_v", "cielab_l"]


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def all_colours(dev):
    img = synth.all_colours_image()
    return img, to_dev(img, dev)


@pytest.mark.parametrize("kind", KINDS)
def test_all_colours_exhaustive(dev, all_colours, kind):
    img, x = all_colours
    f32, u8 = P.channel_batch([x], kind, torch.float32, torch.uint8)[0]
    want = oracle.comparator_image(img, kind)
    check_f32(f32.cpu().numpy(), want, "all colours " + kind)
    check_u8(u8.cpu().numpy(), want, "all colours u8 " + kind)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dtype", [np.float16, np.float32])
def test_float_inputs(dev, kind, dtype):
    img = synth.random_image(61, 77, 131, dtype, scale=3.0)
    got = P.channel_batch([to_dev(img, dev)], kind)[0].cpu().numpy()
    check_f32(got, oracle.comparator_image(img, kind), "%s %s" % (kind, np.dtype(dtype).name),
              rel="lightness" if kind == "cielab_l" else True)


@pytest.mark.parametrize("kind", KINDS)
def test_mixed_batch_and_views(dev, kind):
    rng = np.random.default_rng(62)
    imgs = [synth.sdr_pixels(rng, 37, 53), synth.hdr_pixels(rng, 64, 129),
            synth.random_image(63, 5, 4099, np.float32), synth.sdr_pixels(rng, 1, 1)]
    xs = [to_dev(a, dev) for a in imgs]
    big = synth.sdr_pixels(rng, 40, 96)
    xs.append(to_dev(big, dev)[:, 1:71])  # a view starting at an odd pixel
    imgs.append(big[:, 1:71])
    outs = P.channel_batch(xs, kind)
    for a, o in zip(imgs, outs):
        check_f32(o.cpu().numpy(), oracle.comparator_image(a, kind), kind + " batch",
                  rel="lightness" if kind == "cielab_l" else True)
