"""Batches of thousands of tiny images of mixed types in one call: every
image's result against the oracle (decolorization, global and local tone map)
and against a call on it alone, exercising descriptor tables, the tile-owner
search and the per-type runs far from the benchmark's shapes."""
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


@pytest.fixture(scope="module")
def tiny(dev):
    rng = np.random.default_rng(71)
    imgs = []
    for i in range(3000):
        h, w = (int(v) for v in rng.integers(1, 21, 2))
        dt = (np.uint8, np.float16, np.float32)[i % 3]
        imgs.append(synth.random_image(1000 + i, h, w, dt, scale=3.0))
    return imgs, [to_dev(a, dev) for a in imgs]


def test_decolorize_batch_of_3000(dev, tiny):
    imgs, xs = tiny
    outs = P.decolorize_batch(xs)
    worst = 0.0
    for a, o in zip(imgs, outs):
        want = oracle.decolorize(a)
        got = o.cpu().numpy().astype(np.float64)
        worst = max(worst, float(np.max(np.abs(got - want) / np.maximum(1.0, want))))
    report("3000 tiny images: max scaled error %.3e" % worst)
    assert worst <= 1e-5


@pytest.mark.parametrize("local", [False, True])
def test_tonemap_batch_of_3000(dev, tiny, local):
    imgs, xs = tiny
    fn = P.tonemap_local if local else P.tonemap_global
    outs, _, _ = fn(xs, torch.float32, **TM)
    worst = 0.0
    for i in range(0, len(xs), 97):
        ref = (oracle.tonemap_local(imgs[i], **TM)[0] if local else oracle.tonemap(imgs[i], **TM)[0])
        worst = max(worst, float(np.max(np.abs(outs[i].cpu().numpy() - ref))))
        one = fn([xs[i]], torch.float32, **TM)[0][0]
        assert torch.equal(one, outs[i]), i
    report("3000 tiny images, %s tone map: max |dT| %.3e on every 97th" %
           ("local" if local else "global", worst))
    assert worst <= 1e-5


def test_empty_batches_are_no_ops(dev):
    assert P.decolorize_batch([]) == []
    assert P.tonemap_global([]) == ([], None, None)
    assert P.tonemap_local([]) == ([], None, None)
    assert P.channel_batch([], "y601") == []
