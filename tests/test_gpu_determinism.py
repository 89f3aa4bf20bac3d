"""Bitwise repeatability of every reduction on the path: the tone maps'
statistics (fixed chunks, fixed merge trees, no float atomics) and the local
map's histograms (integer atomics) must give the same bits on every run, under
every launch shape and schedule the tuner can pick, and whatever else shares
the batch; so must the weight sweep."""
import numpy as np
import pytest
import torch

import paper_2108_13656_amd as P
import synth
from gpuhelp import need_gpu, to_dev

pytestmark = pytest.mark.gpu
RUNS = 100


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def batch(dev):
    rng = np.random.default_rng(90)
    imgs = [synth.sdr_pixels(rng, 301, 517), synth.hdr_pixels(rng, 640, 480),
            synth.random_image(91, 129, 255, np.float32, scale=50.0), synth.hdr_pixels(rng, 77, 1031)]
    return [to_dev(a, dev) for a in imgs]


def _global(xs):
    outs, _, st = P.tonemap_global(xs)
    return outs, st


def _local(xs):
    outs, _, st = P.tonemap_local(xs)
    return outs, st


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a[0], b[0])) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("fn", [_global, _local], ids=["global", "local"])
def test_hundred_runs_same_bits(dev, batch, fn):
    want = fn(batch)
    torch.cuda.synchronize()
    bad = [r for r in range(RUNS) if not _same(fn(batch), want)]
    assert not bad, "runs %s differ" % bad[:10]


def test_launch_shapes_and_schedules_same_bits(dev, batch):
    t0 = P.get_tuning()
    try:
        want = _global(batch)
        for pipe in (0, 1):
            for g1 in (0, 1, 4, 16):
                for g2 in (0, 2, 8):
                    t = dict(t0)
                    t.update(tonemap_pipeline=pipe, pass1_grid_per_cu=g1, pass2_grid_per_cu=g2)
                    P.set_tuning(t)
                    assert _same(_global(batch), want), (pipe, g1, g2)
    finally:
        P.set_tuning(t0)


def test_batch_mixes_same_bits(dev, batch):
    """Each image's T and statistics do not depend on the other images of the
    call, their number or their order."""
    alone = [_global([x]) for x in batch]
    for order in ([3, 1, 0, 2], [2, 2, 0], [1, 3]):
        outs, st = _global([batch[i] for i in order])
        for k, i in enumerate(order):
            assert torch.equal(outs[k], alone[i][0][0]), (order, i)
            assert torch.equal(st[k], alone[i][1][0]), (order, i)


def test_sweep_same_bits(dev, batch):
    x = batch[0]
    betas = [(0.1 * i, 1.0 - 0.1 * i) for i in range(11)]
    want = P.beta_sweep(x, betas)
    for _ in range(20):
        assert torch.equal(P.beta_sweep(x, betas), want)
