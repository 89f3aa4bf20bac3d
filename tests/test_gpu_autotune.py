"""GPU tests of the launch-shape autotuner (dc_autotune): on the batch it was
tuned on, the chosen shapes are never slower than the library's defaults
(within the run-to-run noise of a median over graph replays), and with
DC_AUTOTUNE=0 the call measures nothing and keeps the shapes in place."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import paper_2108_13656_amd as P
import synth
from gpuhelp import need_gpu, report, to_dev

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NOISE = 1.05  # medians over alternating rounds still move by a few per cent


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _plan_ms(plan, s, reps):
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.run(s)
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _compare(kind, xs, outs, stats, tune_a, tune_b, rounds=5, reps=11):
    """Median step time of plans frozen with shapes a and b, measured in
    alternating rounds (so drifts of clock and temperature hit both)."""
    s = torch.cuda.Stream()
    plans = []
    for t in (tune_a, tune_b):
        P.set_tuning(t)
        plans.append(P.Plan(kind, xs, outs, stats=stats, graph=True))
    ta, tb = [], []
    with torch.cuda.stream(s):
        for p in plans:
            for _ in range(3):
                p.run(s)
        for _ in range(rounds):
            ta.append(_plan_ms(plans[0], s, reps))
            tb.append(_plan_ms(plans[1], s, reps))
    for p in plans:
        p.close()
    return float(np.median(ta)), float(np.median(tb))


def _defaults():
    """The shapes a new context starts from (no tuning file applied)."""
    return {"groups": [1, 2, 2], "mixed_groups": 1, "decolor_grid_per_cu": 0,
            "mixed_grid_per_cu": 0, "pass1_grid_per_cu": 16, "pass2_grid_per_cu": 0,
            "tonemap_pipeline": 0}


@pytest.mark.parametrize("kind", ["decolorize", "tonemap"])
def test_tuned_shapes_never_slower_than_defaults(dev, kind):
    rng = np.random.default_rng(5)
    if kind == "decolorize":
        # 48 frames of 1920 x 1080 8-bit: ~0.2 ms per step
        frame = synth.sdr_pixels(rng, 1080, 1920)
        xs = [to_dev(frame, dev) for _ in range(48)]
        pk = P.PLAN_DECOLORIZE
    else:
        # 16 images of 2048 x 2048 binary16: ~0.2 ms per step
        img = synth.hdr_pixels(rng, 2048, 2048)
        xs = [to_dev(img, dev) for _ in range(16)]
        pk = P.PLAN_TONEMAP
    outs = [torch.empty(x.shape[:2], dtype=torch.float32, device=dev) for x in xs]
    stats = torch.empty((len(xs), P.STATS_BYTES), dtype=torch.uint8, device=dev) \
        if kind == "tonemap" else None
    saved = P.get_tuning()
    try:
        P.set_tuning(_defaults())
        chosen = P.autotune(pk, xs, outs)
        t_default, t_tuned = _compare(pk, xs, outs, stats, _defaults(), chosen)
        report("%s: default %.4f ms, tuned %.4f ms (%s)" % (kind, t_default, t_tuned, chosen))
        assert t_tuned <= NOISE * t_default
    finally:
        P.set_tuning(saved)


SCRIPT = r"""
import sys, time
sys.path.insert(0, %r)
import numpy as np, torch
import paper_2108_13656_amd as P
import synth
dev = torch.device("cuda", 0)
xs = [torch.from_numpy(synth.sdr_pixels(np.random.default_rng(1), 512, 512)).to(dev)]
outs = [torch.empty((512, 512), dtype=torch.float32, device=dev)]
before = P.get_tuning()
odd = dict(before, groups=[4, 4, 4], decolor_grid_per_cu=2)
P.set_tuning(odd)
t0 = time.time()
chosen = P.autotune(P.PLAN_DECOLORIZE, xs, outs)
print("same", chosen == odd and P.get_tuning() == odd, "seconds %%.3f" %% (time.time() - t0))
""" % ROOT


def test_autotune_switch_off_keeps_shapes(dev):
    env = dict(os.environ, DC_AUTOTUNE="0", DC_LOG_LEVEL="2")
    env.pop("DC_AUTOTUNE_CACHE", None)
    res = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True,
                         timeout=240)
    report(res.stdout.strip() + " | " + res.stderr.strip()[-200:])
    assert res.returncode == 0, res.stderr[-2000:]
    assert "same True" in res.stdout
    assert "DC_AUTOTUNE=0" in res.stderr
