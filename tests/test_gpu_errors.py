"""Error paths of the compute ABI on a GPU: every documented rejection returns
its status (no partial work, no abort) and the context stays usable after it."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2108_13656_amd as P
import synth
from gpuhelp import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _status(fn, *a, **kw):
    with pytest.raises(P.DecolorError) as e:
        fn(*a, **kw)
    assert P.last_error()
    return e.value.status


def test_graph_plan_needs_a_stream(dev):
    x = to_dev(synth.random_image(81, 16, 16, np.uint8), dev)
    o = torch.empty((16, 16), device=dev)
    plan = P.Plan(P.PLAN_DECOLORIZE, [x], [o], graph=True)
    rc = P.lib().dc_plan_run(plan._h, ctypes.c_void_p(0))
    assert rc == P.DC_ERR_INVALID_ARG
    plan.close()


def test_bad_tuning_and_autotune_kind(dev):
    t = P.get_tuning()
    assert _status(P.set_tuning, dict(t, groups=[3, 2, 2])) == P.DC_ERR_INVALID_ARG
    assert _status(P.set_tuning, dict(t, pass1_grid_per_cu=65)) == P.DC_ERR_INVALID_ARG
    assert P.get_tuning() == t
    x = to_dev(synth.random_image(82, 8, 8, np.uint8), dev)
    o = torch.empty((8, 8), device=dev)
    assert _status(P.autotune, P.PLAN_LOCAL, [x], [o]) == P.DC_ERR_INVALID_ARG


def test_bad_parameters_rejected_before_any_work(dev):
    x = to_dev(synth.random_image(83, 8, 8, np.uint8), dev)
    o = torch.full((8, 8), -7.0, device=dev)
    assert _status(P.decolorize, x, out=o, beta_r=1.5) == P.DC_ERR_INVALID_ARG
    assert _status(P.tonemap_global, [x], outs=[o], eps=0.0) == P.DC_ERR_INVALID_ARG
    assert _status(P.tonemap_local, [x], outs=[o], strength=2.0) == P.DC_ERR_INVALID_ARG
    assert _status(P.tonemap_global, [x], outs=[torch.empty((8, 8, 3), device=dev)],
                   colour=True, saturation=3.0) == P.DC_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((o == -7.0).all())  # nothing was written
    # the context still works
    assert float(P.decolorize(x).max()) <= 1.0


def test_output_overlapping_input_rejected(dev):
    buf = torch.zeros(64 * 64 * 3, dtype=torch.uint8, device=dev)
    x = buf.view(64, 64, 3)
    alias = buf[: 64 * 64].view(64, 64)  # u8 output over the input's first bytes
    assert _status(P.decolorize, x, out=alias) == P.DC_ERR_ALIAS
    assert _status(P.tonemap_local, [x], outs=[alias]) == P.DC_ERR_ALIAS


def test_unknown_channel_and_plan_kind(dev):
    x = to_dev(synth.random_image(84, 8, 8, np.uint8), dev)
    o = torch.empty((8, 8), device=dev)
    arr = (P.DcImage * 1)(P._image(x, o, None))
    ctx = P.context(dev).handle
    assert P.lib().dc_channel_batch(ctx, arr, 1, 9, None) == P.DC_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert P.lib().dc_plan_create(ctx, 7, arr, 1, None, None, None, 0, ctypes.byref(h)) == \
        P.DC_ERR_INVALID_ARG
    assert not h.value


def test_failed_allocation_reported_and_recovered(dev):
    """A server whose budget the device cannot hold (1 TiB): creation fails with
    DC_ERR_NO_MEMORY, nothing is left half-built, and the next calls on the
    context run and report DC_OK (the failed allocation's error does not leak
    into their launch checks)."""
    x = to_dev(synth.sdr_pixels(np.random.default_rng(5), 64, 80), dev)
    want = P.decolorize(x)
    with pytest.raises(P.DecolorError) as e:
        P.Server(budget_bytes=1 << 40)
    assert e.value.status == P.DC_ERR_NO_MEMORY
    assert "arena" in P.last_error()
    assert torch.equal(P.decolorize(x), want)
    outs, _, _ = P.tonemap_global([x])
    srv = P.Server(budget_bytes=1 << 24)
    srv.close()
    torch.cuda.synchronize()
    assert outs[0].shape == (64, 80)
