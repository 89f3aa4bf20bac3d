"""GPU tests of the continuous-batching tone-map server (dc_server_*): every
request's result is bit-identical alone and inside a mixed continuous batch,
admission by the device-memory budget never deadlocks, oversized requests are
rejected, queued requests can be cancelled, and trace replay completes every
request."""
import numpy as np
import pytest
import torch

import paper_2108_13656_amd as P
import synth
from gpuhelp import need_gpu, report, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _mixed_requests(dev, n, seed):
    rng = np.random.default_rng(seed)
    xs, outs = [], []
    for i in range(n):
        h, w = (int(v) for v in np.rint(np.exp(rng.uniform(np.log(16), np.log(700), 2))))
        if i % 3 == 2:
            xs.append(to_dev(synth.hdr_pixels(rng, h, w), dev))
            outs.append(torch.full((h, w), -1.0, device=dev))
        else:
            xs.append(to_dev(synth.sdr_pixels(rng, h, w), dev))
            outs.append(torch.zeros((h, w), dtype=torch.uint8, device=dev))
    return xs, outs


def test_results_identical_alone_and_in_mix(dev):
    xs, outs = _mixed_requests(dev, 40, 1)
    srv = P.Server(budget_bytes=64 << 20, max_batch=16, max_inflight=3)
    srv.submit([P.request_for(i, x, o) for i, (x, o) in enumerate(zip(xs, outs))])
    done = []
    while len(done) < len(xs):
        srv.step()
        done += srv.poll()
    srv.close()
    torch.cuda.synchronize()
    assert sorted(c.id for c in done) == list(range(len(xs)))
    assert all(c.status == P.DC_OK for c in done)
    sizes = [c.batch_size for c in done]
    report("batch sizes seen: %s" % sorted(set(sizes)))
    assert max(sizes) > 1
    for i, (x, o) in enumerate(zip(xs, outs)):
        alone, _, _ = P.tonemap_global([x], o.dtype)
        assert torch.equal(alone[0], o), i


def test_cancel_queued_requests(dev):
    """Requests cancelled before their launch complete with DC_ERR_CANCELLED
    and leave their caller output untouched; a cancel of a request that has
    finished (or never existed) returns False; the rest run as usual."""
    xs, outs = _mixed_requests(dev, 24, 4)
    for o in outs:
        o.fill_(7 if o.dtype == torch.uint8 else 7.0)
    srv = P.Server(budget_bytes=64 << 20, max_batch=4, max_inflight=1)
    srv.submit([P.request_for(i, x, o) for i, (x, o) in enumerate(zip(xs, outs))])
    cancel = {3, 10, 11, 23}
    for i in sorted(cancel):
        assert srv.cancel(i)  # nothing has been stepped: all are still queued
    assert not srv.cancel(1000)
    done = []
    while len(done) < len(xs):
        srv.step()
        done += srv.poll()
    assert not srv.cancel(0)  # already complete
    srv.close()
    torch.cuda.synchronize()
    by_id = {c.id: c for c in done}
    assert sorted(by_id) == list(range(len(xs)))
    for i, (x, o) in enumerate(zip(xs, outs)):
        if i in cancel:
            assert by_id[i].status == P.DC_ERR_CANCELLED
            assert bool((o == 7).all()), i
        else:
            assert by_id[i].status == P.DC_OK
            assert torch.equal(P.tonemap_global([x], o.dtype)[0][0], o), i


def test_cancel_admitted_request(dev):
    """A request that is admitted (its output allocated from the budget) but
    not yet launched can be cancelled: one lane taking one request per
    launch, a budget for two outputs; the first step admits requests 0 and 1
    and launches 0, so 1 is cancelled from the admitted queue, and 2 runs."""
    rng = np.random.default_rng(5)
    xs = [to_dev(synth.sdr_pixels(rng, 256, 256), dev) for _ in range(3)]
    budget = 2 * 256 * 256 * 4 + 4096  # two f32 outputs
    srv = P.Server(budget_bytes=budget, max_batch=1, max_inflight=1)
    srv.submit([P.request_for(i, x, out_dtype=torch.float32) for i, x in enumerate(xs)])
    srv.step()
    assert srv.cancel(1)
    done = []
    while len(done) < 3:
        srv.step()
        done += srv.poll()
    srv.close()
    by_id = {c.id: c for c in done}
    assert by_id[0].status == P.DC_OK and by_id[2].status == P.DC_OK
    assert by_id[1].status == P.DC_ERR_CANCELLED and by_id[1].t_launch == 0.0


def test_budget_admission_and_rejection(dev):
    rng = np.random.default_rng(2)
    xs = [to_dev(synth.sdr_pixels(rng, 300, 400), dev) for _ in range(30)]
    big = to_dev(synth.sdr_pixels(rng, 700, 800), dev)
    # budget holds two 300x400 f32 outputs (rows padded to 16 bytes), not the big one
    budget = 2 * 300 * 1600 + 4096
    srv = P.Server(budget_bytes=budget, max_batch=8, max_inflight=2)
    reqs = [P.request_for(i, x, out_dtype=torch.float32) for i, x in enumerate(xs)]
    reqs.append(P.request_for(99, big, out_dtype=torch.float32))
    srv.submit(reqs)
    done = []
    for _ in range(1000000):
        srv.step()
        done += srv.poll()
        if len(done) == len(reqs):
            break
    srv.close()
    by_id = {c.id: c for c in done}
    assert len(by_id) == len(reqs)
    assert by_id[99].status == P.DC_ERR_NO_MEMORY
    ok = [by_id[i] for i in range(len(xs))]
    assert all(c.status == P.DC_OK for c in ok)
    assert max(c.batch_size for c in ok) <= 2  # never more admitted than the budget holds
    admits = [c.t_admit for c in ok]
    assert admits == sorted(admits)  # FIFO admission


def test_replay_trace_completes(dev):
    xs, outs = _mixed_requests(dev, 60, 3)
    reqs = [P.request_for(i, x, o) for i, (x, o) in enumerate(zip(xs, outs))]
    arrivals = list(np.cumsum(np.random.default_rng(4).exponential(2e-5, len(reqs))) - 2e-5)
    srv = P.Server(budget_bytes=64 << 20, max_batch=32, max_inflight=4)
    done = srv.replay(reqs, arrivals)
    host_s, launches = srv.host_stats()
    srv.close()
    torch.cuda.synchronize()
    assert sorted(c.id for c in done) == list(range(len(reqs)))
    # every completed request rode in some launch; host time was spent on each
    assert 1 <= launches <= len(reqs) and host_s > 0.0
    report("replay: %d launches, %.1f us of host time each" % (launches, 1e6 * host_s / launches))
    lat = np.array([c.t_done - c.t_submit for c in done])
    report("replay latency p50 %.1f us p99 %.1f us" % (1e6 * np.median(lat),
                                                       1e6 * np.quantile(lat, 0.99)))
    assert np.all(lat > 0)
    for c in done:
        assert c.t_submit <= c.t_admit <= c.t_launch <= c.t_done
    for i, (x, o) in enumerate(zip(xs, outs)):
        alone, _, _ = P.tonemap_global([x], o.dtype)
        assert torch.equal(alone[0], o), i


def test_colour_requests_in_mix(dev):
    """Requests with re-coloured RGB outputs (DC_IMG_RGB_OUT) batched with gray
    ones: each equals the direct colour tone map of its image alone."""
    xs, outs = _mixed_requests(dev, 24, 5)
    for i in range(1, len(xs), 2):
        h, w = xs[i].shape[:2]
        outs[i] = torch.zeros((h, w, 3), dtype=torch.uint8 if i % 4 == 1 else torch.float16,
                              device=dev)
    srv = P.Server(budget_bytes=64 << 20, max_batch=16, max_inflight=3, saturation=0.7)
    srv.submit([P.request_for(i, x, o) for i, (x, o) in enumerate(zip(xs, outs))])
    done = []
    while len(done) < len(xs):
        srv.step()
        done += srv.poll()
    srv.close()
    torch.cuda.synchronize()
    assert all(c.status == P.DC_OK for c in done)
    for i, (x, o) in enumerate(zip(xs, outs)):
        alone, _, _ = P.tonemap_global([x], o.dtype, colour=o.dim() == 3, saturation=0.7)
        assert torch.equal(alone[0], o), i


def test_host_input_requests(dev):
    """Requests whose inputs are pinned host tensors (DC_IMG_HOST_SRC): the
    server copies each into its budget before the kernels; results equal the
    device-input tone map bit for bit, alone and mixed with device inputs."""
    xs, outs = _mixed_requests(dev, 20, 7)
    hosts = [x.cpu().pin_memory() if i % 2 == 0 else x for i, x in enumerate(xs)]
    srv = P.Server(budget_bytes=64 << 20, max_batch=8, max_inflight=3)
    srv.submit([P.request_for(i, h, o) for i, (h, o) in enumerate(zip(hosts, outs))])
    done = []
    while len(done) < len(xs):
        srv.step()
        done += srv.poll()
    srv.close()
    torch.cuda.synchronize()
    assert all(c.status == P.DC_OK for c in done)
    for i, (x, o) in enumerate(zip(xs, outs)):
        alone, _, _ = P.tonemap_global([x], o.dtype)
        assert torch.equal(alone[0], o), i


def test_pitched_host_input_requests(dev):
    """Pinned host inputs whose rows are further apart than their bytes (crops
    of a wider pinned image, some starting at an odd element): the server
    gathers the rows into its budget with a copy kernel; results equal the
    device-input tone map bit for bit."""
    rng = np.random.default_rng(12)
    reqs, xs, outs = [], [], []
    for i, (h, w, pad, off) in enumerate([(37, 101, 9, 1), (300, 517, 64, 3), (5, 4099, 1, 0),
                                          (1, 33, 0, 2), (256, 256, 128, 5)]):
        kind = np.uint8 if i % 2 == 0 else np.float16
        img = synth.sdr_pixels(rng, h, w) if kind == np.uint8 else synth.hdr_pixels(rng, h, w)
        t = torch.from_numpy(img)
        pitch = 3 * w + 3 * pad
        buf = torch.zeros(off + h * pitch + 8, dtype=t.dtype).pin_memory()
        view = buf[off:off + h * pitch].view(h, pitch)[:, :3 * w].view(h, w, 3)
        view.copy_(t)
        xs.append(t.to(dev))
        o = torch.empty((h, w), dtype=torch.float32, device=dev)
        outs.append(o)
        reqs.append(P.request_for(i, view, o))
        assert reqs[-1].img.src_pitch == pitch * t.element_size()
    srv = P.Server(budget_bytes=64 << 20, max_batch=4, max_inflight=2)
    srv.submit(reqs)
    done = []
    while len(done) < len(reqs):
        srv.step()
        done += srv.poll()
    srv.close()
    torch.cuda.synchronize()
    assert all(c.status == P.DC_OK for c in done)
    for i, (x, o) in enumerate(zip(xs, outs)):
        alone, _, _ = P.tonemap_global([x], o.dtype)
        assert torch.equal(alone[0], o), i


def test_host_input_budget_counts_the_copy(dev):
    """An input copy larger than the whole budget is rejected at once."""
    x = torch.zeros((512, 512, 3), dtype=torch.float16).pin_memory()
    out = torch.empty((512, 512), device=dev)
    srv = P.Server(budget_bytes=1 << 20, max_batch=4, max_inflight=1)
    srv.submit([P.request_for(0, x, out)])
    done = []
    while not done:
        srv.step()
        done += srv.poll()
    srv.close()
    assert done[0].status == P.DC_ERR_NO_MEMORY
