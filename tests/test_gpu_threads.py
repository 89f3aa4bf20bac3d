"""Python threads sharing a device's context: the binding serialises calls on
the context (a dc_ctx serves one host thread at a time), so concurrent callers
on their own streams get exactly the results of sequential calls."""
import threading

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


def test_threads_share_the_context(dev):
    imgs = [synth.hdr_pixels(np.random.default_rng(80 + i), 96 + 16 * i, 200) for i in range(4)] + \
           [synth.sdr_pixels(np.random.default_rng(90 + i), 128, 64 + 32 * i) for i in range(4)]
    xs = [to_dev(a, dev) for a in imgs]
    want_t = [P.tonemap_global([x])[0][0] for x in xs]
    want_l = [P.decolorize(x) for x in xs]
    torch.cuda.synchronize()
    errors = []

    def worker(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep in range(25):
                    i = (k + rep) % len(xs)
                    t = P.tonemap_global([xs[i]], stream=s)[0][0]
                    lum = P.decolorize(xs[i], stream=s)
                    s.synchronize()
                    if not (torch.equal(t, want_t[i]) and torch.equal(lum, want_l[i])):
                        errors.append((k, rep, i))
        except Exception as e:  # reported below, on the main thread
            errors.append((k, repr(e)))

    threads = [threading.Thread(target=worker, args=(k,), daemon=True) for k in range(8)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads)
    assert not errors, errors[:5]
