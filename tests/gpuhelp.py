"""Shared helpers of the GPU parity tests: tolerances, comparisons, reporting."""
import sys

import numpy as np
import pytest
import torch

F32_ABS_TOL = 1e-5  # FP32 output vs the FP64 oracle on the [0, 1] scale
F32_REL_TOL = 1e-5  # linear (HDR) inputs: relative to the oracle value
U8_MAX_LSB = 1      # 8-bit outputs: at most one code apart
U8_MAX_MISMATCH_FRACTION = 1e-4


def report(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2108_13656_amd as P
    P.lib()  # raises if the HIP library is not built
    return torch.device("cuda", 0)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


F32_FLUSH = 1e-30    # linear inputs: results below this may be flushed (absolute error < 1e-30)


def check_f32(got, want_lhat, what, rel=False):
    """FP32 output against the oracle.

    rel=False: |got - want| <= 1e-5 (absolute, outputs on the [0, 1] scale).
    rel=True: |got - want| <= 1e-5 |want| + 1e-30, a true relative bound for
    radiance from linear inputs, with the documented flush floor only.
    rel="lightness": relative to max(1, |want|), for CIE L* / 100 from linear
    inputs, a perceptual scale whose value near 0 is a difference of two
    nearly equal terms, so 1e-5 is absolute below 1 and relative above.
    Reports the worst error in the same measure."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want_lhat, np.float64)
    err = np.abs(got - want)
    if rel is True:
        ok = err <= F32_REL_TOL * np.abs(want) + F32_FLUSH
        with np.errstate(divide="ignore", invalid="ignore"):
            relerr = np.where(np.abs(want) >= F32_FLUSH, err / np.abs(want), 0.0)
        worst = float(np.max(relerr)) if err.size else 0.0
        kind = "relative"
    else:
        scale = np.maximum(1.0, np.abs(want)) if rel == "lightness" else 1.0
        ok = err / scale <= (F32_REL_TOL if rel else F32_ABS_TOL)
        worst = float(np.max(err / scale)) if err.size else 0.0
        kind = "scaled" if rel else "abs"
    report("%s: max %s error %.3e over %d px" % (what, kind, worst, err.size))
    assert bool(np.all(ok)), "%s: %d values outside the bound (worst %s %.3e)" % (
        what, int(np.count_nonzero(~ok)), kind, worst)
    return worst


def u8_mismatches_at_ties(got, want, slack=255.0 * F32_ABS_TOL):
    """Largest distance, in code units, between the oracle's unrounded value
    255 * want and the midpoint of the two codes wherever the GPU code differs
    from the oracle's: every such pixel must sit within the FP32 error of a
    rounding midpoint (the kernel rounds its FP32 value, the oracle its FP64
    value, and only near a midpoint can the two round apart). Returns that
    distance (0 when no code differs) after asserting it is <= slack."""
    import oracle
    want = np.asarray(want, np.float64)
    codes = oracle.encode_u8(want).astype(np.int32)
    got = np.asarray(got).astype(np.int32)
    off = got != codes
    if not np.any(off):
        return 0.0
    mid = (got[off] + codes[off]) / 2.0
    dist = float(np.max(np.abs(255.0 * want[off] - mid)))
    assert dist <= slack, "a code differs away from a rounding midpoint (%.3e)" % dist
    return dist


def check_u8(got, want, what, max_fraction=U8_MAX_MISMATCH_FRACTION):
    """8-bit GPU codes vs the oracle's min(255, floor(255 want + 0.5)) of its
    unrounded values want (the [0, 1] scale): at most one code apart, only at
    rounding midpoints (u8_mismatches_at_ties), in at most max_fraction of
    the pixels."""
    import oracle
    got = np.asarray(got).astype(np.int32)
    codes = oracle.encode_u8(np.asarray(want, np.float64)).astype(np.int32)
    diff = np.abs(got - codes)
    n_off = int(np.count_nonzero(diff))
    frac = n_off / max(1, diff.size)
    assert int(diff.max() if diff.size else 0) <= U8_MAX_LSB, what
    dist = u8_mismatches_at_ties(got, want)
    report("%s: u8 max |diff| %d, %d of %d codes off by one (fraction %.3e), all within %.2e "
           "of a rounding midpoint" % (what, int(diff.max()) if diff.size else 0, n_off, diff.size,
                                       frac, dist))
    assert frac <= max_fraction, what
    return frac


def check_f16(got_half, want_half, what):
    """GPU binary16 output vs the oracle's round-to-nearest-even encoding of the
    FP64 value: equal, or one binary16 step apart where FP32 rounding moved the
    value across a rounding midpoint."""
    g = np.asarray(got_half, np.float16).astype(np.float64)
    w = np.asarray(want_half, np.float16).astype(np.float64)
    step = np.spacing(np.abs(w).astype(np.float16)).astype(np.float64)
    bad = np.abs(g - w) > step
    n_off = int(np.count_nonzero(g != w))
    report("%s: f16 %d of %d values one step off" % (what, n_off, g.size))
    assert not np.any(bad), what
