"""The GPU tests' 8-bit comparison accepts a code that differs from the
oracle's only where the oracle's value sits at a rounding midpoint, and
rejects one anywhere else (checked here on planted codes, no GPU)."""
import numpy as np
import pytest

from gpuhelp import u8_mismatches_at_ties


def test_equal_codes_pass():
    want = np.array([0.0, 0.25, 0.5, 1.0, 1.7])
    codes = np.array([0, 64, 128, 255, 255])  # floor(255 v + 0.5), saturated
    assert u8_mismatches_at_ties(codes, want) == 0.0


def test_difference_at_a_midpoint_passes():
    v = (100.5 + 1e-4) / 255.0  # just above the 100 | 101 midpoint: the oracle says 101
    assert u8_mismatches_at_ties(np.array([100]), np.array([v])) <= 2e-4


def test_difference_away_from_a_midpoint_fails():
    v = 100.3 / 255.0  # the oracle says 100; 101 is no rounding question
    with pytest.raises(AssertionError):
        u8_mismatches_at_ties(np.array([101]), np.array([v]))
