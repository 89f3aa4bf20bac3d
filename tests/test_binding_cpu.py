"""Host-side argument checks of the Python binding (no GPU): a caller's
statistics tensor is checked before its address reaches the library, which
writes STATS_BYTES per image there on the device."""
import pytest
import torch

import paper_2108_13656_amd as P


def test_stats_tensor_checked_before_the_call():
    cpu = torch.device("cpu")
    ok = torch.empty((3, P.STATS_BYTES), dtype=torch.uint8)
    assert P._stats_ptr(ok, 3, cpu).value == ok.data_ptr()
    assert P._stats_ptr(None, 3, cpu).value in (0, None)
    # any element type, as long as the bytes suffice
    as_f64 = torch.empty((3 * P.STATS_BYTES) // 8, dtype=torch.float64)
    assert P._stats_ptr(as_f64, 3, cpu).value == as_f64.data_ptr()
    with pytest.raises(ValueError, match="holds"):
        P._stats_ptr(torch.empty((2, P.STATS_BYTES), dtype=torch.uint8), 3, cpu)
    with pytest.raises(ValueError, match="contiguous"):
        P._stats_ptr(torch.empty((P.STATS_BYTES, 6), dtype=torch.uint8).t(), 3, cpu)
    with pytest.raises(ValueError, match="device"):
        P._stats_ptr(ok, 3, torch.device("cuda", 0))
    with pytest.raises(ValueError, match="tensor"):
        P._stats_ptr(bytearray(100), 3, cpu)
