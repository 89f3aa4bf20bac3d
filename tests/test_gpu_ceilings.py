"""GPU checks of the memory-ceiling kernels the benchmark times
(libdc_ceilings.so, not part of the product): each stream writes every byte
it claims to write, so the ceilings it reports are of the stated traffic.
(Whether the loads happen is shown by the rocprofv3 counters; a load whose
data could be dropped would also drop the store that depends on it.)"""
import ctypes
import os

import pytest
import torch

from gpuhelp import need_gpu, report

pytestmark = pytest.mark.gpu
SENT = 0xAB


@pytest.fixture(scope="module")
def lib():
    need_gpu()
    from paper_2108_13656_amd import build as B
    if not os.path.exists(B.CEIL_LIB):
        pytest.fail("libdc_ceilings.so is not built")
    L = ctypes.CDLL(B.CEIL_LIB)
    sig = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
           ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.dcx_stream.argtypes = sig
    L.dcx_stream12.argtypes = sig
    L.dcx_stage.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.dcx_stage_parked.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]
    return L


def _bufs(nr, nw):
    dev = torch.device("cuda", 0)
    src = torch.arange(nr, dtype=torch.int32, device=dev).to(torch.uint8) if nr else \
        torch.zeros(16, dtype=torch.uint8, device=dev)
    dst = torch.full((max(nw, 16),), SENT, dtype=torch.uint8, device=dev)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    return src, dst, sink


@pytest.mark.parametrize("fn,reads,writes,rb,wb", [
    ("dcx_stream", 0, 8, 0, 1 << 20), ("dcx_stream", 6, 4, 3 << 19, 1 << 20),
    ("dcx_stream", 3, 5, 3 * 81920, 5 * 81920), ("dcx_stream", 4, 4, 1 << 20, 1 << 20),
    ("dcx_stream12", 6, 6, 12 * 98304, 8 * 98304), ("dcx_stream12", 0, 8, 0, 8 * 65536)])
@pytest.mark.parametrize("grid", [0, 7])
def test_streams_write_every_byte(lib, fn, reads, writes, rb, wb, grid):
    src, dst, sink = _bufs(rb, wb)
    s = torch.cuda.current_stream()
    rc = getattr(lib, fn)(src.data_ptr(), rb, dst.data_ptr(), wb, reads, writes, grid,
                          sink.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    assert rc == 0
    # every 4-byte word of the destination holds a value the kernel wrote
    words = dst[:wb].view(torch.int32)
    assert int((words == int.from_bytes(bytes([SENT] * 4), "little", signed=True)).sum()) == 0
    report("%s %d:%d grid %d: %d bytes written" % (fn, reads, writes, grid, wb))


@pytest.mark.parametrize("grid", [0, 5])
def test_lagged_stages_write_every_output(lib, grid):
    nimg, tpi = 3, 4
    dev = torch.device("cuda", 0)
    src = torch.arange(nimg * tpi * 24576, device=dev).to(torch.uint8)
    mid = torch.full((nimg * tpi * 16384,), SENT, dtype=torch.uint8, device=dev)
    out = torch.full((nimg * tpi * 16384,), SENT, dtype=torch.uint8, device=dev)
    out2 = torch.full((nimg * tpi * 16384,), SENT, dtype=torch.uint8, device=dev)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream()
    for st in range(nimg + 1):
        assert lib.dcx_stage(src.data_ptr(), out.data_ptr(), st, nimg, tpi, grid,
                             sink.data_ptr(), s.cuda_stream) == 0
        assert lib.dcx_stage_parked(src.data_ptr(), mid.data_ptr(), out2.data_ptr(), st, nimg,
                                    tpi, grid, sink.data_ptr(), s.cuda_stream) == 0
    torch.cuda.synchronize()
    sent = int.from_bytes(bytes([SENT] * 4), "little", signed=True)
    for name, b in (("two-pass output", out), ("parked intermediate", mid),
                    ("parked output", out2)):
        assert int((b.view(torch.int32) == sent).sum()) == 0, name
    # out-of-range stages and shapes are refused before any launch
    assert lib.dcx_stage(src.data_ptr(), out.data_ptr(), nimg + 1, nimg, tpi, 0,
                         sink.data_ptr(), s.cuda_stream) != 0
    assert lib.dcx_stream(src.data_ptr(), 1 << 20, out.data_ptr(), 1 << 20, 5, 5, 0,
                          sink.data_ptr(), s.cuda_stream) != 0
