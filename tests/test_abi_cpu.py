"""C-ABI checks that need no GPU: the library loads, exports every function
include/decolor.h declares, and its host-side validation returns the
documented status for each kind of bad argument."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2108_13656_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "decolor.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dc_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libdecolor.so is not built (run __graft_entry__.build())")
    return P.lib()


def test_header_declares_entry_points():
    names = _declared_functions()
    for want in ("dc_create", "dc_destroy", "dc_validate", "dc_decolorize", "dc_decolorize_batch",
                 "dc_tonemap_global", "dc_status_string", "dc_last_error_message", "dc_version"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], stdout=subprocess.PIPE,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (dc_\w+)$", out, flags=re.M))
    for name in _declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_version_and_status_strings(lib):
    assert lib.dc_version() == 1
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.dc_status_string(code).decode()
    assert lib.dc_status_string(-99).decode() == "unknown status"


def test_struct_layouts_match_header():
    assert ctypes.sizeof(P.DcImage) == 72
    assert ctypes.sizeof(P.DcStats) == 24
    assert ctypes.sizeof(P.DcParams) == 8
    assert ctypes.sizeof(P.DcTmParams) == 20


def _img(**kw):
    # Fake device addresses: dc_validate never dereferences them.
    d = dict(src=0x10000000, dst=0x20000000, dst2=None, src_pitch=30, dst_pitch=40, dst2_pitch=0,
             width=10, height=4, src_dtype=P.DC_U8, dst_dtype=P.DC_F32, dst2_dtype=P.DC_NONE,
             flags=0)
    d.update(kw)
    return P.DcImage(**d)


def test_validate_accepts_good_images(lib):
    assert P.validate([_img()]) == P.DC_OK
    assert P.validate([]) == P.DC_OK
    assert P.validate([_img(dst2=0x30000000, dst2_dtype=P.DC_U8, dst2_pitch=10)]) == P.DC_OK
    assert P.validate([_img(src_dtype=P.DC_F16, src_pitch=64)]) == P.DC_OK
    assert P.validate([_img()], tm=(1e-4, 2.0, 1e-3)) == P.DC_OK


@pytest.mark.parametrize("kw", [
    dict(src=None), dict(dst=None), dict(width=0), dict(height=-1), dict(flags=8),
    dict(src_dtype=3), dict(dst_dtype=-1), dict(dst2_dtype=7, dst2=0x30000000, dst2_pitch=40),
    dict(dst2=0x30000000), dict(dst2_dtype=P.DC_F32), dict(src_pitch=29), dict(dst_pitch=39),
    dict(src_dtype=P.DC_F16, src_pitch=59), dict(src_dtype=P.DC_F32, src=0x10000002, src_pitch=120),
    dict(dst=0x20000001), dict(src_pitch=1 << 62, height=8),
])
def test_validate_rejects_bad_image(lib, kw):
    assert P.validate([_img(**kw)]) == P.DC_ERR_INVALID_ARG
    assert P.last_error()


@pytest.mark.parametrize("beta_r,beta_k", [(float("nan"), 0.8), (0.55, 1.5), (-0.1, 0.8),
                                           (0.55, float("inf"))])
def test_validate_rejects_bad_params(lib, beta_r, beta_k):
    assert P.validate([_img()], beta_r=beta_r, beta_k=beta_k) == P.DC_ERR_INVALID_ARG


@pytest.mark.parametrize("tm", [(0.0, 2.0, 1e-3), (1e-4, -2.0, 1e-3), (1e-4, 2.0, 0.0),
                                (float("nan"), 2.0, 1e-3)])
def test_validate_rejects_bad_tm(lib, tm):
    assert P.validate([_img()], tm=tm) == P.DC_ERR_INVALID_ARG


TM = (1e-4, 2.0, 1e-3, 1.0)


def test_colour_output_flag(lib):
    """DC_IMG_RGB_OUT: tone map only; dst rows hold 3 channels."""
    rgb = dict(flags=P.DC_IMG_RGB_OUT, dst_pitch=120)
    assert P.validate([_img(**rgb)], tm=TM) == P.DC_OK
    assert P.validate([_img(**rgb)]) == P.DC_ERR_UNSUPPORTED  # not a tone map
    assert P.validate([_img(flags=P.DC_IMG_RGB_OUT, dst_pitch=119)], tm=TM) == \
        P.DC_ERR_INVALID_ARG
    assert P.validate([_img(flags=P.DC_IMG_RGB_OUT | 4, dst_pitch=120)], tm=TM) == \
        P.DC_ERR_INVALID_ARG
    # host inputs are for server requests only
    assert P.validate([_img(flags=P.DC_IMG_HOST_SRC)], tm=TM) == P.DC_ERR_UNSUPPORTED
    assert P.validate([_img(flags=P.DC_IMG_HOST_SRC)]) == P.DC_ERR_UNSUPPORTED
    # the 3-channel extent (3 * 120 + 120 = 480 bytes) counts for aliasing
    assert P.validate([_img(**rgb), _img(src=0x40000000, dst=0x20000000 + 480)], tm=TM) == P.DC_OK
    assert P.validate([_img(**rgb), _img(src=0x40000000, dst=0x20000000 + 476)], tm=TM) == \
        P.DC_ERR_ALIAS


@pytest.mark.parametrize("s,ok", [(0.0, True), (0.6, True), (2.0, True), (-0.01, False),
                                  (2.01, False), (float("nan"), False), (float("inf"), False)])
def test_saturation_range(lib, s, ok):
    rc = P.validate([_img(flags=P.DC_IMG_RGB_OUT, dst_pitch=120)], tm=(1e-4, 2.0, 1e-3, s))
    assert rc == (P.DC_OK if ok else P.DC_ERR_INVALID_ARG)


@pytest.mark.parametrize("strength,ok", [(0.0, True), (0.5, True), (1.0, True), (-0.01, False),
                                         (1.01, False), (float("nan"), False)])
def test_local_strength_range(lib, strength, ok):
    rc = P.validate([_img()], tm=(1e-4, 2.0, 1e-3, 1.0, strength))
    assert rc == (P.DC_OK if ok else P.DC_ERR_INVALID_ARG)


def test_validate_rejects_negative_count_and_null_list(lib):
    p = P.DcParams(0.55, 0.8)
    assert lib.dc_validate(None, 1, ctypes.byref(p), None) == P.DC_ERR_INVALID_ARG
    assert lib.dc_validate(None, -1, ctypes.byref(p), None) == P.DC_ERR_INVALID_ARG
    assert lib.dc_validate(None, 0, None, None) == P.DC_OK


def test_validate_alias(lib):
    # dst inside src
    assert P.validate([_img(dst=0x10000000 + 8)]) == P.DC_ERR_ALIAS
    # dst and dst2 overlap
    assert P.validate([_img(dst2=0x20000000 + 16, dst2_dtype=P.DC_U8, dst2_pitch=10)]) == P.DC_ERR_ALIAS
    # across images: output of image 1 overlaps input of image 0
    a = _img()
    b = _img(src=0x40000000, dst=0x10000000 + 100)
    assert P.validate([a, b]) == P.DC_ERR_ALIAS
    # two images writing the same output
    assert P.validate([_img(), _img(src=0x40000000)]) == P.DC_ERR_ALIAS
    # shared input is fine
    assert P.validate([_img(), _img(dst=0x50000000)]) == P.DC_OK
    # adjacent, non-overlapping outputs are fine: dst extent is 3*40+40 = 160 bytes
    assert P.validate([_img(), _img(dst=0x20000000 + 160)]) == P.DC_OK
    assert P.validate([_img(), _img(dst=0x20000000 + 156)]) == P.DC_ERR_ALIAS


def test_batch_validation_is_all_or_nothing(lib):
    assert P.validate([_img(), _img(dst=0x50000000, width=0)]) == P.DC_ERR_INVALID_ARG
    assert "image 1" in P.last_error()


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.dc_create(ctypes.byref(h), 0) == P.DC_ERR_NO_DEVICE
    assert not h.value
    assert lib.dc_destroy(None) == P.DC_OK
    assert lib.dc_create(None, 0) == P.DC_ERR_INVALID_ARG


def test_compute_calls_reject_null_context(lib):
    d = _img()
    p = P.DcParams(0.55, 0.8)
    assert lib.dc_decolorize(None, ctypes.byref(d), ctypes.byref(p), None) == P.DC_ERR_INVALID_ARG
    assert lib.dc_decolorize_batch(None, ctypes.byref(d), 1, ctypes.byref(p), None) == \
        P.DC_ERR_INVALID_ARG
    assert lib.dc_tonemap_global(None, ctypes.byref(d), 1, ctypes.byref(p), None, None, None) == \
        P.DC_ERR_INVALID_ARG
    assert lib.dc_decolorize_batch_betas(None, ctypes.byref(d), 1, ctypes.byref(p), None) == \
        P.DC_ERR_INVALID_ARG
    assert lib.dc_tonemap_local(None, ctypes.byref(d), 1, ctypes.byref(p), None, None, None) == \
        P.DC_ERR_INVALID_ARG
    assert lib.dc_tonemap_global_noalloc(None, ctypes.byref(d), 1, ctypes.byref(p), None, None,
                                         None) == P.DC_ERR_INVALID_ARG


def test_binding_refuses_cpu_tensors():
    import torch
    x = torch.zeros((4, 4, 3), dtype=torch.uint8)
    with pytest.raises(TypeError):
        P.decolorize(x)


def test_server_calls_reject_bad_arguments(lib):
    cfg = P.DcServerConfig(1 << 20, 8, 2, 0, P.DcParams(0.55, 0.8), P.DcTmParams(1e-4, 2.0, 1e-3, 1.0, 0.5))
    h = ctypes.c_void_p()
    assert lib.dc_server_create(None, ctypes.byref(cfg), ctypes.byref(h)) == P.DC_ERR_INVALID_ARG
    assert lib.dc_server_create(None, ctypes.byref(cfg), None) == P.DC_ERR_INVALID_ARG
    assert lib.dc_server_step(None) == P.DC_ERR_INVALID_ARG
    assert lib.dc_server_submit(None, None, 0, -1.0) == P.DC_ERR_INVALID_ARG
    assert lib.dc_server_poll(None, None, 0) == P.DC_ERR_INVALID_ARG
    assert lib.dc_server_cancel(None, 7) == P.DC_ERR_INVALID_ARG
    assert lib.dc_server_host_stats(None, None, None) == P.DC_ERR_INVALID_ARG
    assert lib.dc_server_destroy(None) == P.DC_OK
    assert lib.dc_plan_destroy(None) == P.DC_OK
    assert lib.dc_plan_run(None, None) == P.DC_ERR_INVALID_ARG
