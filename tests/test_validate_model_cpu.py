"""dc_validate's aliasing verdict against a brute-force model on random small
batches (hypothesis): every output's byte extent, (height - 1) * pitch + its
row bytes from its base, must be disjoint from every other output's extent
and from every input's; inputs may overlap one another. The library sorts the
outputs and binary-searches each input; the model compares all pairs."""
import os

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import paper_2108_13656_amd as P

ES = {P.DC_U8: 1, P.DC_F16: 2, P.DC_F32: 4}


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libdecolor.so is not built (run __graft_entry__.build())")


@st.composite
def image(draw):
    w = draw(st.integers(1, 6))
    h = draw(st.integers(1, 4))
    sd = draw(st.sampled_from([P.DC_U8, P.DC_F16, P.DC_F32]))
    dd = draw(st.sampled_from([P.DC_U8, P.DC_F16, P.DC_F32]))
    two = draw(st.booleans())
    d2 = draw(st.sampled_from([P.DC_U8, P.DC_F16, P.DC_F32])) if two else P.DC_NONE
    # addresses on a 4-byte grid in a 1 KB window, so extents often collide
    base = 0x100000
    src = base + 4 * draw(st.integers(0, 250))
    dst = base + 4 * draw(st.integers(0, 250))
    dst2 = base + 4 * draw(st.integers(0, 250)) if two else None
    sp = 3 * ES[sd] * w + 4 * draw(st.integers(0, 3))
    dp = ES[dd] * w + 4 * draw(st.integers(0, 3))
    d2p = ES[d2] * w + 4 * draw(st.integers(0, 3)) if two else 0
    return dict(src=src, dst=dst, dst2=dst2, src_pitch=sp, dst_pitch=dp, dst2_pitch=d2p,
                width=w, height=h, src_dtype=sd, dst_dtype=dd, dst2_dtype=d2, flags=0)


def _extent(base, pitch, row, h):
    return (base, base + pitch * (h - 1) + row)


def _model_aliases(imgs):
    ins, outs = [], []
    for m in imgs:
        w, h = m["width"], m["height"]
        ins.append(_extent(m["src"], m["src_pitch"], 3 * ES[m["src_dtype"]] * w, h))
        outs.append(_extent(m["dst"], m["dst_pitch"], ES[m["dst_dtype"]] * w, h))
        if m["dst2"] is not None:
            outs.append(_extent(m["dst2"], m["dst2_pitch"], ES[m["dst2_dtype"]] * w, h))

    def overlap(a, b):
        return a[0] < b[1] and b[0] < a[1]

    for i, o in enumerate(outs):
        if any(overlap(o, x) for x in ins):
            return True
        if any(overlap(o, x) for j, x in enumerate(outs) if j != i):
            return True
    return False


@settings(max_examples=600, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.lists(image(), min_size=1, max_size=5))
def test_alias_verdict_matches_brute_force(imgs):
    rc = P.validate([P.DcImage(**m) for m in imgs])
    want = P.DC_ERR_ALIAS if _model_aliases(imgs) else P.DC_OK
    assert rc == want, (rc, imgs)
