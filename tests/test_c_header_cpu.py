"""The ABI is plain C: include/decolor.h compiles as strict C99 (-pedantic
-Werror), and a C program links against libdecolor.so and validates a
descriptor on the host (no GPU needed): the struct sizes it sees are the ones
the library and the Python binding use."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2108_13656_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include "decolor.h"
#include <stdio.h>

int main(void)
{
    dc_image im = {0};
    im.src = (const void *)0x1000;
    im.dst = (void *)0x100000;
    im.width = 4;
    im.height = 2;
    im.src_dtype = DC_U8;
    im.src_pitch = 12;
    im.dst_dtype = DC_F32;
    im.dst_pitch = 16;
    im.dst2_dtype = DC_NONE;
    dc_params p = {0.55f, 0.8f};
    int ok = dc_validate(&im, 1, &p, NULL);
    im.dst_pitch = 8; /* shorter than a row */
    int bad = dc_validate(&im, 1, &p, NULL);
    printf("%d %d %d %d %d %d %d\n", ok, bad, (int)sizeof(dc_image), (int)sizeof(dc_params),
           (int)sizeof(dc_tm_params), (int)sizeof(dc_stats), dc_version());
    return 0;
}
"""


def test_c_program_uses_the_abi(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libdecolor.so is not built (run __graft_entry__.build())")
    src = tmp_path / "abi.c"
    src.write_text(PROGRAM)
    exe = str(tmp_path / "abi")
    libdir = os.path.dirname(P.LIB_PATH)
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", exe, "-L", libdir,
                    "-ldecolor", "-Wl,-rpath," + libdir], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True, timeout=60).stdout.split()
    ok, bad, s_img, s_par, s_tm, s_st, ver = (int(v) for v in out)
    assert ok == P.DC_OK and bad == P.DC_ERR_INVALID_ARG
    assert s_img == ctypes.sizeof(P.DcImage) == 72
    assert s_par == ctypes.sizeof(P.DcParams)
    assert s_tm == ctypes.sizeof(P.DcTmParams)
    assert s_st == ctypes.sizeof(P.DcStats)
    assert ver == 1
