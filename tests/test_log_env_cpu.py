"""Host-side environment switches, without a GPU: DC_LOG_LEVEL=1 prints each
failing call's message to stderr, and nothing is printed by default."""
import os
import subprocess
import sys

import pytest

import paper_2108_13656_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import ctypes, sys
sys.path.insert(0, %r)
import paper_2108_13656_amd as P
L = P.lib()
p = P.DcParams(2.0, 0.8)  # beta_r out of [0, 1]
rc = L.dc_validate(None, 0, ctypes.byref(p), None)
print("status", rc)
""" % ROOT


def _run(env_extra):
    env = dict(os.environ)
    env.pop("DC_LOG_LEVEL", None)
    env.update(env_extra)
    return subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True,
                          timeout=120)


def test_log_level_prints_failures():
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libdecolor.so is not built")
    quiet = _run({})
    assert "status %d" % P.DC_ERR_INVALID_ARG in quiet.stdout
    assert "[decolor]" not in quiet.stderr
    loud = _run({"DC_LOG_LEVEL": "1"})
    assert "status %d" % P.DC_ERR_INVALID_ARG in loud.stdout
    assert "[decolor] error %d: beta_r and beta_k must be finite" % P.DC_ERR_INVALID_ARG in loud.stderr
