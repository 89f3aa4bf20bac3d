"""The serving loop's admission policy (paper_2108_13656_amd/csrc/serve_policy.h,
the code dc_server_step runs) under simulated launches on the CPU: FIFO
admission, no overlapping or out-of-arena blocks, every request completed
once, only oversized requests rejected, cancels that succeed exactly for
queued requests, a coalesced free list, and the whole arena free again at the
end (tests/serve_sim.cpp checks these and prints "ok").
Several seeds vary the budget, lane count, batch size and request mix."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("serve") / "serve_sim")
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe,
                    os.path.join(HERE, "serve_sim.cpp")], check=True)
    return exe


@pytest.fixture(scope="module")
def sim_sanitized(tmp_path_factory):
    """The same simulation built with AddressSanitizer and UBSan (host code)."""
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("serve_asan") / "serve_sim")
    res = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
                          os.path.join(HERE, "serve_sim.cpp")], capture_output=True, text=True)
    if res.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + res.stderr[-200:])
    return exe


@pytest.mark.parametrize("seed", [1, 5, 9])
def test_policy_under_sanitizers(sim_sanitized, seed):
    out = subprocess.run([sim_sanitized, str(seed)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")


@pytest.mark.parametrize("seed", range(1, 13))
def test_policy_invariants(sim, seed):
    out = subprocess.run([sim, str(seed)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    ok, admitted, rejected, max_in_use, blocked, cancelled = out.stdout.split()
    assert ok == "ok"
    assert int(admitted) > 0 and int(rejected) > 0 and int(max_in_use) > 0
    assert int(blocked) > 0  # the load filled the arena, so the FIFO rule was exercised
    assert int(cancelled) > 0
