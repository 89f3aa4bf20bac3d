"""bench.py's host logic: the one-GPU guard, the counter-traffic lookup that
is gated on the kernel source hash recorded in a profile summary, and the
counter rate derived from it."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_traffic_only_from_profiles_of_the_current_source(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "a.md").write_text(
        "source sha256 (k.hip): %s\n\n```\ntraffic_bytes pass_a 1000\ntraffic_bytes pass_b 2000\n```\n"
        % digest)
    (tmp_path / "profiles" / "b.md").write_text(
        "source sha256 (k.hip): %s\n\n```\ntraffic_bytes pass_c 3000\n```\n" % ("0" * 64))
    (tmp_path / "profiles" / "c.md").write_text("no source line\ntraffic_bytes pass_d 4000\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.profiled_traffic() == {"pass_a": 1000, "pass_b": 2000}
    src.write_text("kernel source, changed\n")
    assert b.profiled_traffic() == {}


def test_counter_rate_beside_the_algorithmic_one():
    b = _bench()
    # 2e9 algorithmic bytes at 5000 GB/s = 0.4 ms; 2.2e9 counted bytes in 0.4 ms = 5500 GB/s
    obj = {"x": {"roofline": {"achieved": 5000.0, "algorithmic_bytes": 2e9, "traffic": 2.2e9,
                              "peak": 8000.0}},
           "y": {"achieved": 100.0, "algorithmic_bytes": 1e9, "traffic": None, "peak": 8000.0}}
    out = b.add_traffic_rates(obj)
    r = out["x"]["roofline"]
    assert abs(r["traffic_gbs"] - 5500.0) < 0.1
    assert abs(r["traffic_frac"] - 0.6875) < 1e-4
    assert "traffic_gbs" not in out["y"]


def test_committed_profiles_carry_their_source_and_traffic():
    import glob
    import re
    files = glob.glob(os.path.join(ROOT, "profiles", "*.md"))
    with_traffic = 0
    for fn in files:
        text = open(fn).read()
        if "traffic_bytes" in text:
            with_traffic += 1
            m = re.search(r"source sha256 \((\S+)\): ([0-9a-f]{64})", text)
            assert m and os.path.exists(os.path.join(ROOT, m.group(1))), fn
            assert re.search(r"^rocprofv3 .* -- python3 bench\.py", text, re.M), fn
    assert with_traffic >= 6


def test_valu_slots_from_profiles_and_issue_time(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "a.md").write_text(
        "source sha256 (k.hip): %s\n\n```\nvalu_slots_per_px pass_a 43.47\n"
        "traffic_bytes pass_a 1000\n```\n" % digest)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.profiled_counters("valu_slots_per_px") == {"pass_a": 43.47}
    assert b.profiled_traffic() == {"pass_a": 1000}
    # 43.47 slots/px on 16 x 4096^2 px: 43.47 * 268435456 / (16 * 1024 * 2.4e9) s = 0.2967 ms
    assert abs(b.valu_issue_ms(43.47, 16 * 4096 * 4096) - 0.29675) < 1e-4
