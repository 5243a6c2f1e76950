"""Host logic of the benchmark (no GPU): the byte counters are reported only
while they belong to the current meet-kernel sources, and more than one GPU
is refused before anything touches a device."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_only_for_the_current_kernel_sources(tmp_path):
    fp = bench.kernel_fingerprint()
    assert len(fp) == 16 and int(fp, 16) >= 0
    good = tmp_path / "t.json"
    good.write_text(json.dumps({"source_sha256_16": fp, "bytes_per_launch": 123.0}))
    assert bench.measured_traffic(str(good)) == 123.0
    stale = tmp_path / "s.json"
    stale.write_text(json.dumps({"source_sha256_16": "0" * 16, "bytes_per_launch": 123.0}))
    assert bench.measured_traffic(str(stale)) is None
    broken = tmp_path / "b.json"
    broken.write_text("{")
    assert bench.measured_traffic(str(broken)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.json")) is None
    multi = tmp_path / "m.json"
    multi.write_text(json.dumps({"source_sha256_16": fp, "kernels": {
        "k_a": {"bytes_per_launch": [10.0, 20.0]}, "k_b": {"bytes_per_launch": []}}}))
    assert bench.measured_traffic(str(multi), "k_a") == 15.0
    assert bench.measured_traffic(str(multi), "k_b") is None
    assert bench.measured_traffic(str(multi), "k_c") is None


def test_fingerprint_ignores_comments_only():
    """The counters stay valid across comment edits (the compiler sees the
    same code) and not across code edits; literals keep their slashes."""
    code = 'int f(int x) {\n    return x + 1;   // one more\n}\n/* a\n block */\nconst char *s = "a // b /* c */";\n'
    same = '// header\nint f(int x) {\n\n    return x + 1;\n}\nconst char *s = "a // b /* c */";  \n'
    other = code.replace("x + 1", "x + 2")
    assert bench.strip_comments(code) == bench.strip_comments(same)
    assert bench.strip_comments(code) != bench.strip_comments(other)
    assert '"a // b /* c */"' in bench.strip_comments(code)
    assert "one more" not in bench.strip_comments(code) and "block" not in bench.strip_comments(code)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_roofline_object_uses_12_bytes_per_move():
    """Algorithmic bytes per walk step: an 8-byte row read and a 4-byte edge
    read; the fraction is against the published 8 TB/s HBM peak."""
    r = bench.roofline("k", moves=4e9, seconds=0.01, traffic=5e10, traffic_source="profile")
    assert r["bytes_per_move"] == 12
    assert abs(r["achieved"] - 12 * 4e9 / 0.01 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    assert abs(r["achieved_8B_gather_layout"] - 8 * 4e9 / 0.01 / 1e9) < 1e-6
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["traffic"] == 5e10
    assert r["traffic_source"] == "profile" and r["bound"] == "random-gather"
    assert bench.roofline("k", 1.0, 0.0)["achieved"] == 0.0
