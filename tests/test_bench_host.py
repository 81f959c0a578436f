"""Host-side logic of bench.py (no GPU): the algorithmic-byte model, the
counter-summary lookup behind roofline.traffic, and the one-GPU guard."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_forces_and_fused_share():
    n, p = 1000, 24000
    assert bench.algorithmic_bytes("forces", n, p, 0, 0) == 58 * n + 4 * p
    # a pass that runs the next step's kick and drift: +48 read, +80 written,
    # no 24 bytes of forces stored
    assert bench.algorithmic_bytes("forces", n, p, 0, 0, fused=1.0) == (58 + 104) * n + 4 * p
    half = bench.algorithmic_bytes("forces", n, p, 0, 0, fused=0.5)
    assert half == pytest.approx((58 + 52) * n + 4 * p)
    assert bench.algorithmic_bytes("density", n, p, 0, 0) == 74 * n + 4 * p


def test_algorithmic_bytes_stage_counts_trials_and_draws():
    n, pmc = 1000, 14000  # 14 pairs per site
    nt, ncells = 500.0, 125.0
    want = nt * (26 + 21 * 14) + ncells * 24
    assert bench.algorithmic_bytes("stage", n, 0, pmc, (nt, ncells)) == pytest.approx(want)
    assert bench.algorithmic_bytes("nonesuch", n, 0, pmc, 0) is None


def _profile(tmp_path, src_text, sha=None, tiling="batch:16", value=12345):
    src = tmp_path / "k.hip"
    src.write_text(src_text)
    digest = sha or hashlib.sha256(src_text.encode()).hexdigest()
    prof = tmp_path / "k_traffic.md"
    lines = ["    kernel: k", f"    source: {src.name}", f"    source_sha256: {digest}",
             f"    traffic_bytes_per_launch: {value}"]
    if tiling:
        lines.insert(1, f"    tiling: {tiling}")
    prof.write_text("# summary\n\n" + "\n".join(lines) + "\n")
    return src, prof


def test_measured_traffic_needs_matching_source_and_tiling(tmp_path, monkeypatch):
    src, prof = _profile(tmp_path, "kernel source v1\n")
    monkeypatch.setitem(bench.TRAFFIC, "t", ("k", str(src), str(prof)))
    assert bench.measured_traffic("t", "batch:16") == 12345
    assert bench.measured_traffic("t", None) == 12345
    assert bench.measured_traffic("t", "stage:1") is None  # other tiling
    src.write_text("kernel source v2\n")  # kernel changed since the counters
    assert bench.measured_traffic("t", "batch:16") is None
    assert bench.measured_traffic("missing-class", "batch:16") is None


def test_measured_traffic_without_tiling_line(tmp_path, monkeypatch):
    src, prof = _profile(tmp_path, "md source\n", tiling=None, value=777)
    monkeypatch.setitem(bench.TRAFFIC, "t2", ("k", str(src), str(prof)))
    assert bench.measured_traffic("t2", "anything:1") == 777


def test_bench_runs_on_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_autotune_cache_key_names_operating_point():
    """The tiling cache separates operating points (the batched pipeline's
    cost depends on how often stages are accepted) and buckets the shape."""
    from paper_1012_5082_amd.autotune import cache_key
    a = cache_key("gfx950", 1, 1956428, 6859, (-0.21919, 1000.0, 0.03, 700.0))
    b = cache_key("gfx950", 1, 1956428, 6859, (-0.22622, 1000.0, 0.03, 700.0))
    c = cache_key("gfx950", 1, 1900000, 7000, (-0.21919, 1000.0, 0.03, 700.0))
    assert a != b and a == c
    assert cache_key("gfx950", 1, 1956428, 6859) != a
