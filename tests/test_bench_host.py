"""Host-side helpers of bench.py (no GPU): the means of the GTEPS convention
and the source-hash gate of the measured traffic, which must report a
committed rocprofv3 figure only while the kernel's source is the one the
counters were taken on."""
import hashlib
import math
import os

import bench


def test_means():
    assert math.isclose(bench.harmonic([1.0, 2.0, 4.0]), 3.0 / 1.75)
    assert math.isclose(bench.geometric([1.0, 4.0, 16.0]), 4.0)
    # sources that found nothing (0 GTEPS) are left out, as the bench does
    assert math.isclose(bench.harmonic([0.0, 2.0, 2.0]), 2.0)
    assert bench.harmonic([]) == 0.0 and bench.geometric([0.0]) == 0.0


def _tree(tmp_path, text):
    csrc = tmp_path / "paper_1803_03922_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text(text)
    (tmp_path / "profiles").mkdir()
    return hashlib.sha256(text.encode()).hexdigest()


def test_traffic_follows_source_hash(tmp_path, monkeypatch):
    h = _tree(tmp_path, "__global__ void k_a() {}\n")
    (tmp_path / "profiles" / "k_a.md").write_text(
        "# summary\n\n"
        f"traffic: kernel=k_a workload=RMAT26_TH32_x source_sha256={h} bytes_per_launch=12345\n"
        f"traffic: kernel=k_b workload=RMAT26_TH32_x source_sha256={h} bytes_per_launch=7\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the workload is matched with spaces written as underscores
    assert bench.measured_traffic("k_a", "RMAT26 TH32 x", "k.hip") == 12345.0
    assert bench.measured_traffic("k_b", "RMAT26_TH32_x", "k.hip") == 7.0
    assert bench.measured_traffic("k_a", "RMAT24 x", "k.hip") is None
    assert bench.measured_traffic("k_c", "RMAT26 TH32 x", "k.hip") is None
    # any change to the kernel's source retires the figure
    (tmp_path / "paper_1803_03922_amd" / "csrc" / "k.hip").write_text(
        "__global__ void k_a() { }\n")
    assert bench.measured_traffic("k_a", "RMAT26 TH32 x", "k.hip") is None


def test_committed_traffic_lines_parse():
    """Every traffic line in profiles/ names a kernel, a workload, a 64-digit
    source hash and a positive byte count."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    seen = 0
    for f in sorted(os.listdir(os.path.join(root, "profiles"))):
        for line in open(os.path.join(root, "profiles", f)):
            if not line.startswith("traffic: "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            assert set(kv) == {"kernel", "workload", "source_sha256", "bytes_per_launch"}, f
            assert len(kv["source_sha256"]) == 64 and int(kv["source_sha256"], 16) >= 0
            assert float(kv["bytes_per_launch"]) > 0
            seen += 1
    assert seen >= 2
