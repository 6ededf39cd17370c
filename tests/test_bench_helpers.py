"""Host logic of bench.py (no GPU): the name of pass B's kernel read back from the
autotuner's cache file, and the measured-traffic figure, which counts only for the
profiled kernel and while the kernel's sources are the profiled ones."""
import json

import bench

KEY_127 = "gfx950|d3|N20|B8|n3|p1|s0"  # 3D, N = 2,048,383, B = 256, n = 40, FP32, RBGS


def _cache(tmp_path, table):
    p = tmp_path / "tiles.json"
    p.write_text(json.dumps(table))
    return str(p)


def test_pass_b_kernel_from_tuner_cache(tmp_path):
    other = "gfx950|d2|N20|B8|n3|p1|s0"
    path = _cache(tmp_path, {KEY_127: [1, 2, 4, 512, 2, 2, 1, 2, 2, 2, 2, 2],
                             other: [1, 4, 4, 512, 1, 1, 1]})
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "fp32", False) == \
        "k_zmarch<2, 1, double, 2, 0, 2>"
    # paired updates of x: the two variants alternate
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "fp32") == \
        "k_zmarch<2, 1, double, 2, 1, 2> / k_zmarch<2, 1, double, 2, 2, 2>"
    # taller tiles (four nodes per thread) only with at most two queries per block
    path = _cache(tmp_path, {KEY_127: [1, 1, 2, 512, 2, 2, 2, 2, 2, 4, 2, 1]})
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "fp32", False) == \
        "k_zmarch<1, 1, double, 4, 0, 1>"
    path = _cache(tmp_path, {KEY_127: [1, 4, 2, 512, 2, 2, 2, 2, 2, 4, 2, 1]})
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "fp32", False) == \
        "k_zmarch<4, 1, double, 2, 0, 1>"
    # a marching pass B without its number of plane buffers: no claim about the kernel
    path = _cache(tmp_path, {KEY_127: [1, 1, 2, 512, 2, 2, 2, 2, 2, 4, 2]})
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "fp32") == "pass B (tiles unknown)"
    path = _cache(tmp_path, {KEY_127: [1, 4, 4, 512, 2, 1]})
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "fp32", False) == "k_pass_b<3, 4, 0>"
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "fp32") == \
        "k_pass_b<3, 4, 1> / k_pass_b<3, 4, 2>"
    # another precision, a missing file, an unreadable file: no claim about the kernel
    assert bench.pass_b_kernel(path, 3, 2048383, 256, 40, "bf16") == "pass B (tiles unknown)"
    assert bench.pass_b_kernel(str(tmp_path / "none.json"), 3, 1, 1, 1, "fp32") == \
        "pass B (tiles unknown)"
    (tmp_path / "bad.json").write_text("{not json")
    assert bench.pass_b_kernel(str(tmp_path / "bad.json"), 3, 1, 1, 1, "fp32") == \
        "pass B (tiles unknown)"


def test_measured_traffic_needs_the_profiled_kernel_and_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    prof = tmp_path / "prof.md"
    prof.write_text(f"text\n\ntraffic_bytes_per_launch: 123456 sources_sha256: {h} "
                    "kernel: k_zmarch<2, 1, double, 2, 1> / k_zmarch<2, 1, double, 2, 2>\n"
                    f"traffic_bytes_per_launch: 654321 sources_sha256: {h} "
                    "kernel: k_zmarch<1, 1, double, 4, 1> / k_zmarch<1, 1, double, 4, 2>\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", "prof.md")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.measured_traffic("3d127", "fp32", 256, "k_zmarch<2, 1, double, 2, 1> / k_zmarch<2, 1, double, 2, 2>") == 123456
    # one line per profiled tile choice
    assert bench.measured_traffic("3d127", "fp32", 256, "k_zmarch<1, 1, double, 4, 1> / k_zmarch<1, 1, double, 4, 2>") == 654321
    assert bench.measured_traffic("3d127", "fp32", 256, "k_pass_b<3, 2>") is None
    assert bench.measured_traffic("3d127", "bf16", 256, "k_zmarch<2, 1, double, 2, 1> / k_zmarch<2, 1, double, 2, 2>") is None
    assert bench.measured_traffic("3d255", "fp32", 64, "k_zmarch<2, 1, double, 2, 1> / k_zmarch<2, 1, double, 2, 2>") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("3d127", "fp32", 256, "k_zmarch<2, 1, double, 2, 1> / k_zmarch<2, 1, double, 2, 2>") is None

