"""Host logic of bench.py, on the CPU: the code hash that ties the committed
HBM-traffic counters to the kernel sources, the lookup of those counters, the
roofline arithmetic and its algorithmic flop counts, and the one-GPU
contract of the command line."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports numpy only; nothing touches a GPU)


def test_code_hash_ignores_comments_blank_lines_and_indentation(tmp_path):
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {\n    return x + 1;  // one more\n}\n")
    b = tmp_path / "b.hip"
    b.write_text("/* a header\n   over two lines */\nint f(int x) {\n  return x + 1;\n\n}\n// end\n")
    c = tmp_path / "c.hip"
    c.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert bench.code_sha256(str(a)) == bench.code_sha256(str(b))
    assert bench.code_sha256(str(a)) != bench.code_sha256(str(c))


def test_traffic_is_reported_only_for_the_profiled_code_and_tree(tmp_path, monkeypatch):
    src = tmp_path / "paper_0908_0673_amd" / "csrc" / bench.KERNEL_SOURCES["m2l"]
    src.parent.mkdir(parents=True)
    src.write_text("int g() { return 3; }\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "m2l_meshx_hbm_traffic.txt").write_text(
        "# a summary\nkernel: k\nB: 48\ntheta: 0.5\nkappa: 0.0\n"
        f"code_sha256: {bench.code_sha256(str(src))}\nhbm_bytes_per_launch: 1234\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.hbm_traffic("m2l", "meshx", 48, 0.5, 0.0) == 1234.0
    assert bench.hbm_traffic("m2l", "meshx", 64, 0.5, 0.0) is None  # another leaf size
    assert bench.hbm_traffic("m2l", "meshx", 48, 0.55, 0.0) is None  # another separation factor
    assert bench.hbm_traffic("m2l", "meshx", 48, 0.5, 2.2) is None  # another wavenumber bound
    assert bench.hbm_traffic("m2l", "meshy", 48, 0.5, 0.0) is None  # no summary for that mesh
    src.write_text("// a comment added\n   int g() { return 3; }  /* and another */\n\n")
    assert bench.hbm_traffic("m2l", "meshx", 48, 0.5, 0.0) == 1234.0  # same code
    src.write_text("int g() { return 4; }\n")
    assert bench.hbm_traffic("m2l", "meshx", 48, 0.5, 0.0) is None  # the kernel changed


def test_algorithmic_flop_counts():
    stats = {"n_p2p": 10, "n_m2l": 3}
    assert bench.algorithmic_flops(stats, 165, False) == {"p2p": 190.0, "m2l": 2.0 * 165 * 165 * 3}
    assert bench.algorithmic_flops(stats, 165, True) == {"p2p": 370.0, "m2l": 8.0 * 165 * 165 * 3}


def test_roofline_arithmetic():
    r = bench.roofline("m2l", 12.5e9, 0.25, 10, 2.0e8)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["traffic"] == 2.0e8
    assert r["achieved"] == pytest.approx(12.5e9 / 0.25e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.FP32_MFMA_PEAK)
    # three fp16 products per FP32-equivalent one, on 176 x 192 padded tiles of the 165 x 165 operator
    assert r["fp16_executed_tflops"] == pytest.approx(r["achieved"] * 3 * 176 * 192 / 165 ** 2)
    assert r["fp16_frac"] == pytest.approx(r["fp16_executed_tflops"] / bench.FP16_MFMA_PEAK)
    q = bench.roofline("p2p", 6.0e9, 0.2, 10, None)
    assert q["bound"] == "alu" and q["traffic"] is None
    assert q["frac"] == pytest.approx(q["achieved"] / bench.FP32_VEC_PEAK)
    assert q["frac_unpacked"] == pytest.approx(q["achieved"] / bench.FP32_VEC_UNPACKED)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
