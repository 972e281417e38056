"""CPU checks of bench.py's host logic (no GPU): the one-GPU refusal, the
counter summariser's calibration arithmetic, and the rule that the committed
HBM traffic is reported only for the kernel sources and formats it was
measured on."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_pmc_summary_scales_by_the_calibration_kernel(tmp_path):
    # the calibration kernel moves 1 GiB each way; a counter that reads it as
    # 2 GiB (FETCH) or 1 GiB (WRITE) gives factors 0.5 and 1.0
    gib_kib = float(1 << 30) / 1024.0
    fetch, write = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    # (other elementwise kernels, such as the random-number fill of the
    # products mode, are not the calibration kernel)
    calib = "void at::native::vectorized_elementwise_kernel<4, AUnaryFunctor<MulFunctor<double>>>"
    _write_counters(fetch, "FETCH_SIZE", [
        (calib, 2 * gib_kib),
        ("void at::native::distribution_elementwise_grid_stride_kernel<float>", 31.0),
        ("lsqr::k_fwd_lcol<double, double>", 1000.0), ("lsqr::k_fwd_lcol<double, double>", 3000.0),
        ("lsqr::k_adj_npair<double, double, 2>", 500.0)])
    _write_counters(write, "WRITE_SIZE", [
        (calib, gib_kib),
        ("void at::native::distribution_elementwise_grid_stride_kernel<float>", 9.0),
        ("lsqr::k_fwd_lcol<double, double>", 10.0), ("lsqr::k_fwd_lcol<double, double>", 30.0),
        ("lsqr::k_adj_npair<double, double, 2>", 4.0)])
    out = bench.pmc_summary(fetch, write, formats="4/4")
    assert out["FETCH_SIZE_factor"] == pytest.approx(0.5)
    assert out["WRITE_SIZE_factor"] == pytest.approx(1.0)
    assert out["fwd_FETCH_SIZE_bytes"] == pytest.approx(2000.0 * 1024 * 0.5)
    assert out["fwd_WRITE_SIZE_bytes"] == pytest.approx(20.0 * 1024)
    assert out["adj_traffic_bytes"] == pytest.approx(500.0 * 1024 * 0.5 + 4.0 * 1024)
    assert out["formats"] == "4/4" and out["source_sha256_16"] == bench.source_hash()


def test_traffic_only_for_matching_sources_and_formats(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text(f"# comment\nfwd_traffic_bytes 123.0\nadj_traffic_bytes 45.0\n"
                 f"source_sha256_16 {bench.source_hash()}\nformats 4/4\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("fwd", "4/4") == 123.0
    assert bench.measured_traffic("adj", "4/4") == 45.0
    assert bench.measured_traffic("fwd", "1/2") is None           # other formats
    f.write_text("fwd_traffic_bytes 123.0\nsource_sha256_16 0000000000000000\nformats 4/4\n")
    assert bench.measured_traffic("fwd", "4/4") is None           # kernels changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("fwd", "4/4") is None

