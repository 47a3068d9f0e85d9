"""Host-side checks of the benchmark's reporting (no GPU): the roofline
object's definitions, the traffic record's kernel-version check, and the
one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_reports_algorithmic_flops_against_the_operand_peak():
    # 10 launches of 1e14 algorithmic flops in 1000 ms: 1 PFLOP/s
    r = bench.roofline_of("bf16x3", 1e15, 10, 1000.0, 2.0, 10.0, 1.0, 65536, 1024)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(1000.0)
    assert r["peak"] == 2516.6 and r["frac"] == pytest.approx(1000.0 / 2516.6, abs=1e-4)
    # three MFMA products per complex product are reported beside, not as achieved
    assert r["mfma_issued"]["tflops"] == pytest.approx(3000.0)
    assert r["mfma_issued"]["products_per_complex_product"] == 3
    assert r["avg_launch_ms"] == pytest.approx(100.0) and r["launches"] == 10
    assert r["time_share"]["contract"] == pytest.approx(0.5)
    f = bench.roofline_of("fp32", 1e15, 10, 1000.0, 2.0, 10.0, 1.0, 65536, 1024)
    assert f["peak"] == 157.3 and f["mfma_issued"]["tflops"] == pytest.approx(f["achieved"])
    two = bench.roofline_of("fp16x3", 1e15, 10, 1000.0, 2.0, 10.0, 1.0, 65536, 1024, products=2)
    assert two["kernel"] == "contract_lp_kernel<f16,2>" and two["mfma_issued"]["tflops"] == pytest.approx(2000.0)


def test_roofline_reports_the_measurement_kernel_against_the_hbm_peak():
    # 4 measurement launches moving 1 GB each in 1 ms in all: 4 TB/s of the 8 TB/s peak
    r = bench.roofline_of("fp16f6", 1e15, 10, 1000.0, 2.0, 1.0, 1.0, 65536, 1024, m_bytes=4e9, m_n=4)
    m = r["measure"]
    assert m["bound"] == "hbm" and m["unit"] == "GB/s" and m["peak"] == 8000.0
    assert m["achieved"] == pytest.approx(4000.0) and m["frac"] == pytest.approx(0.5)
    assert m["bytes_per_launch"] == 1000000000 and m["avg_launch_ms"] == pytest.approx(0.25) and m["launches"] == 4
    assert "measure" not in bench.roofline_of("fp16f6", 1e15, 10, 1000.0, 2.0, 1.0, 1.0, 65536, 1024)


def test_traffic_record_is_ignored_for_another_kernel_version(tmp_path, monkeypatch):
    rec = {"kernel_sha": bench.kernel_hash("bf16x3"), "chunk": 65536, "chi": 1024, "bytes_per_launch": 123}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_bf16x3.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda form: rec["kernel_sha"])
    assert bench.traffic_for("bf16x3", 65536, 1024) == 123
    assert bench.traffic_for("bf16x3", 32768, 1024) is None  # taken at another chunk
    assert bench.traffic_for("bf16x3", 65536, 10000) is None  # taken at another bond dimension
    monkeypatch.setattr(bench, "kernel_hash", lambda form: "0" * 16)
    assert bench.traffic_for("bf16x3", 65536, 1024) is None  # source changed since
    assert bench.traffic_for("fp32", 65536, 1024) is None  # no record


def test_more_than_one_gpu_is_refused():
    env = dict(os.environ, WORLD_SIZE="1")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, env=env, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_small_bond_roofline():
    r = bench.roofline_small(3e12, 3, 300.0, 1.0)  # 1e12 flops per 100 ms launch
    assert r["achieved"] == pytest.approx(10.0) and r["peak"] == 157.3
    assert r["kernel"] == "sweep_small_kernel" and r["avg_launch_ms"] == pytest.approx(100.0)
    assert r["time_share"]["sweep_small"] == pytest.approx(0.3)


def test_cpu_baseline_reports_threads_host_and_single_thread_leg():
    """The oracle baseline names the host (nproc, CPU model, BLAS library),
    times an all-threads and a one-thread leg, and the small chain in full."""
    from paper_2512_20064_amd import synth
    t, _, _ = synth.small_chain(2, M=8, d=2, chi_max=8)
    r = bench.cpu_baseline(t, 5, 64, 6, 16)
    assert r["kind"] == "oracle" and r["unit"] == "site-samples/s" and r["value"] > 0
    assert r["cores"] >= 1 and r["single_thread"]["cores"] == 1 and r["single_thread"]["value"] > 0
    assert "0..63" in r["sample"] and "6 sites" in r["sample"]
    h = r["host"]
    assert h["nproc"] >= 1 and h["affinity"] >= 1
    assert h["blas"] is None or h["blas"]["library"]
    s = r["small_chain_full"]
    assert s["value"] > 0 and s["single_thread_value"] > 0 and "N=4096" in s["workload"]


def test_cpu_baseline_takes_the_displacements_of_a_displaced_run():
    """With per-sample displacements the oracle legs run displaced too (the
    same D(mu) per sample and site as the GPU run) and say so."""
    import numpy as np
    from paper_2512_20064_amd import synth
    t, _, _ = synth.small_chain(2, M=8, d=2, chi_max=8)
    rng = np.random.default_rng(3)
    mu = (rng.standard_normal((64, 8)) + 1j * rng.standard_normal((64, 8))) * 0.3
    r = bench.cpu_baseline(t, 5, 64, 6, 16, mu=mu)
    assert r["value"] > 0 and "displaced" in r["sample"]
    assert "displaced" not in bench.cpu_baseline(t, 5, 64, 6, 16)["sample"]

