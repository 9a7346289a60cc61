"""bench.py: refuses more than one GPU with a message (single-GPU build), and
reports counter traffic only where the counters apply."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_multi_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_traffic_only_for_its_workload(tmp_path, monkeypatch):
    """The HBM traffic from the committed counters is reported only for the
    kernel sources and the workload they were taken on."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    f = tmp_path / "pmc.json"
    f.write_text(json.dumps({"sources_sha256": bench.kernel_sources_sha256(), "workload": "W",
                             "kernels": {"jacobi_fp64": [{"kernel": "rpk::k_jacobi_sliced<double, true, true>",
                                                          "traffic_bytes_per_launch": 123.0}]}}))
    monkeypatch.setattr(bench, "PMC_FILE", str(f))
    assert bench.pmc_traffic("jacobi_fp64", "rpk::k_jacobi_sliced<double", "W") == 123.0
    assert bench.pmc_traffic("jacobi_fp64", "rpk::k_jacobi_sliced<double", "another") is None
    assert bench.pmc_traffic("jacobi_fp64", "rpk::k_jacobi_tile<double, 2>", "W") is None
    f.write_text(json.dumps({"sources_sha256": "0" * 64, "workload": "W", "kernels": {}}))
    assert bench.pmc_traffic("jacobi_fp64", None, "W") is None
