"""Host logic of bench.py, on the CPU: when a committed HBM-traffic record is
reported, the roofline object's arithmetic, and the one-GPU contract."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _record(path, sha, algo, traffic):
    path.write_text("# test record\nkernel = k_rowop<float, 2, 7>\n"
                    f"traffic_bytes_per_launch = {traffic}\n"
                    f"algorithmic_bytes_per_launch = {algo}\n"
                    f"kernel_source_sha256 = {sha}\n")


def test_traffic_record_reported_only_for_the_same_kernels_and_launches(tmp_path, monkeypatch):
    b = _bench()
    key = ("smooth", "test_workload", "mixed")
    rec = tmp_path / "rec.txt"
    monkeypatch.setitem(b.TRAFFIC_FILES, key, str(rec))
    _record(rec, b.kernel_source_hash(), 1000000, 1850000)
    assert b.measured_traffic(*key, 1000000.0) == 1850000.0
    # another launch mix (different algorithmic bytes per launch): not reported
    assert b.measured_traffic(*key, 1000002.0) is None
    # counters taken with other kernel code: not reported
    _record(rec, "0" * 64, 1000000, 1850000)
    assert b.measured_traffic(*key, 1000000.0) is None
    # no record for this kernel class and workload
    assert b.measured_traffic("smooth", "no_such_workload", "mixed", 1.0) is None


def test_committed_traffic_records_are_well_formed():
    b = _bench()
    for (kclass, workload, prec), rel in b.TRAFFIC_FILES.items():
        kv = {}
        for line in open(os.path.join(ROOT, rel)):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        assert kclass in b.KCLASS and len(kv["kernel_source_sha256"]) == 64
        assert os.path.exists(os.path.join(ROOT, kv.get("kernel_source", b.ROW_KERNELS)))
        algo, traffic = float(kv["algorithmic_bytes_per_launch"]), float(kv["traffic_bytes_per_launch"])
        # HBM traffic is at least the algorithmic bytes, and the two counter
        # passes were scaled by a copy calibration
        assert 1.0 <= traffic / algo < 4.0
        assert abs(float(kv["traffic_over_algorithmic"]) - traffic / algo) < 0.01


def test_roofline_object():
    b = _bench()
    r = b.roofline("smooth", 2.0, 8e9, 100)  # 8 GB in 2 ms: 4 TB/s
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 4000.0) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12
    assert r["peak"] == 8000.0 and r["per_unit"] == 8e7 and r["avg_unit_us"] == 20.0
    g = b.roofline("gram", 1.0, 7.86e9, 10)  # 7.86 GFLOP in 1 ms: 7.86 TFLOP/s
    assert g["bound"] == "mfma" and abs(g["frac"] - 0.1) < 1e-12
    assert b.roofline("ritz", 1.0, 0.0, 4)["bound"] == "latency"
    assert b.roofline("smooth", 0.0, 1.0, 1) is None and b.roofline("smooth", 1.0, 1.0, 0) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stdout
