"""Host logic of the benchmark: the HBM traffic figure, i.e. the FETCH_SIZE /
WRITE_SIZE counter values per dispatch (KiB) of the outer SpMV scaled by what
the same counters read for a copy kernel of known size (synthetic counter
files), and the refusal of runs on more than one GPU."""
import csv
import json
import os
import sys

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)
    return str(path)


def test_traffic_scaled_by_copy_calibration(tmp_path, monkeypatch):
    kib = bench.COPY_BYTES / 1024.0
    copy_f = _csv(tmp_path / "cf.csv", [{"Kernel_Name": "at::native::elementwise_kernel", "Counter_Name":
                                        "FETCH_SIZE", "Counter_Value": kib / 2.0}] * 3)
    copy_w = _csv(tmp_path / "cw.csv", [{"Kernel_Name": "at::native::elementwise_kernel", "Counter_Name":
                                        "WRITE_SIZE", "Counter_Value": kib}] * 3)
    loop = "void dfamg::k_outer<0, 4, dfamg::SellM<double, 1, false, false> >(...)"
    tuned = "void dfamg::k_outer<0, 4, dfamg::SellM<double, 2, false, false> >(...)"
    # in-loop launches: 150,000 KiB fetched, 20,000 written; skipped launches
    # after convergence read almost nothing; the tuner's candidate launches
    # of another layout are fewer and must not count
    fetch = ([{"Kernel_Name": loop, "Counter_Name": "FETCH_SIZE", "Counter_Value": 150000.0}] * 9 +
             [{"Kernel_Name": loop, "Counter_Name": "FETCH_SIZE", "Counter_Value": 3.0}] * 4 +
             [{"Kernel_Name": tuned, "Counter_Name": "FETCH_SIZE", "Counter_Value": 999999.0}] * 2)
    write = ([{"Kernel_Name": loop, "Counter_Name": "WRITE_SIZE", "Counter_Value": 20000.0}] * 9 +
             [{"Kernel_Name": loop, "Counter_Name": "WRITE_SIZE", "Counter_Value": 1.0}] * 4 +
             [{"Kernel_Name": tuned, "Counter_Name": "WRITE_SIZE", "Counter_Value": 888888.0}] * 2)
    sf = _csv(tmp_path / "sf.csv", fetch)
    sw = _csv(tmp_path / "sw.csv", write)
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.write_traffic(sf, sw, copy_f, copy_w) == 0
    t = json.load(open(out))
    assert abs(t["copy_scale_fetch"] - 2.0) < 1e-12 and abs(t["copy_scale_write"] - 1.0) < 1e-12
    assert t["launches_counted"] == [9, 9]
    assert abs(t["fetch_bytes"] - 150000.0 * 2.0 * 1024.0) < 1e-3
    assert abs(t["write_bytes"] - 20000.0 * 1024.0) < 1e-3
    assert abs(t["bytes_per_launch"] - (t["fetch_bytes"] + t["write_bytes"])) < 1e-3
    assert t["kernel_source_hash"] == bench.kernel_source_hash()


def test_more_than_one_gpu_is_refused():
    # the solve is measured on one GPU; --gpus above 1 exits with a message
    # before anything touches a device, and prints no result line
    import subprocess
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""
