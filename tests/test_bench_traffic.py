"""Host logic of the benchmark: the HBM traffic figures, i.e. the FETCH_SIZE /
WRITE_SIZE counter values per dispatch (KiB) of the outer SpMV and of the
level-0 restriction scaled by what the same counters read for a copy kernel of
known size (synthetic counter files), kept only for the layout they were
taken on, and the refusal of runs on more than one GPU."""
import csv
import json
import os
import sys

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)
    return str(path)


def _rows(name, grid, counter, value, count):
    return [{"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value}] * count


LAYOUT_TEXT = ("outer sell1/i32; L0{A sell2/i16/stage, B csr16/t64/glist, P sell2/i16/sorted/stage} "
               "L1{A sell1/i16/sorted/stage, B csr16/t64/glist, P sell2/i16/sorted/stage}")


def test_parse_layouts():
    lay = bench.parse_layouts(LAYOUT_TEXT)
    assert lay == {"spmv": "sell1/i32", "presmooth0": "B csr16/t64/glist",
                   "prolong0": "P sell2/i16/sorted/stage", "postsmooth0": "A sell2/i16/stage"}
    unfused = bench.parse_layouts("outer csr8; L0{A sell1/i32, R csr16/t64/glist, P sell1/i32}")
    assert unfused["presmooth0"] == "A sell1/i32"


def _traffic(tmp_path, monkeypatch):
    kib = bench.COPY_BYTES / 1024.0
    copy_f = _csv(tmp_path / "cf.csv", _rows("at::native::elementwise_kernel", 1, "FETCH_SIZE", kib / 2.0, 3))
    copy_w = _csv(tmp_path / "cw.csv", _rows("at::native::elementwise_kernel", 1, "WRITE_SIZE", kib, 3))
    loop = "k_outer<0, 4, dfamg::SellM<double, 1, false, false> >(...)"
    tuned = "k_outer<0, 4, dfamg::SellM<double, 2, false, false> >(...)"
    restr = "k_restrict<double, double, dfamg::CsrM<double, 16, true> >(...)"
    # outer: in-loop launches 150,000 KiB fetched / 20,000 written; skipped
    # launches after convergence read almost nothing; the tuner's candidate
    # launches of another layout are fewer and must not count.
    # restriction: one instance per level (level 0 moves the most bytes);
    # level 1's launches are as many as level 0's but must not count, nor
    # the tuner's few launches of another layout
    fetch = (_rows(loop, 540000, "FETCH_SIZE", 150000.0, 9) + _rows(loop, 540000, "FETCH_SIZE", 3.0, 4) +
             _rows(tuned, 270000, "FETCH_SIZE", 999999.0, 2) +
             _rows(restr, 2160000, "FETCH_SIZE", 200000.0, 9) + _rows(restr, 290000, "FETCH_SIZE", 50000.0, 9) +
             _rows(restr, 9000000, "FETCH_SIZE", 777777.0, 2))
    write = (_rows(loop, 540000, "WRITE_SIZE", 20000.0, 9) + _rows(loop, 540000, "WRITE_SIZE", 1.0, 4) +
             _rows(tuned, 270000, "WRITE_SIZE", 888888.0, 2) +
             _rows(restr, 2160000, "WRITE_SIZE", 4000.0, 9) + _rows(restr, 290000, "WRITE_SIZE", 600.0, 9) +
             _rows(restr, 9000000, "WRITE_SIZE", 666666.0, 2))
    sf = _csv(tmp_path / "sf.csv", fetch)
    sw = _csv(tmp_path / "sw.csv", write)
    lay = tmp_path / "layouts.json"
    lay.write_text(json.dumps({"fp64": bench.parse_layouts(LAYOUT_TEXT)}))
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.write_traffic(sf, sw, copy_f, copy_w, str(lay)) == 0
    return json.load(open(out))


def test_traffic_scaled_by_copy_calibration(tmp_path, monkeypatch):
    t = _traffic(tmp_path, monkeypatch)["kernels"]
    o = t["spmv"]
    assert abs(o["copy_scale_fetch"] - 2.0) < 1e-12 and abs(o["copy_scale_write"] - 1.0) < 1e-12
    assert o["launches_counted"] == [9, 9] and o["grid"] == 540000
    assert abs(o["fetch_bytes"] - 150000.0 * 2.0 * 1024.0) < 1e-3
    assert abs(o["write_bytes"] - 20000.0 * 1024.0) < 1e-3
    assert abs(o["bytes_per_launch"] - (o["fetch_bytes"] + o["write_bytes"])) < 1e-3
    assert o["kernel_source_hash"] == bench.kernel_source_hash()
    assert o["layout"] == "sell1/i32"
    r = t["presmooth0"]
    assert r["grid"] == 2160000 and r["launches_counted"] == [9, 9]
    assert abs(r["fetch_bytes"] - 200000.0 * 2.0 * 1024.0) < 1e-3
    assert abs(r["write_bytes"] - 4000.0 * 1024.0) < 1e-3
    assert r["layout"] == "B csr16/t64/glist"


def test_column_tiled_restriction_sums_its_two_kernels(tmp_path, monkeypatch):
    # "B seg...": the level-0 restriction is the partial-sum kernel plus the
    # per-row combine; each is taken at its heaviest instance (level 0, whose
    # grid may be smaller than level 1's) and the two are added; the FP32
    # instances of the mixed path do not count
    kib = bench.COPY_BYTES / 1024.0
    copy_f = _csv(tmp_path / "cf.csv", _rows("at::native::elementwise_kernel", 1, "FETCH_SIZE", kib / 2.0, 3))
    copy_w = _csv(tmp_path / "cw.csv", _rows("at::native::elementwise_kernel", 1, "WRITE_SIZE", kib, 3))
    loop = "k_outer<0, 4, dfamg::SellM<double, 1, false, false> >(...)"
    part = "void dfamg::k_seg_partial<double, double, 1024>(...)"
    part1 = "void dfamg::k_seg_partial<double, double, 512>(...)"
    comb = "void dfamg::k_seg_combine<double>(...)"
    combf = "void dfamg::k_seg_combine<float>(...)"
    fetch = (_rows(loop, 540000, "FETCH_SIZE", 150000.0, 9) + _rows(part, 425984, "FETCH_SIZE", 160000.0, 9) +
             _rows(part1, 557056, "FETCH_SIZE", 9000.0, 9) + _rows(comb, 540672, "FETCH_SIZE", 7000.0, 9) +
             _rows(combf, 540672, "FETCH_SIZE", 99999.0, 9))
    write = (_rows(loop, 540000, "WRITE_SIZE", 20000.0, 9) + _rows(part, 425984, "WRITE_SIZE", 8000.0, 9) +
             _rows(part1, 557056, "WRITE_SIZE", 500.0, 9) + _rows(comb, 540672, "WRITE_SIZE", 4200.0, 9) +
             _rows(combf, 540672, "WRITE_SIZE", 99999.0, 9))
    sf = _csv(tmp_path / "sf.csv", fetch)
    sw = _csv(tmp_path / "sw.csv", write)
    text = LAYOUT_TEXT.replace("L0{A sell2/i16/stage, B csr16/t64/glist", "L0{A sell2/i16/stage, B seg8192/b1024")
    lay = tmp_path / "layouts.json"
    lay.write_text(json.dumps({"fp64": bench.parse_layouts(text)}))
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.write_traffic(sf, sw, copy_f, copy_w, str(lay)) == 0
    r = json.load(open(out))["kernels"]["presmooth0"]
    assert r["layout"] == "B seg8192/b1024"
    assert r["grid"] == [425984, 540672] and r["launches_counted"] == [[9, 9], [9, 9]]
    assert abs(r["fetch_bytes"] - (160000.0 + 7000.0) * 2.0 * 1024.0) < 1e-3
    assert abs(r["write_bytes"] - (8000.0 + 4200.0) * 1024.0) < 1e-3
    assert "k_seg_partial" in r["kernel"] and "k_seg_combine<double>" in r["kernel"]


def test_traffic_dropped_when_layout_differs(tmp_path, monkeypatch):
    _traffic(tmp_path, monkeypatch)
    same = bench.parse_layouts(LAYOUT_TEXT)
    assert bench.load_traffic("spmv", same) is not None
    assert bench.load_traffic("presmooth0", same) is not None
    other = dict(same, spmv="sell2/i16/stage")
    assert bench.load_traffic("spmv", other) is None
    assert bench.load_traffic("presmooth0", other) is not None


def test_more_than_one_gpu_is_refused():
    # the solve is measured on one GPU; --gpus above 1 exits with a message
    # before anything touches a device, and prints no result line
    import subprocess
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""
