"""Host-side logic of bench.py (no GPU): the one-GPU contract and the HBM
traffic record built from rocprofv3 counter CSVs."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, name, value in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record(tmp_path):
    """Copy calibration: a 1024 MiB copy that reads FETCH_SIZE = 512 Ki KiB
    and writes WRITE_SIZE = 1 Mi KiB gives the factors 2 and 1.  Each kernel
    averages its last 6 dispatches; bytes = FETCH x 1024 x 2 + WRITE x 1024."""
    row_k = "void snlm::snlm_kernel<10, 3, false, false, true>(snlm::KernelArgs)"
    col_k = "void snlm::snlm_kernel<10, 3, false, false, false>(snlm::KernelArgs)"
    cf, cw = str(tmp_path / "cf.csv"), str(tmp_path / "cw.csv")
    _csv(cf, "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 524288.0)])
    _csv(cw, "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 1048576.0)])
    # 8 dispatches per kernel: the first two (warm-up) are large and must be
    # left out; a counter split over two records of one dispatch is summed
    fetch = [(d, row_k, 1000.0 if d > 2 else 9e9) for d in range(1, 9)]
    fetch += [(d, col_k, 400.0 if d > 12 else 9e9) for d in range(11, 19)]
    fetch += [(d, col_k, 100.0) for d in range(13, 19)]  # second record of the same dispatches
    write = [(d, row_k, 3000.0 if d > 2 else 9e9) for d in range(1, 9)]
    write += [(d, col_k, 2000.0 if d > 12 else 9e9) for d in range(11, 19)]
    f, w = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    _csv(f, "FETCH_SIZE", fetch)
    _csv(w, "WRITE_SIZE", write)
    out = str(tmp_path / "traffic.json")
    rec = bench.write_traffic(f, w, cf, cw, 1024, out_path=out)
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    row, col = rec["launches"][row_k], rec["launches"][col_k]
    assert row["bytes"] == 1000.0 * 1024 * 2 + 3000.0 * 1024
    assert col["FETCH_SIZE_KiB"] == 500.0
    assert col["bytes"] == 500.0 * 1024 * 2 + 2000.0 * 1024
    assert rec["hbm_bytes_per_step"] == int(row["bytes"] + col["bytes"])
    assert rec["source_sha256"] == bench.source_sha()
    assert json.load(open(out)) == rec
