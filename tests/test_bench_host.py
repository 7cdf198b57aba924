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


def test_counter_record(tmp_path):
    """Counters of two groups (two CSVs) merge per kernel; each averages its
    last 3 dispatches; per-pair figures divide lane-instructions by pixels x S."""
    import numpy as np
    from paper_1407_2343_amd.synth import batch_workload
    row_k = "void snlm::snlm_kernel<10, 3, false, false, true, true>(snlm::KernelArgs)"
    col_k = "void snlm::snlm_kernel<10, 3, false, false, true, false>(snlm::KernelArgs)"
    pairs = sum(img.size for img, _ in batch_workload(64, 128, 1024, seed=2000)) * 10
    a, b = str(tmp_path / "a.csv"), str(tmp_path / "b.csv")
    rows_a = [(d, k, c, v) for k in (row_k, col_k)
              for d in range(1, 6)
              for c, v in (("SQ_INSTS_VALU", pairs * 11 / 64 if d > 2 else 1.0),
                           ("SQ_INSTS_VALU_TRANS_F32", pairs / 64 if d > 2 else 1.0))]
    rows_b = [(d, k, c, v) for k in (row_k, col_k)
              for d in range(11, 16)
              for c, v in (("SQ_WAVE_CYCLES", 1000.0), ("SQ_WAIT_INST_ANY", 250.0), ("SQ_ACTIVE_INST_VALU", 500.0))]
    for path, rows in ((a, rows_a), (b, rows_b)):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=FIELDS)
            w.writeheader()
            for d, k, c, v in rows:
                w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})
    out = str(tmp_path / "counters.json")
    rec = bench.write_counters([a, b], out_path=out)
    for k in (row_k, col_k):
        lr = rec["launches"][k]
        assert np.isclose(lr["valu_per_pair"], 11.0) and np.isclose(lr["trans_per_pair"], 1.0)
        assert lr["wait_inst_share"] == 0.25 and lr["valu_active_share"] == 0.5
    assert np.isclose(rec["step"]["valu_per_pair"], 11.0)
    assert rec["source_sha256"] == bench.source_sha()


def test_serving_overlap(tmp_path):
    """Kernel intervals [0,10) and [5,20) on two queues, plus a kernel of
    another library: busy 20 us, two at once for 5 us."""
    path = str(tmp_path / "trace.csv")
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Queue_Id", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerow({"Kernel_Name": "snlm_kernel<5,2>", "Queue_Id": 1, "Start_Timestamp": 0, "End_Timestamp": 10000})
        w.writerow({"Kernel_Name": "snlm_copy_images", "Queue_Id": 2, "Start_Timestamp": 5000,
                    "End_Timestamp": 20000})
        w.writerow({"Kernel_Name": "elementwise_kernel", "Queue_Id": 3, "Start_Timestamp": 0,
                    "End_Timestamp": 50000})
    r = bench.serving_overlap(path)
    assert r["dispatches"] == 2 and r["busy_us"] == 20.0 and r["max_concurrent"] == 2
    assert r["overlap_share_of_busy"] == 0.25


def _names_oracle(node):
    import ast
    for n in ast.walk(node):
        if isinstance(n, ast.Name) and n.id == "oracle":
            return True
        if isinstance(n, (ast.Import, ast.ImportFrom)):
            mods = [a.name for a in n.names] + ([n.module] if isinstance(n, ast.ImportFrom) and n.module else [])
            if any(m == "oracle" or m.startswith("oracle.") for m in mods):
                return True
    return False


def test_oracle_only_in_cpu_baseline():
    """The oracle is test infrastructure: in bench.py only the cpu_baseline
    leg may import or call it, and no module of the GPU library names it."""
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = [n.name for n in tree.body if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef)) and _names_oracle(n)]
    top = [n for n in tree.body if not isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef)) and _names_oracle(n)]
    assert users == ["cpu_baseline"] and not top, users
    pkg = os.path.join(ROOT, "paper_1407_2343_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                path = os.path.join(dirpath, f)
                assert not _names_oracle(ast.parse(open(path).read())), path
