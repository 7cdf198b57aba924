"""Benchmark of separable PatchLift NLM on one MI355X.

One step = one batched launch over the ragged batch workload: 64 FP32 images,
H and W drawn log-uniform in [128, 1024] per axis, sigma drawn from
{10, 20, 30, 40} per image with h = 10 sigma, S = 10, K = 3, box patch kernel,
rows then columns.  Every step runs the whole hot path: reflected loads,
lifting, diagonal running sums, weights, accumulation and normalisation for
both passes of all 64 images, as two persistent launches replayed from one HIP
graph.  Inputs are resident in HBM before timing starts.

The JSON line also carries: the plain single-image launches (the same 64
images one by one, and one 512 x 512 image in the four kernel/order
variants), the roofline of the batched kernels (device time from HIP events
on the stream they run on), the serving workload (2000 requests, Poisson
arrivals, p50/p99 latency and Mpixel/s, against FIFO plain launches), the
precision variants' throughput on 2048 x 2048 and 4096 x 4096 images (their
error against the FP64 oracle is a GPU test), the SURE-optimal combination of
the two orders on a 2048 x 2048 image (``sure_combination``), the recursive
Gaussian patch kernel on a 2048 x 2048 image (``recursive_gaussian``), a
256 x 256 x 256 volume (``volume``), and the
FP64 oracle timed on the host cores on a bounded sample of the batch
(``cpu_baseline``, the only part that runs the oracle).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-serve] [--no-precision] [--no-sure]
                    [--no-iir] [--iir-only] [--no-volume] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

S, K = 10, 3
# FP32 vector peak of MI355X from its unit counts and clock: 256 CUs x 4 SIMDs
# x 32 FP32 lanes per clock x 2.4 GHz = 78.6 T lane-instructions/s (157.3
# TFLOP/s counting an FMA as two).  Measured on the device: plain FP32
# instructions (FMA, add, sub, mul, with or without VOP3 modifiers) from two
# waves of one SIMD issue one wave64 instruction per 2.2 clocks; one wave alone
# issues one per 4.4 clocks.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
# Algorithmic lane-instructions per unordered pair (u, u+s) of one pass, box
# kernel, on the scaled samples: one lifted difference, two fused multiply-adds
# for the window recursion (entering and leaving term), one exp2 for the
# weight, and two fused multiply-adds and two adds for the two accumulations.
# The exp issues from the same VALU (and, measured, stops two waves of one SIMD
# from pairing their FP32 instructions), so it is counted like the others.
PAIR_VALU = 8


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(items, budget_s: float = 12.0, single_budget_s: float = 6.0):
    """The FP64 oracle on the first images of the batch until ~budget_s of
    wall time with every host core, then on the first images again with one
    thread until ~single_budget_s."""
    import oracle
    orc = oracle.load()

    def run(threads, budget):
        px = n = 0
        t0 = time.perf_counter()
        for img, sig in items:
            orc.snlm(img.astype(np.float64), S, K, 10.0 * sig, "box", "row_col", threads=threads)
            px += img.size
            n += 1
            if time.perf_counter() - t0 > budget:
                break
        return px, n, time.perf_counter() - t0

    cores = orc.max_threads()
    px, n, dt = run(cores, budget_s)
    px1, n1, dt1 = run(1, single_budget_s)
    return {"value": round(px / dt / 1e6, 4), "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_thread_mpx_per_s": round(px1 / dt1 / 1e6, 4),
            "sample": "first %d of the 64 batch images (%d px), FP64 direct separable NLM, "
                      "S=10 K=3 box row_col, %.1f s wall on %d threads; single thread: first %d "
                      "images (%d px), %.1f s" % (n, px, dt, cores, n1, px1, dt1)}


def source_sha():
    """SHA-256 over the kernel source and the host planner (both decide the
    bytes a batched step moves)."""
    h = hashlib.sha256()
    for f in ("snlm_device.hpp", "snlm_api.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1407_2343_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_from_profiles():
    """HBM bytes per batched step from the committed counter summary, if it was
    taken on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_batch.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != source_sha():
        return None
    return rec.get("hbm_bytes_per_step")


def write_traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_mib, last=6, out_path=None):
    """Writes profiles/traffic_batch.json from four rocprofv3 --pmc counter
    CSVs: FETCH_SIZE and WRITE_SIZE of a --profile-batch run, and the same two
    counters of a --calibrate-copy run of copy_mib MiB.  Each batched launch
    averages its last `last` dispatches (the timed steps).  Returns the
    record; out_path defaults to profiles/traffic_batch.json."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        vals = defaultdict(dict)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            vals[r["Kernel_Name"]][int(r["Dispatch_Id"])] = \
                vals[r["Kernel_Name"]].get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
        return vals

    def copy_kib(path, counter):
        v = per_kernel(path, counter)
        name = [k for k in v if "copyBuffer" in k][0]
        return max(v[name].values())

    copy_bytes = copy_mib << 20
    ff = copy_bytes / (copy_kib(copy_fetch_csv, "FETCH_SIZE") * 1024.0)
    wf = copy_bytes / (copy_kib(copy_write_csv, "WRITE_SIZE") * 1024.0)
    fv, wv = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    launches = {}
    for name in sorted(k for k in fv if "snlm_kernel" in k):
        f = [fv[name][d] for d in sorted(fv[name])[-last:]]
        w = [wv[name][d] for d in sorted(wv[name])[-last:]]
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        launches[name] = {"FETCH_SIZE_KiB": fk, "WRITE_SIZE_KiB": wk,
                          "bytes": fk * 1024 * ff + wk * 1024 * wf}
    from paper_1407_2343_amd.synth import batch_workload
    px = sum(img.size for img, _ in batch_workload(64, 128, 1024, seed=2000))
    total = sum(v["bytes"] for v in launches.values())
    rec = {"what": "HBM bytes of one batched step (first-pass + second-pass persistent launches) "
                   "of the 64-image ragged batch, S=10 K=3 box row_col",
           "fetch_factor": ff, "write_factor": wf, "launches": launches,
           "hbm_bytes_per_step": int(total), "algorithmic_bytes_per_step": int(px * 16),
           "ratio_to_algorithmic": total / (px * 16), "source_sha256": source_sha()}
    with open(out_path or os.path.join(ROOT, "profiles", "traffic_batch.json"), "w") as fo:
        json.dump(rec, fo, indent=1)
    print(json.dumps({k: rec[k] for k in ("hbm_bytes_per_step", "ratio_to_algorithmic")}))
    return rec


def counters_path():
    return os.path.join(ROOT, "profiles", "counters_batch.json")


def write_counters(csv_paths, last=3, out_path=None):
    """Writes profiles/counters_batch.json from rocprofv3 --pmc CSVs of
    --profile-batch runs (any SQ counters, one group per run).  Per batched
    launch, each counter is the mean over the last `last` dispatches (the timed
    steps) of its sum over shader engines and XCDs.  Derived per launch:
    issued VALU, transcendental and SALU lane-instructions per algorithmic
    unordered pair (pixels x S per pass), the shares of wave time spent issuing
    VALU instructions and waiting, and the issue rates over the dispatch time.
    Returns the record."""
    import csv
    from collections import defaultdict

    per = defaultdict(dict)  # kernel -> counter -> value
    dur = defaultdict(list)
    for path in csv_paths:
        vals = defaultdict(lambda: defaultdict(float))
        span = {}
        for r in csv.DictReader(open(path)):
            k = r["Kernel_Name"]
            if "snlm_kernel" not in k:
                continue
            d = int(r["Dispatch_Id"])
            vals[(k, d)][r["Counter_Name"]] += float(r["Counter_Value"])
            if "Start_Timestamp" in r:
                span[(k, d)] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        kern = defaultdict(list)
        for (k, d) in vals:
            kern[k].append(d)
        for k, ds in kern.items():
            ds = sorted(ds)[-last:]
            for c in vals[(k, ds[0])]:
                per[k][c] = sum(vals[(k, d)][c] for d in ds) / len(ds)
            dur[k] += [span[(k, d)] for d in ds if (k, d) in span]
    from paper_1407_2343_amd.synth import batch_workload
    px = sum(img.size for img, _ in batch_workload(64, 128, 1024, seed=2000))
    pairs = px * S  # unordered pairs of one pass
    launches = {}
    for k, c in per.items():
        rec = {"counters": c, "pairs": pairs}
        ns = sum(dur[k]) / len(dur[k]) if dur[k] else None
        rec["dispatch_ns_under_counters"] = ns
        for name, key in (("valu_per_pair", "SQ_INSTS_VALU"), ("trans_per_pair", "SQ_INSTS_VALU_TRANS_F32"),
                          ("salu_per_pair", "SQ_INSTS_SALU"), ("lds_per_pair", "SQ_INSTS_LDS"),
                          ("vmem_per_pair", "SQ_INSTS_VMEM")):
            if key in c:
                rec[name] = c[key] * 64 / pairs
        if "SQ_WAVE_CYCLES" in c:
            for name, key in (("valu_active_share", "SQ_ACTIVE_INST_VALU"), ("any_active_share", "SQ_ACTIVE_INST_ANY"),
                              ("wait_inst_share", "SQ_WAIT_INST_ANY"), ("wait_any_share", "SQ_WAIT_ANY")):
                if key in c:
                    rec[name] = c[key] / c["SQ_WAVE_CYCLES"]
        if ns and "SQ_INSTS_VALU" in c:
            rec["valu_lane_T_per_s"] = c["SQ_INSTS_VALU"] * 64 / ns / 1e3
        if ns and "SQ_INSTS_VALU_TRANS_F32" in c:
            rec["trans_lane_T_per_s"] = c["SQ_INSTS_VALU_TRANS_F32"] * 64 / ns / 1e3
        launches[k] = rec
    tot = {}
    for name in ("valu_per_pair", "trans_per_pair", "salu_per_pair"):
        if all(name in v for v in launches.values()) and launches:
            tot[name] = sum(v[name] for v in launches.values()) / len(launches)
    rec = {"what": "SQ counters of the batched step (row-pass and column-pass persistent launches) of the "
                   "64-image ragged batch, S=10 K=3 box row_col, 2 waves per SIMD",
           "launches": launches, "step": tot, "algorithmic_valu_per_pair": PAIR_VALU,
           "source_sha256": source_sha()}
    with open(out_path or counters_path(), "w") as fo:
        json.dump(rec, fo, indent=1)
    print(json.dumps({k: round(v, 3) for k, v in tot.items()}))
    return rec


def counters_from_profiles():
    """Counter-measured instructions per pair of the batched step from the
    committed record, if it was taken on the current sources (else None)."""
    path = counters_path()
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != source_sha():
        return None
    out = {k: round(v, 3) for k, v in rec["step"].items()}
    for k, v in rec["launches"].items():
        tag = "rows" if k.rstrip(")").endswith("true>(snlm::KernelArgs") or ", true>" in k else "cols"
        out[tag] = {n: round(v[n], 3) for n in ("valu_per_pair", "trans_per_pair", "salu_per_pair",
                                                 "valu_active_share", "wait_inst_share") if n in v}
    return out


# ----------------------------------------------------------------- serving --
def serving(torch, snlm, n_req=2000, rate_frac=0.7, seed=4000, check=32, fifo=True):
    """2000 requests (sizes log-uniform 64..2048 per axis, sigma U[10,40],
    S in {5,10,15}, K in {2,3,4}, box/Gauss and both orders 50/50), inputs
    generated on the device before timing and submitted by the library's own
    request driver (snlm_submit_many).  Saturation throughput first (every
    request at t = 0), then Poisson arrivals at rate_frac of it; p50/p99 of
    the device-measured latency (the submit event on the caller's stream to
    the end of the job's round, both GPU timestamps) and of the host-observed
    one.  `check` requests are compared bitwise with plain launches of the same
    job.  Baseline: the same arrivals served FIFO by plain single-image
    launches, one at a time."""
    from paper_1407_2343_amd.synth import clean_image, serving_requests
    reqs = serving_requests(n_req, seed=seed, rate_per_s=1.0)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    pool = [torch.from_numpy(clean_image(2048, 2048, np.random.default_rng(seed + i))).to("cuda:0")
            .to(torch.float32) for i in range(4)]
    rng = np.random.default_rng(seed + 7)
    xs, outs = [], []
    for i, r in enumerate(reqs):
        base = pool[i % 4]
        y0 = int(rng.integers(0, 2048 - r["H"] + 1))
        x0 = int(rng.integers(0, 2048 - r["W"] + 1))
        noise = torch.randn((r["H"], r["W"]), generator=g, device="cuda:0")
        xs.append((base[y0:y0 + r["H"], x0:x0 + r["W"]] + r["sigma"] * noise).contiguous())
        outs.append(torch.empty((r["H"], r["W"]), dtype=torch.float32, device="cuda:0"))
    torch.cuda.synchronize()
    total_px = sum(r["H"] * r["W"] for r in reqs)
    arena = 1 << 30  # HBM budget of in-flight jobs: staged input, intermediate, output slot
    srv = snlm.Context(arena_bytes=arena)
    job_list = [srv.job_for(x, o, r["S"], r["K"], 10.0 * r["sigma"], r["kernel"], r["order"])
                for x, o, r in zip(xs, outs, reqs)]
    jobs = snlm.job_array(job_list)

    def run(arrivals, sub):
        t0 = time.perf_counter()
        tickets = srv.submit_many(sub, arrivals)
        t_sub = time.perf_counter() - t0
        host, dev, first, last = [], [], None, None
        pending = list(tickets)
        while pending:
            rest = []
            for t in pending:
                ts, ta, td = srv.job_times(t)
                if td > 0:
                    dms = srv.job_device_ms(t)
                    st = srv.poll(t)
                    if st != snlm.OK:
                        raise RuntimeError("served job failed: %d %s" % (st, srv.last_error()))
                    host.append((td - ts) / 1e3)
                    dev.append(dms)
                    first = ts if first is None else min(first, ts)
                    last = td if last is None else max(last, td)
                else:
                    rest.append(t)
            pending = rest
            if pending:
                time.sleep(0.0002)
        return np.array(host), np.array(dev), (last - first) / 1e6, t_sub

    run(None, snlm.job_array(job_list[:64]))  # warm every kernel class once
    r0, j0, us0 = srv.serving_stats()
    _, dev_sat, span_sat, sub_sat = run(None, jobs)
    r1, j1, us1 = srv.serving_stats()
    sat_rounds, sat_jobs, sat_host_us = r1 - r0, j1 - j0, us1 - us0
    sat_rate = n_req / span_sat
    rate = rate_frac * sat_rate
    arr_rng = np.random.default_rng(seed + 11)
    arrivals = np.cumsum(arr_rng.exponential(1.0 / rate, n_req))
    host, dev, span, _ = run(list(arrivals), jobs)
    torch.cuda.synchronize()
    # served results against plain launches of the same jobs, bitwise
    pick = np.random.default_rng(seed + 13).choice(n_req, size=min(check, n_req), replace=False) if check else []
    served = [outs[i].clone() for i in pick]
    srv.close()
    plain = snlm.Context(arena_bytes=arena)
    same = True
    for i, got in zip(pick, served):
        plain.denoise_job_sync(job_list[i])
        same = same and bool(torch.equal(outs[i], got))

    rec = {
        "requests": n_req, "pixels": int(total_px), "arena_bytes": arena,
        "admission": "staged input + FP32 intermediate + FP32 output slot per job within the arena",
        "saturation_req_per_s": round(sat_rate, 1),
        "saturation_mpx_per_s": round(total_px / span_sat / 1e6, 1),
        "saturation_submit_s": round(sub_sat, 4),
        "saturation_device_p50_ms": round(float(np.percentile(dev_sat, 50)), 3),
        "saturation_rounds": sat_rounds, "saturation_jobs_per_round": round(sat_jobs / max(sat_rounds, 1), 2),
        "saturation_scheduler_host_us_per_round": round(sat_host_us / max(sat_rounds, 1), 1),
        "rate_req_per_s": round(rate, 1),
        "p50_ms": round(float(np.percentile(dev, 50)), 3),
        "p99_ms": round(float(np.percentile(dev, 99)), 3),
        "latency_is": "device: submit event on the caller's stream to the end of the job's round",
        "host_p50_ms": round(float(np.percentile(host, 50)), 3),
        "host_p99_ms": round(float(np.percentile(host, 99)), 3),
        "mpx_per_s": round(total_px / span / 1e6, 1),
        "checked_requests": len(pick), "checked_bitwise_equal_to_plain": same,
    }
    if not fifo:
        plain.close()
        return rec
    # The same requests as one offline batched call (every class planned at
    # once, nothing arriving over time, no slot copies), for scale: default
    # waves per SIMD, then the batch autotuner's choice per class.
    off_outs = [torch.empty_like(o) for o in outs]
    off = snlm.Context(arena_bytes=sum(snlm.workspace_bytes(r["H"], r["W"]) for r in reqs) + (1 << 20))
    off_jobs = snlm.job_array([off.job_for(x, o, r["S"], r["K"], 10.0 * r["sigma"], r["kernel"], r["order"])
                               for x, o, r in zip(xs, off_outs, reqs)])
    for key, tune in (("offline_batch", False), ("offline_batch_autotuned", True)):
        if tune:
            off.autotune_batch(off_jobs)
        ms_off, _ = time_steps(torch, lambda: off.denoise_jobs(off_jobs), 5, 2)
        rec[key + "_ms"] = round(ms_off, 3)
        rec[key + "_mpx_per_s"] = round(total_px / ms_off / 1e3, 1)
    off.close()
    del off_outs
    # FIFO plain launches at the same arrival times
    for j in job_list[:64]:
        plain.denoise_job(j)
    plain.sync()
    t_start = time.perf_counter()
    plat = []
    for j, a in zip(job_list, arrivals):
        while time.perf_counter() - t_start < a:
            pass
        plain.denoise_job(j)
        plain.sync()
        plat.append((time.perf_counter() - t_start - a) * 1e3)
    plain_span = time.perf_counter() - t_start
    plain.close()
    plat = np.array(plat)
    rec.update({
        "plain_fifo_p50_ms": round(float(np.percentile(plat, 50)), 3),
        "plain_fifo_p99_ms": round(float(np.percentile(plat, 99)), 3),
        "plain_fifo_mpx_per_s": round(total_px / plain_span / 1e6, 1),
    })
    return rec


def serving_overlap(path):
    """From a rocprofv3 kernel-trace CSV of a --serve-only run: the served
    batched kernels (snlm_kernel launches and the staging copies) per queue,
    the share of their busy time during which kernels of two or more rounds
    run at once, and the most kernels running at once."""
    import csv
    ev = []
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        if "snlm_kernel" not in name and "snlm_copy_images" not in name:
            continue
        ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Queue_Id", "?"), name))
    if not ev:
        return {"dispatches": 0}
    pts = sorted([(s, 1) for s, _, _, _ in ev] + [(e, -1) for _, e, _, _ in ev])
    busy = multi = 0
    depth, last, peak = 0, pts[0][0], 0
    for t, d in pts:
        if depth >= 1:
            busy += t - last
        if depth >= 2:
            multi += t - last
        depth += d
        peak = max(peak, depth)
        last = t
    queues = {}
    for _, _, q, _ in ev:
        queues[q] = queues.get(q, 0) + 1
    return {"dispatches": len(ev), "queues": queues, "busy_us": round(busy / 1e3, 1),
            "overlap_share_of_busy": round(multi / busy, 4) if busy else 0.0, "max_concurrent": peak}


# --------------------------------------------------------------- precision --
def precision(torch, snlm, sizes=(2048, 4096), sigma=30.0):
    """n x n images, sigma 30, S=15, K=4, box, h = 10 sigma: Mpixel/s of
    {FP16, FP32 storage} x {block-restarted, plain, Kahan} running sums.  Their
    error against the FP64 oracle over every pixel is a GPU test of the same
    images (tests/test_gpu_systems.py, test_precision_variants_whole_image);
    here, each variant's distance from the FP32 Kahan result, for scale."""
    from paper_1407_2343_amd.synth import noisy_image
    out = {}
    for n in sizes:
        img = noisy_image(n, n, sigma, seed=3001 + n)
        ctx = snlm.Context(arena_bytes=snlm.workspace_bytes(n, n) + (1 << 20))
        ys, rec_n = {}, {}
        for dtype in ("f32", "f16"):
            x = torch.from_numpy(img.astype(np.float16 if dtype == "f16" else np.float32)).to("cuda:0")
            for sm in ("kahan", "block", "plain"):
                y_t = torch.empty((n, n), device="cuda:0")
                j = ctx.job_for(x, y_t, 15, 4, 10 * sigma, "box", "row_col", sm)
                ms, _ = time_steps(torch, lambda: ctx.denoise_job(j), 3, 1)
                name = "%s_%s" % (dtype, sm)
                ys[name] = y_t.cpu().numpy().astype(np.float64)
                e = ys[name] - ys["f32_kahan"]
                rec_n[name] = {"mpx_per_s": round(n * n / ms / 1e3, 1),
                               "max_abs_vs_f32_kahan": float(np.max(np.abs(e))),
                               "rms_vs_f32_kahan": float(np.sqrt(np.mean(e * e)))}
        ctx.close()
        out["%dx%d" % (n, n)] = rec_n
    return {"image": "sigma=%g S=15 K=4 box row_col h=10 sigma" % sigma,
            "error_vs_fp64_oracle": "every pixel, tests/test_gpu_systems.py::test_precision_variants_whole_image",
            "variants": out}


# ----------------------------------------------------------- SURE combination --
def sure_combination(torch, snlm, n=2048, sigma=30.0):
    """SNLM with the SURE-optimal combination of the two orders (Alg. 4) on an
    n x n image with a known clean image (eq. noise), S=10, K=3, box, h = 10
    sigma: Mpixel/s of the whole call (four divergence-carrying passes, the
    FP64 image sums, the 2x2 solve and the combination), theta, the MSE of each
    order and of the combination against the clean image, and the SURE
    estimate.  Parity against the FP64 oracle is tests/test_gpu_sure.py."""
    from paper_1407_2343_amd.synth import clean_image
    rng = np.random.default_rng(6001)
    f0 = clean_image(n, n, rng)
    f = (f0 + sigma * rng.standard_normal(f0.shape)).astype(np.float32)
    x = torch.from_numpy(f).to("cuda:0")
    ctx = snlm.Context(arena_bytes=snlm.sure_workspace_bytes(n, n) + (1 << 20))
    out = torch.empty_like(x)
    res = {}

    def call():
        res["r"] = ctx.denoise_sure(x, S, K, 10 * sigma, sigma, "box", out=out)

    ms, _ = time_steps(torch, call, 5, 2)
    _, theta, stats = res["r"]
    planes = ctx.sure_planes(n, n)
    f_cr = planes["f_cr"].cpu().numpy().astype(np.float64)
    d_rc = planes["d_rc"].cpu().numpy().astype(np.float64)
    d_cr = planes["d_cr"].cpu().numpy().astype(np.float64)
    y = out.cpu().numpy().astype(np.float64)
    f_rc = (y - theta[1] * f_cr) / theta[0] if theta[0] != 0 else None
    f0d, fd = f0.astype(np.float64), f.astype(np.float64)
    mse = float(np.mean((y - f0d) ** 2))
    phi = float(np.mean((y - fd) ** 2) - sigma ** 2
                + 2 * sigma ** 2 / fd.size * (theta[0] * d_rc.sum() + theta[1] * d_cr.sum()))
    rec = {"image": "%dx%d sigma=%g S=%d K=%d box h=10 sigma" % (n, n, sigma, S, K),
           "mpx_per_s": round(n * n / ms / 1e3, 1), "ms": round(ms, 3),
           "theta": [round(t, 6) for t in theta], "mse_combined": round(mse, 4),
           "sure": round(phi, 4)}
    if f_rc is not None:
        rec["mse_row_col"] = round(float(np.mean((f_rc - f0d) ** 2)), 4)
    rec["mse_col_row"] = round(float(np.mean((f_cr - f0d) ** 2)), 4)
    # SNLM[f]: the combination followed by the bilateral filter (Sec. 3.2)
    ctx.ensure_arena(snlm.full_workspace_bytes(n, n) + (1 << 20))
    full = torch.empty_like(x)

    def call_full():
        res["f"] = ctx.denoise_full(x, S, K, 10 * sigma, sigma, "box", out=full)

    ms_full, _ = time_steps(torch, call_full, 5, 2)
    ss, sr = snlm.bilateral_params(sigma)
    bf_out = torch.empty_like(x)
    ms_bf, _ = time_steps(torch, lambda: ctx.bilateral(out, ss, sr, out=bf_out), 10, 2)
    yf = full.cpu().numpy().astype(np.float64)
    mse_full = float(np.mean((yf - f0d) ** 2))
    rec["full_snlm"] = {"mpx_per_s": round(n * n / ms_full / 1e3, 1), "ms": round(ms_full, 3),
                        "bilateral_ms": round(ms_bf, 3), "sigma_s": round(ss, 4), "sigma_r": round(sr, 3),
                        "mse": round(mse_full, 4),
                        "psnr_db": round(10 * np.log10(255.0 ** 2 / mse_full), 3),
                        "psnr_db_before_bilateral": round(10 * np.log10(255.0 ** 2 / mse), 3)}
    ctx.close()
    return rec


# ------------------------------------------------------------------ volumes --
def volume(torch, snlm, n=256, sigma=20.0):
    """An n x n x n FP32 volume (smooth pattern plus noise), S=10, K=3, box,
    h = 10 sigma: the 1D pass along x, y and z in turn (three launches),
    Mvoxel/s of the whole call, events on the stream it runs on.  Parity
    against the FP64 oracle is tests/test_gpu_volume.py."""
    from paper_1407_2343_amd.synth import noisy_volume
    x = torch.from_numpy(noisy_volume(n, n, n, sigma, seed=9001)).to("cuda:0")
    out = torch.empty_like(x)
    ctx = snlm.Context(arena_bytes=snlm.workspace3d_bytes(n, n, n) + (1 << 20))
    rec = {"volume": "%dx%dx%d sigma=%g S=%d K=%d box h=10 sigma" % (n, n, n, sigma, S, K)}
    for axes in ("xyz", "zyx"):
        ms, _ = time_steps(torch, lambda: ctx.denoise3d(x, S, K, 10 * sigma, "box", axes, out=out), 10, 2)
        rec[axes] = {"mvoxel_per_s": round(n ** 3 / ms / 1e3, 1), "ms": round(ms, 3)}
    ctx.close()
    return rec


# ------------------------------------------------------- recursive Gaussian --
def recursive_gaussian(torch, snlm, n=2048, sigma=30.0):
    """The Gaussian patch kernel by the recursive filter (kernel "gauss_iir")
    on an n x n image, S=10, h = 10 sigma sqrt(sqrt(2 pi) beta / 7): Mpixel/s
    at beta = 2 and at beta = 8 (a width the exact FIR, K <= 8, cannot reach),
    beside the exact FIR at beta = 2 with K = 4 and K = 6, and the recursive
    kernel's distance from the exact FIR with taps out to 3 beta at beta = 1,
    2, 8/3 (its approximation error, not a parity figure), beside the box
    kernel's.  Parity against the FP64 oracle is tests/test_gpu_iir.py."""
    from paper_1407_2343_amd.synth import noisy_image
    img = noisy_image(n, n, sigma, seed=7001)
    x = torch.from_numpy(img).to("cuda:0")
    ctx = snlm.Context(arena_bytes=snlm.workspace_bytes(n, n) + (1 << 20))

    def h_for(beta):
        return 10.0 * sigma * float(np.sqrt(np.sqrt(2 * np.pi) * beta / 7.0))

    rec = {"image": "%dx%d sigma=%g S=%d row_col" % (n, n, sigma, S)}
    outs = {}
    for name, kern, KK, beta in (("iir_beta2", "gauss_iir", 0, 2.0), ("iir_beta8", "gauss_iir", 0, 8.0),
                                 ("fir_beta2_K4", "gauss", 4, 2.0), ("fir_beta2_K6", "gauss", 6, 2.0)):
        y = torch.empty_like(x)
        j = ctx.job_for(x, y, S, KK, h_for(beta), kern, "row_col", "block", beta)
        ms, _ = time_steps(torch, lambda: ctx.denoise_job(j), 10, 2)
        outs[name] = y.cpu().numpy().astype(np.float64)
        rec[name] = {"mpx_per_s": round(n * n / ms / 1e3, 1), "ms": round(ms, 3)}
    # HBM roofline of the recursive path at beta = 2 (both passes): per pass,
    # the forward recursion reads x and writes its FP64 state at every block
    # start (3 S ((n + L - 1) / 16 + 2) words per line), the NLM kernel reads
    # the states back (once each at least: segment warm-ups re-read a few
    # blocks), reads x and writes y; the row pass adds a transposed copy of
    # its input (read + write).  The method's own minimum is x in and y out.
    L = int(np.ceil(6 * 2.0)) + S + 3
    nblk = (n + L - 1) // 16 + 2
    per_pass = n * (4 * 3 * n + 2 * 8 * 3 * S * nblk)
    staged = 2 * per_pass + 8 * n * n
    method = 2 * 8 * n * n  # x in and y out, per pass
    ms2 = rec["iir_beta2"]["ms"]
    gbs = method / (ms2 * 1e-3) / 1e9
    rec["iir_beta2"]["roofline"] = {
        "bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
        "bytes": int(method), "bytes_are": "the method's own: x in and y out (4 + 4 B per pixel) per pass, "
        "over the whole-path time (five launches)",
        "staged_bytes": int(staged), "staged_gb_per_s": round(staged / (ms2 * 1e-3) / 1e9, 1),
        "staged_are": "forward states written and read once, x read twice, y written once per pass, plus "
        "the row pass's transposed input"}
    rec["iir_beta2"]["max_abs_vs_exact_fir_K6"] = float(np.max(np.abs(outs["iir_beta2"] - outs["fir_beta2_K6"])))
    rec["iir_beta2"]["rms_vs_exact_fir_K6"] = float(np.sqrt(np.mean((outs["iir_beta2"] - outs["fir_beta2_K6"]) ** 2)))
    # the approximation error against the exact FIR with taps out to 3 beta,
    # at the widths the FIR reaches (K <= 8), and the box kernel's distance
    # from the same FIR for scale
    approx = {}
    for beta in (1.0, 2.0, 8.0 / 3.0):
        KK = min(8, int(np.ceil(3 * beta)))
        ys = {}
        for kern, kk, hh in (("gauss_iir", 0, h_for(beta)), ("gauss", KK, h_for(beta)),
                             ("box", KK, h_for(beta) * float(np.sqrt((2 * KK + 1) / (np.sqrt(2 * np.pi) * beta))))):
            y = torch.empty_like(x)
            ctx.denoise_job(ctx.job_for(x, y, S, kk, hh, kern, "row_col", "block", beta))
            torch.cuda.synchronize()
            ys[kern] = y.cpu().numpy().astype(np.float64)
        d_iir, d_box = ys["gauss_iir"] - ys["gauss"], ys["box"] - ys["gauss"]
        approx["beta_%.3g_K%d" % (beta, KK)] = {
            "iir_max_abs": round(float(np.max(np.abs(d_iir))), 4), "iir_rms": round(float(np.sqrt(np.mean(d_iir ** 2))), 4),
            "box_max_abs": round(float(np.max(np.abs(d_box))), 4), "box_rms": round(float(np.sqrt(np.mean(d_box ** 2))), 4)}
    rec["error_vs_exact_fir"] = approx
    ctx.close()
    return rec


def plain_512(torch, ctx):
    """One 512 x 512 FP32 image (sigma 20, h = 10 sigma, S=10, K=3), box and
    Gaussian, both orders: device time of each of 60 single launches (both
    passes), events on the stream they run on."""
    from paper_1407_2343_amd.synth import noisy_image
    x512 = torch.from_numpy(noisy_image(512, 512, 20.0, seed=1001)).to("cuda:0")
    o512 = torch.empty_like(x512)
    res = {}
    for kernel in ("box", "gauss"):
        for order in ("row_col", "col_row"):
            j512 = ctx.job_for(x512, o512, S, K, 200.0, kernel, order)
            for _ in range(3):
                ctx.denoise_job(j512)
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(60)]
            for e0, e1 in evs:
                e0.record()
                ctx.denoise_job(j512)
                e1.record()
            torch.cuda.synchronize()
            t = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
            p50, p99 = float(np.percentile(t, 50)), float(np.percentile(t, 99))
            res["%s_%s" % (kernel, order)] = {
                "mpx_per_s_p50": round(512 * 512 / (p50 * 1e-3) / 1e6, 1),
                "ms_p50": round(p50, 4), "ms_p99": round(p99, 4), "launches": len(t)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sure", action="store_true")
    ap.add_argument("--no-iir", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--batch-waves", type=int, default=0, metavar="N",
                    help="use N persistent waves per SIMD for the batch instead of autotuning (counter runs)")
    ap.add_argument("--issue-rate", action="store_true",
                    help="print the issue-rate probe of the pair body (snlm_issue_rate) and exit")
    ap.add_argument("--serve-only", type=int, default=0, metavar="N",
                    help="run only the serving section with N requests and print it (kernel traces)")
    ap.add_argument("--serving-overlap", metavar="KERNEL_TRACE_CSV",
                    help="print how the served kernels of a rocprofv3 kernel trace overlap in time (no GPU)")
    ap.add_argument("--iir-only", action="store_true",
                    help="run only the recursive-Gaussian section and print it")
    ap.add_argument("--volume-only", action="store_true",
                    help="run only the volume section and print it (kernel traces)")
    ap.add_argument("--sure-only", action="store_true",
                    help="run only the SURE-combination and SNLM[f] section and print it (kernel traces)")
    ap.add_argument("--plain-only", action="store_true",
                    help="run only the plain 512 x 512 single-image launches and print them (kernel traces)")
    ap.add_argument("--profile-batch", action="store_true",
                    help="only the batched steps (for rocprofv3 kernel traces and counters)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only a device-to-device copy of MIB MiB (counter calibration)")
    ap.add_argument("--write-counters", nargs="+", metavar="CSV",
                    help="write profiles/counters_batch.json from rocprofv3 --pmc CSVs (no GPU)")
    ap.add_argument("--write-traffic", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                         "COPY_WRITE_CSV", "COPY_MIB"),
                    help="write profiles/traffic_batch.json from rocprofv3 counter CSVs (no GPU)")
    a = ap.parse_args()
    if a.serving_overlap:
        print(json.dumps(serving_overlap(a.serving_overlap)))
        return
    if a.write_counters:
        write_counters(a.write_counters)
        return
    if a.write_traffic:
        write_traffic(*a.write_traffic[:4], int(a.write_traffic[4]))
        return
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(independent images would shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1407_2343_amd as snlm
    from paper_1407_2343_amd.synth import batch_workload, noisy_image

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if a.calibrate_copy:
        n = a.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}), flush=True)
        return
    if a.iir_only:
        print(json.dumps({"recursive_gaussian": recursive_gaussian(torch, snlm)}), flush=True)
        return
    if a.volume_only:
        print(json.dumps({"volume": volume(torch, snlm)}), flush=True)
        return
    if a.sure_only:
        print(json.dumps({"sure_combination": sure_combination(torch, snlm)}), flush=True)
        return
    if a.plain_only:
        ctx = snlm.Context(arena_bytes=64 << 20)
        print(json.dumps({"plain_512_mpx": plain_512(torch, ctx)}), flush=True)
        ctx.close()
        return
    if a.issue_rate:
        rows = {}
        for mode, name in ((0, "fp32_body_8_instr"), (1, "pair_body_7_fp32_plus_exp"), (2, "exp_alone")):
            for w in (1, 2, 4):
                clk, ghz = snlm.issue_rate(mode, w)
                rows["%s_w%d" % (name, w)] = {"clk_per_pair_per_simd": round(clk, 2), "clock_ghz": round(ghz, 3)}
        print(json.dumps({"issue_rate": rows}), flush=True)
        return
    if a.serve_only:
        # the served phases only (no bitwise check, no FIFO baseline): for kernel traces
        print(json.dumps({"serving": serving(torch, snlm, n_req=a.serve_only, check=0, fifo=False)}), flush=True)
        return
    log("generating the batch workload")
    items = batch_workload(64, 128, 1024, seed=2000)
    xs = [torch.from_numpy(img).to("cuda:0") for img, _ in items]
    hs = [10.0 * sig for _, sig in items]
    total_px = sum(x.numel() for x in xs)
    outs = [torch.empty_like(x) for x in xs]
    ctx = snlm.Context(arena_bytes=sum(snlm.workspace_bytes(*x.shape) for x in xs) + (1 << 20))
    jobs = snlm.job_array([ctx.job_for(x, o, S, K, h, "box", "row_col")
                           for x, o, h in zip(xs, outs, hs)])

    def step():
        ctx.denoise_jobs(jobs)

    if a.batch_waves:
        # a fixed choice, loaded as the autotuner's record for this kernel class
        import tempfile
        path = os.path.join(tempfile.gettempdir(), "snlm_batch_waves_%d.json" % os.getpid())
        with open(path, "w") as f:
            json.dump({"arch": "gfx950", "entries": [], "batch": [
                {"bS": S, "K": K, "variant": 0, "order": 0, "waves_per_simd": a.batch_waves}]}, f)
        ctx.load_tuning(path)
        os.remove(path)
        seg = a.batch_waves
    else:
        log("autotuning the batched segment length")
        seg = ctx.autotune_batch(jobs)
    log("batched: warmup + timed")
    ms_step, wall_ms = time_steps(torch, step, a.steps, a.warmup)
    if a.profile_batch:
        print(json.dumps({"batched_ms_per_step": round(ms_step, 4), "waves_per_simd": seg}), flush=True)
        ctx.close()
        return
    # device time of the batched launches on the stream they run on
    ctx.timing_start()
    for _ in range(a.steps):
        step()
    ctx.sync()
    bms, bn, _, _ = ctx.timing_stop()
    kernel_ms = bms / max(bn, 1)
    batched_mpx = total_px / (ms_step * 1e-3) / 1e6

    log("plain launches of the batch images")
    plain_jobs = list(jobs)

    def plain_step():
        for j in plain_jobs:
            ctx.denoise_job(j)

    ms_plain, _ = time_steps(torch, plain_step, max(3, a.steps // 4), 1)
    plain_batch_mpx = total_px / (ms_plain * 1e-3) / 1e6

    plain512 = plain_512(torch, ctx)

    pairs = total_px * 2 * S
    alg_ops = pairs * PAIR_VALU
    achieved = alg_ops / (kernel_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": traffic_from_profiles(),
            "counters": counters_from_profiles(),
            "kernel": "snlm_kernel<10,3,box> row + column persistent launches (one graph replay)",
            "kernel_ms": round(kernel_ms, 4),
            "alg_valu_per_pair": PAIR_VALU, "pairs_per_launch": int(pairs),
            "exp_T_per_s": round(pairs / (kernel_ms * 1e-3) / 1e12, 3),
            "algorithmic_hbm_bytes": int(total_px * 16),
            "hbm_gb_per_s_algorithmic": round(total_px * 16 / (kernel_ms * 1e-3) / 1e9, 1)}

    result = {
        "metric": "Mpixel/s separable NLM S=10 K=3 (batched vs plain); p50/p99 served latency",
        "value": round(batched_mpx, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded shapes + gradient + texture + Gaussian noise)",
        "config": {"workload": "batched: 64 FP32 images, H,W log-uniform [128,1024], "
                               "sigma in {10,20,30,40}, h=10 sigma, S=10, K=3, box, row_col",
                   "pixels_per_step": int(total_px), "images": len(xs),
                   "autotuned_waves_per_simd": seg},
        "plain_same_images_mpx": round(plain_batch_mpx, 1),
        "plain_512_mpx": plain512,
        "wall_ms_per_step": round(wall_ms, 4),
        "roofline": roof,
    }
    ctx.close()
    if not a.no_serve:
        log("serving")
        result["serving"] = serving(torch, snlm)
    if not a.no_precision:
        log("precision")
        result["precision"] = precision(torch, snlm)
    if not a.no_sure:
        log("sure combination")
        result["sure_combination"] = sure_combination(torch, snlm)
    if not a.no_iir:
        log("recursive gaussian")
        result["recursive_gaussian"] = recursive_gaussian(torch, snlm)
    if not a.no_volume:
        log("volume")
        result["volume"] = volume(torch, snlm)
    if not a.no_cpu:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(items)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
