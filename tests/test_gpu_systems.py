"""Batched launches, serving and precision variants on the GPU.

* batch == plain: each image of a ragged batch, run in the persistent batched
  launches (split and fused modes), is bitwise equal to its plain launch, and
  within 1e-3 of the FP64 oracle.
* serving: every served job is bitwise equal to the same job run alone, the
  scheduler overlaps launches (a job admitted while an earlier one is still in
  flight), and misuse is reported (ENOMEM, ENOTICKET).
* precision: FP16/FP32 storage x block/plain/Kahan running sums on the
  2048 x 2048 and 4096 x 4096 images, every pixel against the oracle.
* the benchmark's batch as timed: all 64 images bitwise equal to their plain
  launches and within 1e-3 of the oracle at every pixel; the same images as
  FP16 with the Gaussian kernel in col_row order, likewise.
"""
import math
import os
import time

import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, max_abs, say
from paper_1407_2343_amd.synth import noisy_image

pytestmark = pytest.mark.gpu


def _ctx(arena, mode=None):
    import paper_1407_2343_amd as snlm
    old = os.environ.get("SNLM_BATCH_MODE")
    if mode is not None:
        os.environ["SNLM_BATCH_MODE"] = mode
    try:
        return snlm.Context(arena_bytes=arena)
    finally:
        if mode is not None:
            if old is None:
                os.environ.pop("SNLM_BATCH_MODE", None)
            else:
                os.environ["SNLM_BATCH_MODE"] = old


def _ragged(n, seed, lo=40, hi=300):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        H = int(rng.integers(lo, hi))
        W = int(rng.integers(lo, hi))
        sig = float(rng.choice([10.0, 20.0, 30.0, 40.0]))
        out.append((noisy_image(H, W, sig, seed * 100 + i), sig))
    return out


@pytest.mark.parametrize("mode", ["split", "fused"])
def test_batch_equals_plain(mode):
    import torch
    import paper_1407_2343_amd as snlm
    items = _ragged(12, 5)
    ctx = _ctx(64 << 20, mode)
    xs = [torch.from_numpy(im).to("cuda:0") for im, _ in items]
    outs = ctx.denoise_batch(xs, 10, 3, [10 * s for _, s in items], "box", "row_col", sync=True)
    # same batch again: replays the cached graph and tables
    outs2 = ctx.denoise_batch(xs, 10, 3, [10 * s for _, s in items], "box", "row_col", sync=True)
    for i, ((im, sig), x, o, o2) in enumerate(zip(items, xs, outs, outs2)):
        say("batch", mode, i, im.shape)
        alone = ctx.denoise(x, 10, 3, 10 * sig, "box", "row_col", sync=True)
        assert torch.equal(o, alone), i
        assert torch.equal(o2, alone), i
        if i < 4:
            ref = oracle.snlm(im.astype(np.float64), 10, 3, 10 * sig, "box", "row_col")
            assert max_abs(o.cpu().numpy(), ref) <= TOL
    ctx.close()


@pytest.mark.parametrize("order", ["row_col", "col_row"])
def test_batch_short_last_groups(order):
    """Images whose last line group holds few lines (H or W = 64 q + r with
    r in 1..33; the lanes past r repeat the last line and store its values
    again).  Every output is bitwise its plain launch (box and Gaussian, FP32
    and FP16) and within 1e-3 of the FP64 oracle."""
    import torch
    import paper_1407_2343_amd as snlm
    shapes = [(65, 128), (66, 1000), (95, 129), (96, 255), (97, 300), (128 + 31, 190), (130, 65), (300, 129),
              (1000, 129), (1, 400)]
    ctx = _ctx(64 << 20)
    for kern, dt in (("box", "f32"), ("gauss", "f16")):
        jobs, keep = [], []
        for i, (H, W) in enumerate(shapes):
            img = noisy_image(H, W, 20.0, seed=800 + i)
            x = torch.from_numpy(img.astype(np.float16 if dt == "f16" else np.float32)).to("cuda:0")
            o = torch.full((H, W), -5.0, device="cuda:0")
            jobs.append(ctx.job_for(x, o, 10, 3, 200.0, kern, order))
            keep.append((x, o))
        ctx.denoise_jobs(jobs, sync=True)
        for i, ((x, o), (H, W)) in enumerate(zip(keep, shapes)):
            say("short last group", kern, dt, order, (H, W))
            alone = ctx.denoise(x, 10, 3, 200.0, kern, order, sync=True)
            assert torch.equal(o, alone), (H, W)
            if i % 3 == 0:
                ref = oracle.snlm(x.cpu().numpy().astype(np.float64), 10, 3, 200.0, kern, order)
                assert max_abs(o.cpu().numpy(), ref) <= TOL, (H, W)
    ctx.close()


def test_batch_mixed_classes():
    """Several (S, K, kernel, order) classes in one batch call."""
    import torch
    import paper_1407_2343_amd as snlm
    items = _ragged(8, 6, 30, 200)
    ctx = _ctx(64 << 20)
    jobs, outs, xs = [], [], []
    params = [(5, 2, "box", "row_col"), (10, 3, "gauss", "col_row"), (15, 4, "box", "col_row"),
              (10, 3, "box", "row_col")]
    for i, (im, sig) in enumerate(items):
        x = torch.from_numpy(im).to("cuda:0")
        o = torch.empty_like(x)
        S, K, kern, order = params[i % len(params)]
        jobs.append(ctx.job_for(x, o, S, K, 10 * sig, kern, order))
        xs.append((x, S, K, sig, kern, order))
        outs.append(o)
    ctx.ensure_arena(sum(snlm.workspace_bytes(*x.shape) for x, *_ in xs))
    ctx.denoise_jobs(jobs, sync=True)
    for (x, S, K, sig, kern, order), o in zip(xs, outs):
        alone = ctx.denoise(x, S, K, 10 * sig, kern, order, sync=True)
        assert torch.equal(o, alone)
    ctx.close()


@pytest.mark.parametrize("waves", [1, 2, 3, 4])
def test_batch_fixed_waves_equals_plain(waves, tmp_path):
    """Batched launches at a fixed number of persistent waves per SIMD, loaded
    as the autotuner's record of each kernel class (box row_col, box col_row,
    Gaussian row_col; S=10, K=3).  The planner cuts the line groups at
    positions that depend on the worker count and, at two waves per SIMD, on
    the 2 : 1 split of each SIMD's work between its first and second
    workgroup; every output must still be bitwise its plain launch."""
    import json
    import torch
    import paper_1407_2343_amd as snlm
    classes = [("box", "row_col", 0, 0), ("box", "col_row", 0, 1), ("gauss", "row_col", 2, 0)]
    path = str(tmp_path / "waves.json")
    with open(path, "w") as f:
        json.dump({"arch": "gfx950", "entries": [], "batch": [
            {"bS": 10, "K": 3, "variant": var, "order": order, "waves_per_simd": waves}
            for _, _, var, order in classes]}, f)
    items = _ragged(18, 70 + waves, 64, 900)
    xs = [torch.from_numpy(im).to("cuda:0") for im, _ in items]
    outs = [torch.full_like(x, -5.0) for x in xs]
    # the arena first: a context created for a larger one drops loaded tuning
    ctx = _ctx(sum(snlm.workspace_bytes(*x.shape) for x in xs) + (1 << 20))
    ctx.load_tuning(path)
    cls = [classes[i % len(classes)] for i in range(len(items))]
    jobs = snlm.job_array([ctx.job_for(x, o, 10, 3, 10 * sig, kern, order)
                           for x, o, (_, sig), (kern, order, _, _) in zip(xs, outs, items, cls)])
    ctx.denoise_jobs(jobs, sync=True)
    for i, ((im, sig), x, o, (kern, order, _, _)) in enumerate(zip(items, xs, outs, cls)):
        say("fixed waves", waves, i, kern, order, im.shape)
        alone = ctx.denoise(x, 10, 3, 10 * sig, kern, order, sync=True)
        assert torch.equal(o, alone), i
        if i < len(classes):
            ref = oracle.snlm(im.astype(np.float64), 10, 3, 10 * sig, kern, order)
            assert max_abs(o.cpu().numpy(), ref) <= TOL, i
    ctx.close()


@pytest.mark.parametrize("mode", ["split", "fused"])
def test_batch_degenerate_shapes(mode):
    """Degenerate images in one batched launch beside ordinary ones: 1 x 1,
    single rows and columns, lines shorter than S + K (the reflection wraps
    several periods), widths that leave a one-sample last chunk and a
    one-line last group, and an FP16 image with a row pitch.  Each equals its
    plain launch bitwise and the FP64 oracle within 1e-3."""
    import torch
    import paper_1407_2343_amd as snlm
    shapes = [(1, 1), (1, 300), (257, 1), (3, 2), (7, 13), (65, 17), (17, 65), (129, 64), (64, 129), (200, 201)]
    ctx = _ctx(64 << 20, mode)
    jobs, keep = [], []
    for i, (H, W) in enumerate(shapes):
        img = noisy_image(H, W, 20.0, seed=700 + i, texture=False)
        if i == len(shapes) - 1:  # FP16 storage, pitched
            big = torch.from_numpy(np.pad(img, ((0, 0), (0, 7))).astype(np.float16)).to("cuda:0")
            x = big[:, :W]
        else:
            x = torch.from_numpy(img).to("cuda:0")
        o = torch.full((H, W), -5.0, device="cuda:0")
        jobs.append(ctx.job_for(x, o, 10, 3, 200.0, "box", "row_col"))
        keep.append((x, o))
    ctx.denoise_jobs(jobs, sync=True)
    for (x, o), (H, W) in zip(keep, shapes):
        say("degenerate", mode, (H, W))
        alone = ctx.denoise(x, 10, 3, 200.0, "box", "row_col", sync=True)
        assert torch.equal(o, alone), (H, W)
        ref = oracle.snlm(x.cpu().numpy().astype(np.float64), 10, 3, 200.0, "box", "row_col")
        assert max_abs(o.cpu().numpy(), ref) <= TOL, (H, W)
    ctx.close()


def test_serving_alone_equals_mix():
    import torch
    import paper_1407_2343_amd as snlm
    rng = np.random.default_rng(11)
    # sizes log-uniform over the serving workload's range, 64..2048 per axis;
    # the arena holds a few jobs at a time, so later jobs queue for space
    arena = 96 << 20
    srv = _ctx(arena)
    solo = _ctx(64 << 20)
    reqs = []
    for i in range(48):
        H = int(np.exp(rng.uniform(np.log(64), np.log(2048))))
        W = int(np.exp(rng.uniform(np.log(64), np.log(2048))))
        sig = float(rng.uniform(10, 40))
        S = int(rng.choice([5, 10, 15]))
        K = int(rng.choice([2, 3, 4]))
        kern = "gauss" if rng.random() < 0.5 else "box"
        order = "col_row" if rng.random() < 0.5 else "row_col"
        x = torch.from_numpy(noisy_image(H, W, sig, 500 + i)).to("cuda:0")
        o = torch.full_like(x, -1.0)
        reqs.append((x, o, S, K, 10 * sig, kern, order))
    torch.cuda.synchronize()
    tickets = []
    jobs = [srv.job_for(x, o, S, K, h, kern, order) for (x, o, S, K, h, kern, order) in reqs]
    for j in jobs:  # a burst: later jobs arrive while earlier ones run
        tickets.append(srv.submit(j))
    times = {}
    pending = set(tickets)
    t0 = time.time()
    while pending and time.time() - t0 < 60:
        for t in list(pending):
            ts = srv.job_times(t)
            if ts[2] > 0:
                times[t] = ts
                st = srv.poll(t)
                assert st == snlm.OK, (t, st, srv.last_error())
                pending.discard(t)
        time.sleep(0.001)
    assert not pending, "served jobs did not finish"
    assert srv.poll(tickets[0]) == snlm.ENOTICKET
    # results: bitwise equal to the same job run alone
    for i, (x, o, S, K, h, kern, order) in enumerate(reqs):
        alone = solo.denoise(x, S, K, h, kern, order, sync=True)
        assert torch.equal(o, alone), i
    # parity of a few served results (the smallest ones: the oracle is slow)
    for (x, o, S, K, h, kern, order) in sorted(reqs, key=lambda r: r[0].numel())[:3]:
        ref = oracle.snlm(x.cpu().numpy().astype(np.float64), S, K, h, kern, order)
        assert max_abs(o.cpu().numpy(), ref) <= TOL
    # overlap: some job was admitted while an earlier-admitted one was still in flight
    spans = sorted(times.values(), key=lambda v: v[1])
    overlapped = any(spans[k][1] < spans[j][2] and spans[k][1] > spans[j][1]
                     for j in range(len(spans)) for k in range(j + 1, len(spans)))
    queued = sum(1 for v in spans if v[1] > v[0] + 50.0)
    say("served", len(spans), "overlapped", overlapped, "queued", queued)
    assert overlapped
    assert queued > 0
    srv.close()
    solo.close()


def test_serving_errors():
    import torch
    import paper_1407_2343_amd as snlm
    srv = _ctx(1 << 20)
    x = torch.zeros((300, 300), device="cuda:0")
    o = torch.empty_like(x)
    with pytest.raises(snlm.SnlmError) as e:
        srv.submit(srv.job_for(x, o, 10, 3, 100.0))  # in + mid + out: 1.1 MB > 1 MiB arena
    assert e.value.status == snlm.ENOMEM
    assert srv.poll(12345) == snlm.ENOTICKET
    small = torch.zeros((50, 60), device="cuda:0")
    so = torch.empty_like(small)
    t = srv.submit(srv.job_for(small, so, 5, 2, 100.0))
    srv.close()  # drains in-flight work
    assert float(so.abs().max()) == 0.0


_ORACLE_CACHE = {}


def _precision_case(n, dtype):
    """The precision workload's n x n image (sigma 30, the benchmark's seed) as
    stored on the GPU, and the FP64 oracle (S=15, K=4, box, h = 300, row_col)
    of exactly those values, over the whole image (computed once per case)."""
    import torch
    key = (n, dtype)
    if key not in _ORACLE_CACHE:
        img = noisy_image(n, n, 30.0, seed=3001 + n)
        x = torch.from_numpy(img.astype(np.float16 if dtype == "f16" else np.float32)).to("cuda:0")
        xr = x.cpu().numpy().astype(np.float64)
        t0 = time.time()
        ref = oracle.snlm(xr, 15, 4, 300.0, "box", "row_col")
        say("oracle %dx%d %s in %.1f s" % (n, n, dtype, time.time() - t0))
        for k in [k for k in _ORACLE_CACHE if k[0] != n]:
            del _ORACLE_CACHE[k]  # keep the references of one size at a time
        _ORACLE_CACHE[key] = (x, ref)
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("sum", ["block", "plain", "kahan"])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("n", [2048, 4096])
def test_precision_variants_whole_image(n, dtype, sum):
    """The precision workload at both of its sizes (sigma 30, S=15, K=4, box):
    FP16 / FP32 storage x block-restarted / plain / Kahan running sums, every
    output pixel against the FP64 oracle run on exactly the values the GPU
    read (max-abs <= 1e-3), with the RMS error reported; for FP16 storage
    also the distance from the oracle of the FP32 input before rounding (the
    storage format's own error, reported, not bounded by the tolerance)."""
    import torch
    import paper_1407_2343_amd as snlm
    x, ref = _precision_case(n, dtype)
    ctx = _ctx(snlm.workspace_bytes(n, n) + (1 << 20))
    y = ctx.denoise(x, 15, 4, 300.0, "box", "row_col", sum=sum, sync=True).cpu().numpy().astype(np.float64)
    e = y - ref
    worst, rms = float(np.max(np.abs(e))), float(np.sqrt(np.mean(e * e)))
    line = "precision %dx%d %s %s: max-abs %.3g rms %.3g vs the oracle of the stored values" % (
        n, n, dtype, sum, worst, rms)
    if dtype == "f16":
        _, ref32 = _precision_case(n, "f32")
        e2 = y - ref32
        line += "; vs the FP32 input's oracle max-abs %.3g rms %.3g" % (
            float(np.max(np.abs(e2))), float(np.sqrt(np.mean(e2 * e2))))
    say(line)
    assert worst <= TOL
    ctx.close()


def test_bench_batch_workload_whole():
    """The benchmark's batch exactly as bench.py times it: 64 FP32 images, H
    and W log-uniform in [128, 1024] (seed 2000), h = 10 sigma, S=10, K=3, box,
    row_col, one job array, autotuned persistent waves, replayed launches.
    Every one of the 64 outputs is bitwise equal to its plain launch and within
    1e-3 of the FP64 oracle at every pixel."""
    import torch
    import paper_1407_2343_amd as snlm
    from paper_1407_2343_amd.synth import batch_workload
    items = batch_workload(64, 128, 1024, seed=2000)
    xs = [torch.from_numpy(img).to("cuda:0") for img, _ in items]
    outs = [torch.empty_like(x) for x in xs]
    ctx = _ctx(sum(snlm.workspace_bytes(*x.shape) for x in xs) + (1 << 20))
    jobs = snlm.job_array([ctx.job_for(x, o, 10, 3, 10.0 * sig, "box", "row_col")
                           for x, o, (_, sig) in zip(xs, outs, items)])
    waves = ctx.autotune_batch(jobs)
    for _ in range(3):
        ctx.denoise_jobs(jobs)
    ctx.sync()
    say("bench batch: waves per SIMD", waves, "pixels", sum(x.numel() for x in xs))
    worst = 0.0
    for i, ((img, sig), x, o) in enumerate(zip(items, xs, outs)):
        alone = ctx.denoise(x, 10, 3, 10.0 * sig, "box", "row_col", sync=True)
        assert torch.equal(alone, o), i
        ref = oracle.snlm(img.astype(np.float64), 10, 3, 10.0 * sig, "box", "row_col")
        worst = max(worst, max_abs(o.cpu().numpy(), ref))
    say("  whole-image max-abs over the 64 images", worst)
    assert worst <= TOL
    ctx.close()


def test_bench_batch_workload_gauss_f16_whole():
    """The benchmark's 64 ragged images with the other kernel, order and
    storage: FP16 inputs, Gaussian patch kernel (beta = K / 2), col_row, S=10,
    K=3, default waves.  Every output bitwise equal to its plain launch and
    within 1e-3 of the FP64 oracle (run on the FP16 values) at every pixel."""
    import torch
    import paper_1407_2343_amd as snlm
    from paper_1407_2343_amd.synth import batch_workload
    items = batch_workload(64, 128, 1024, seed=2000)
    xs = [torch.from_numpy(img.astype(np.float16)).to("cuda:0") for img, _ in items]
    outs = [torch.full(x.shape, -3.0, device="cuda:0") for x in xs]
    ctx = _ctx(sum(snlm.workspace_bytes(*x.shape) for x in xs) + (1 << 20))
    jobs = snlm.job_array([ctx.job_for(x, o, 10, 3, 10.0 * sig, "gauss", "col_row")
                           for x, o, (_, sig) in zip(xs, outs, items)])
    ctx.denoise_jobs(jobs, sync=True)
    worst = 0.0
    for i, ((img, sig), x, o) in enumerate(zip(items, xs, outs)):
        alone = ctx.denoise(x, 10, 3, 10.0 * sig, "gauss", "col_row", sync=True)
        assert torch.equal(alone, o), i
        ref = oracle.snlm(x.cpu().numpy().astype(np.float64), 10, 3, 10.0 * sig, "gauss", "col_row")
        worst = max(worst, max_abs(o.cpu().numpy(), ref))
    say("  gauss col_row FP16 batch: whole-image max-abs over the 64 images", worst)
    assert worst <= TOL
    ctx.close()


def test_autotune_keeps_bits():
    import torch
    import paper_1407_2343_amd as snlm
    img = noisy_image(700, 900, 20.0, seed=44)
    x = torch.from_numpy(img).to("cuda:0")
    ctx = _ctx(64 << 20)
    before = ctx.denoise(x, 10, 3, 200.0, sync=True).clone()
    best = ctx.autotune(x, 10, 3, 200.0)
    say("autotune chose", best)
    assert best > 0 and best % 16 == 0
    after = ctx.denoise(x, 10, 3, 200.0, sync=True)
    assert torch.equal(before, after)
    ctx.close()


def test_batch_autotune_and_tuning_file(tmp_path):
    import torch
    import paper_1407_2343_amd as snlm
    items = _ragged(6, 9)
    ctx = _ctx(64 << 20)
    xs = [torch.from_numpy(im).to("cuda:0") for im, _ in items]
    outs = [torch.empty_like(x) for x in xs]
    jobs = [ctx.job_for(x, o, 10, 3, 10 * s) for x, o, (_, s) in zip(xs, outs, items)]
    before = None
    ctx.denoise_jobs(jobs, sync=True)
    before = [o.clone() for o in outs]
    best = ctx.autotune_batch(jobs)
    assert 1 <= best <= 4
    ctx.denoise_jobs(jobs, sync=True)
    for a, b in zip(before, outs):
        assert torch.equal(a, b)
    path = str(tmp_path / "tune.json")
    ctx.save_tuning(path)
    text = open(path).read()
    assert '"batch"' in text and f'"waves_per_simd": {best}' in text
    other = _ctx(64 << 20)
    other.load_tuning(path)
    other.close()
    ctx.close()
