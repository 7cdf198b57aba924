"""Serving and the synchronous / enqueued forms of the direct calls, on the GPU.

* a served job reads its input only after the caller's stream has produced
  it: the input is written by a GPU copy queued behind a long computation on
  the context stream, and the job is submitted with no host synchronisation;
* the native request driver (snlm_submit_many) with Poisson-like arrivals:
  every result equals the same job run alone, and each job reports a device
  latency (submit event to the end of its round) no larger than what the host
  observed;
* direct calls are refused (SNLM_EBUSY) while served jobs hold the arena, and
  the binding refuses to grow the arena under outstanding tickets;
* snlm_denoise_ex and snlm_denoise_batch return with the result in place: a
  copy on an unrelated stream right after the call sees the finished output.
"""
import time

import numpy as np
import pytest

from gpu_helpers import say
from paper_1407_2343_amd.synth import noisy_image

pytestmark = pytest.mark.gpu


def _wait_all(srv, tickets, limit_s=60.0):
    import paper_1407_2343_amd as snlm
    pending = set(tickets)
    t0 = time.time()
    done = {}
    while pending and time.time() - t0 < limit_s:
        for t in list(pending):
            ts = srv.job_times(t)
            if ts[2] > 0:
                done[t] = (ts, srv.job_device_ms(t))
                st = srv.poll(t)
                assert st == snlm.OK, (t, st, srv.last_error())
                pending.discard(t)
        time.sleep(0.0005)
    assert not pending, "served jobs did not finish"
    return done


def test_served_job_ordered_after_caller_stream():
    import torch
    import paper_1407_2343_amd as snlm
    H, W = 1024, 1536
    src = torch.from_numpy(noisy_image(H, W, 20.0, seed=8101)).to("cuda:0")
    a = torch.randn((4096, 4096), device="cuda:0")
    b = torch.randn((4096, 4096), device="cuda:0")
    x = torch.full((H, W), float("nan"), device="cuda:0")
    o = torch.full((H, W), -1.0, device="cuda:0")
    srv = snlm.Context(arena_bytes=64 << 20)
    solo = snlm.Context(arena_bytes=64 << 20)
    job = srv.job_for(x, o, 10, 3, 200.0, "box", "row_col")
    torch.cuda.synchronize()
    # several milliseconds of work on the context stream, then the input is written
    for _ in range(8):
        a = torch.mm(a, b) * 1e-3
    x.copy_(src)
    t = srv.submit(job)  # no host synchronisation in between
    _wait_all(srv, [t])
    torch.cuda.synchronize()
    alone = solo.denoise(src, 10, 3, 200.0, "box", "row_col", sync=True)
    say("ordered after caller stream", bool(torch.equal(o, alone)))
    assert torch.equal(o, alone)
    srv.close()
    solo.close()


def test_submit_many_device_latency_and_mix():
    import torch
    import paper_1407_2343_amd as snlm
    rng = np.random.default_rng(17)
    srv = snlm.Context(arena_bytes=64 << 20)
    solo = snlm.Context(arena_bytes=64 << 20)
    reqs, jobs = [], []
    for i in range(40):
        H = int(np.exp(rng.uniform(np.log(64), np.log(1400))))
        W = int(np.exp(rng.uniform(np.log(64), np.log(1400))))
        sig = float(rng.uniform(10, 40))
        S, K = int(rng.choice([5, 10, 15])), int(rng.choice([2, 3, 4]))
        kern = "gauss" if rng.random() < 0.5 else "box"
        order = "col_row" if rng.random() < 0.5 else "row_col"
        dtype = torch.float16 if i % 5 == 0 else torch.float32
        x = torch.from_numpy(noisy_image(H, W, sig, 8200 + i)).to("cuda:0").to(dtype)
        o = torch.full((H, W), -1.0, device="cuda:0")
        if i % 7 == 3:
            # pitched, unaligned views: the slot copies go row by row
            xb = torch.zeros((H, W + 5), dtype=dtype, device="cuda:0")
            xb[:, 1:1 + W] = x
            x = xb[:, 1:1 + W]
            ob = torch.full((H, W + 3), -1.0, device="cuda:0")
            o = ob[:, 2:2 + W]
        reqs.append((x, o, S, K, 10 * sig, kern, order))
        jobs.append(srv.job_for(x, o, S, K, 10 * sig, kern, order))
    torch.cuda.synchronize()
    arrivals = np.cumsum(rng.exponential(2e-4, len(jobs)))
    tickets = srv.submit_many(jobs, arrivals)
    assert len(set(tickets)) == len(jobs) and all(t > 0 for t in tickets)
    done = _wait_all(srv, tickets)
    for t in tickets:
        (ts, ta, td), dev_ms = done[t]
        assert ts <= ta <= td
        # the device's own submit-to-done time cannot exceed what the host saw
        # by more than the host's sampling of the round's completion
        assert 0.0 < dev_ms <= (td - ts) / 1e3 + 0.5, (dev_ms, (td - ts) / 1e3)
    for i, (x, o, S, K, h, kern, order) in enumerate(reqs):
        alone = solo.denoise(x, S, K, h, kern, order, sync=True)
        assert torch.equal(o, alone), i
    lat = sorted(d for _, d in done.values())
    say("device latency p50 %.3f ms max %.3f ms" % (lat[len(lat) // 2], lat[-1]))
    srv.close()
    solo.close()


def test_direct_calls_refused_while_serving():
    import torch
    import paper_1407_2343_amd as snlm
    srv = snlm.Context(arena_bytes=64 << 20)
    x = torch.from_numpy(noisy_image(2048, 2048, 20.0, seed=8301)).to("cuda:0")
    o = torch.empty_like(x)
    small = torch.from_numpy(noisy_image(64, 80, 20.0, seed=8302)).to("cuda:0")
    torch.cuda.synchronize()
    t = srv.submit(srv.job_for(x, o, 15, 4, 200.0, "box", "row_col"))
    with pytest.raises(snlm.SnlmError) as e:
        srv.denoise(small, 5, 2, 200.0)
    assert e.value.status == snlm.EBUSY
    with pytest.raises(snlm.SnlmError) as e:
        srv.ensure_arena(256 << 20)
    assert e.value.status == snlm.EBUSY
    _wait_all(srv, [t])
    y = srv.denoise(small, 5, 2, 200.0, sync=True)  # allowed again
    assert torch.isfinite(y).all()
    srv.close()


def test_sync_calls_return_finished_results():
    import torch
    import paper_1407_2343_amd as snlm
    side = torch.cuda.Stream()
    own = torch.cuda.Stream()
    ctx = snlm.Context(arena_bytes=256 << 20, stream=own)
    x = torch.from_numpy(noisy_image(2048, 2048, 20.0, seed=8401)).to("cuda:0")
    o = torch.full_like(x, -1.0)
    job = ctx.job_for(x, o, 15, 4, 200.0, "box", "row_col")
    xs = [torch.from_numpy(noisy_image(700 + 13 * i, 900 - 11 * i, 20.0, seed=8410 + i)).to("cuda:0")
          for i in range(6)]
    os_ = [torch.full_like(v, -1.0) for v in xs]
    jobs = snlm.job_array([ctx.job_for(v, w, 10, 3, 200.0) for v, w in zip(xs, os_)])
    torch.cuda.synchronize()
    ctx.denoise_job_sync(job)
    with torch.cuda.stream(side):  # not ordered after the context stream
        got = o.to("cpu")
    ctx.denoise_jobs_sync(jobs)
    with torch.cuda.stream(side):
        got_b = [w.to("cpu") for w in os_]
    torch.cuda.synchronize()
    assert torch.equal(got, o.cpu())
    for g, w in zip(got_b, os_):
        assert torch.equal(g, w.cpu())
    assert (got != -1.0).all()
    ctx.close()
