"""SURE-optimal combination of the two orders on the GPU (Sec. 3.1, Alg. 3,
Alg. 4) against the FP64 oracle run on exactly the values the GPU read.

* the combined output within 1e-3 max-abs (the parity bar of the 1D passes);
* f_cr, left in the workspace, bitwise equal to the plain col_row launch (the
  divergence pass adds accumulators but does not change the NLM arithmetic);
* the chained divergences of f_rc and f_cr within DIV_TOL of the oracle's;
* theta and the seven image sums close to the oracle's.

DIV_TOL: each 1D divergence is (1 + 2 ln2 (T + spread)) / Q evaluated in FP32
from at most 2S+1 weighted terms of centred differences; with FP32 weights
good to a few ulps and |2 ln2 (T + spread)| of order 1 for the workloads here,
the relative error of one factor stays below ~1e-5, and the product of two
below ~2e-5.  DIV_TOL = 2e-4 relative (plus 1e-6 absolute) leaves a 10x margin.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, max_abs, say
from paper_1407_2343_amd.synth import clean_image

pytestmark = pytest.mark.gpu

DIV_TOL = 2e-4


def _noisy(H, W, sigma, seed):
    rng = np.random.default_rng(seed)
    f0 = clean_image(H, W, rng)
    return (f0 + sigma * rng.standard_normal(f0.shape)).astype(np.float32)


def _ctx():
    import paper_1407_2343_amd as snlm
    return snlm.Context(arena_bytes=1 << 20)


def _check_against_oracle(ctx, x, S, K, h, sigma, kernel, xr=None):
    out, theta, stats = ctx.denoise_sure(x, S, K, h, sigma, kernel)
    import torch
    torch.cuda.synchronize()
    H, W = x.shape
    planes = ctx.sure_planes(H, W)
    if xr is None:
        xr = x.cpu().numpy().astype(np.float64)
    ref = oracle.sure(xr, S, K, h, sigma, kernel)
    err_out = max_abs(out.cpu().numpy(), ref["out"])
    err_cr = max_abs(planes["f_cr"].cpu().numpy(), ref["f_cr"])
    d_rc = planes["d_rc"].cpu().numpy().astype(np.float64)
    d_cr = planes["d_cr"].cpu().numpy().astype(np.float64)
    rel_rc = np.max(np.abs(d_rc - ref["d_rc"]) / (np.abs(ref["d_rc"]) + 1e-6 / DIV_TOL))
    rel_cr = np.max(np.abs(d_cr - ref["d_cr"]) / (np.abs(ref["d_cr"]) + 1e-6 / DIV_TOL))
    say("sure", (H, W), S, K, kernel, "theta", np.round(theta, 5), "oracle", np.round(ref["theta"], 5),
        "out %.2e f_cr %.2e div rel %.2e %.2e" % (err_out, err_cr, rel_rc, rel_cr))
    assert err_cr <= TOL
    assert rel_rc <= DIV_TOL and rel_cr <= DIV_TOL
    st = np.array(stats)
    assert np.all(np.abs(st - ref["stats"]) <= 1e-5 * np.abs(ref["stats"]) + 1e-3), (st, ref["stats"])
    assert err_out <= TOL
    return out, theta, ref


@pytest.mark.parametrize("S,K,kernel", [(5, 2, "box"), (4, 3, "gauss"), (10, 3, "box"), (16, 8, "box"),
                                         (16, 8, "gauss")])
def test_sure_parity(S, K, kernel):
    import torch
    sigma = 20.0
    x = torch.from_numpy(_noisy(75, 94, sigma, 31 + S)).to("cuda:0")
    ctx = _ctx()
    _check_against_oracle(ctx, x, S, K, 7.5 * sigma, sigma, kernel)
    ctx.close()


@pytest.mark.parametrize("H,W", [(1, 1), (3, 40), (17, 5), (130, 66)])
def test_sure_ragged(H, W):
    import torch
    sigma = 15.0
    x = torch.from_numpy(_noisy(H, W, sigma, 7 * H + W)).to("cuda:0")
    ctx = _ctx()
    _check_against_oracle(ctx, x, 6, 2, 100.0, sigma, "box")
    ctx.close()


def test_sure_f_cr_bitwise_plain():
    import torch
    x = torch.from_numpy(_noisy(96, 120, 25.0, 5)).to("cuda:0")
    ctx = _ctx()
    ctx.denoise_sure(x, 8, 3, 200.0, 25.0, "gauss")
    torch.cuda.synchronize()
    f_cr = ctx.sure_planes(96, 120)["f_cr"].clone()
    plain = ctx.denoise(x, 8, 3, 200.0, "gauss", "col_row", sync=True)
    assert torch.equal(f_cr, plain)
    ctx.close()


def test_sure_limits():
    """S = 0 leaves the image unchanged (theta1 + theta2 = 1 up to sigma's
    pull, the divergences are 1); h = inf makes the orders equal (theta1 =
    theta2)."""
    import torch
    x = torch.from_numpy(_noisy(40, 50, 10.0, 9)).to("cuda:0")
    ctx = _ctx()
    _check_against_oracle(ctx, x, 0, 2, 50.0, 10.0, "box")
    d = ctx.sure_planes(40, 50)
    assert float(d["d_rc"].min()) == 1.0 and float(d["d_rc"].max()) == 1.0
    _, theta, _ = _check_against_oracle(ctx, x, 4, 2, math.inf, 10.0, "box")
    assert theta[0] == theta[1]
    ctx.close()


def test_sure_f16_input():
    import torch
    x = torch.from_numpy(_noisy(64, 72, 20.0, 12).astype(np.float16)).to("cuda:0")
    ctx = _ctx()
    _check_against_oracle(ctx, x, 5, 2, 150.0, 20.0, "box",
                          xr=x.cpu().numpy().astype(np.float64))
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_sure_pitched_views(dtype):
    """Input and output as views into larger buffers: a base 3 elements past
    a 16-byte boundary and odd pitches, so the row passes cannot stage the
    input through LDS and the output goes out sample by sample.  The result
    is bitwise that of the same image stored contiguously (same arithmetic,
    other load and store paths), and within tolerance of the oracle."""
    import torch
    H, W = 77, 141
    img = _noisy(H, W, 20.0, 61)
    if dtype == "f16":
        img = img.astype(np.float16)
    x = torch.from_numpy(img).to("cuda:0")
    big = torch.full((H + 5, W + 7), 3.0, dtype=x.dtype, device="cuda:0")
    xv = big[2:2 + H, 3:3 + W]
    xv.copy_(x)
    obig = torch.full((H + 3, W + 9), -7.0, device="cuda:0")
    ov = obig[1:1 + H, 5:5 + W]
    ctx = _ctx()
    ref_out, ref_theta, _ = ctx.denoise_sure(x, 7, 2, 160.0, 20.0, "box")
    ref_out = ref_out.clone()
    out, theta, _ = _check_against_oracle(ctx, xv, 7, 2, 160.0, 20.0, "box",
                                          xr=x.cpu().numpy().astype(np.float64))
    assert theta == ref_theta
    assert torch.equal(out, ref_out)
    ov_out, _, _ = ctx.denoise_sure(xv, 7, 2, 160.0, 20.0, "box", out=ov)
    torch.cuda.synchronize()
    assert torch.equal(ov, ref_out)
    # nothing outside the output view was written
    mask = torch.ones_like(obig, dtype=torch.bool)
    mask[1:1 + H, 5:5 + W] = False
    assert bool((obig[mask] == -7.0).all())
    ctx.close()


def test_sure_bench_image_whole():
    """The SURE workload as the benchmark times it: a 2048 x 2048 image
    (synthetic clean image plus noise, sigma 30, the benchmark's seed), S=10,
    K=3, box, h = 10 sigma.  Every pixel of the combination and of f_cr
    within 1e-3 of the FP64 oracle, both divergence planes within 2e-4
    relative, theta and the seven sums as the oracle's."""
    import torch
    n, sigma = 2048, 30.0
    rng = np.random.default_rng(6001)
    f0 = clean_image(n, n, rng)
    f = (f0 + sigma * rng.standard_normal(f0.shape)).astype(np.float32)
    x = torch.from_numpy(f).to("cuda:0")
    ctx = _ctx()
    _check_against_oracle(ctx, x, 10, 3, 10 * sigma, sigma, "box")
    ctx.close()


def test_sure_larger_image():
    import torch
    sigma = 30.0
    x = torch.from_numpy(_noisy(384, 512, sigma, 77)).to("cuda:0")
    ctx = _ctx()
    _check_against_oracle(ctx, x, 10, 3, 10 * sigma, sigma, "box")
    ctx.close()


def test_sure_errors():
    import torch
    import paper_1407_2343_amd as snlm
    x = torch.zeros((32, 32), device="cuda:0")
    ctx = _ctx()
    with pytest.raises(snlm.SnlmError) as e:
        ctx.denoise_sure(x, 3, 2, 10.0, -1.0)
    assert e.value.status == snlm.EINVAL
    o = torch.empty_like(x)
    job = ctx.job_for(x, o, 3, 2, 10.0, "box", "row_col", "kahan")
    import ctypes
    rc = snlm.lib().snlm_denoise_sure(ctx.handle, ctypes.byref(job), 1.0, None, None)
    assert rc == snlm.EINVAL
    small = snlm.Context(arena_bytes=1024)
    job = small.job_for(x, o, 3, 2, 10.0)
    rc = snlm.lib().snlm_denoise_sure(small.handle, ctypes.byref(job), 1.0, None, None)
    assert rc == snlm.ENOMEM
    small.close()
    ctx.close()
