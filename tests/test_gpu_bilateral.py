"""Bilateral post-processing (Sec. 3.2, eq. BF) and the whole SNLM[f] on the
GPU against the FP64 oracle, within 1e-3 max-abs."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, max_abs, say
from paper_1407_2343_amd.synth import clean_image

pytestmark = pytest.mark.gpu


def _noisy(H, W, sigma, seed):
    rng = np.random.default_rng(seed)
    f0 = clean_image(H, W, rng)
    return (f0 + sigma * rng.standard_normal(f0.shape)).astype(np.float32)


@pytest.mark.parametrize("H,W", [(5, 3), (37, 53), (64, 64), (130, 47)])
@pytest.mark.parametrize("ss,sr", [(0.3, 30.0), (0.7069, 77.145), (1.0, 30.0), (2.5, math.inf), (2.95, 60.0)])
def test_bilateral_parity(H, W, ss, sr):
    import torch
    import paper_1407_2343_amd as snlm
    x = torch.from_numpy(_noisy(H, W, 20.0, H * 1000 + W)).to("cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    y = ctx.bilateral(x, ss, sr)
    torch.cuda.synchronize()
    ref = oracle.bilateral(x.cpu().numpy().astype(np.float64), ss, sr)
    err = max_abs(y.cpu().numpy(), ref)
    say("bilateral", (H, W), ss, sr, "max-abs %.2e" % err)
    assert err <= TOL
    ctx.close()


def test_bilateral_pitched():
    import torch
    import paper_1407_2343_amd as snlm
    big = torch.from_numpy(_noisy(40, 70, 15.0, 3)).to("cuda:0")
    x = big[3:33, 5:60]
    out_big = torch.full((35, 64), -7.0, device="cuda:0")
    out = out_big[2:32, 4:59]
    ctx = snlm.Context(arena_bytes=1 << 16)
    ctx.bilateral(x, 1.0, 50.0, out=out)
    torch.cuda.synchronize()
    ref = oracle.bilateral(x.cpu().numpy().astype(np.float64), 1.0, 50.0)
    assert max_abs(out.cpu().numpy(), ref) <= TOL
    assert float(out_big[0].max()) == -7.0 and float(out_big[:, :4].max()) == -7.0
    ctx.close()


def test_bilateral_params_rule():
    import paper_1407_2343_amd as snlm
    for s in (10.0, 15.0, 20.0, 30.0, 40.0):
        a, b = snlm.bilateral_params(s)
        ra, rb = oracle.bf_params(s)
        assert abs(a - ra) <= 1e-6 * abs(ra) and abs(b - rb) <= 1e-6 * abs(rb)


@pytest.mark.parametrize("kernel,S,K", [("box", 10, 3), ("gauss", 6, 2)])
def test_full_snlm(kernel, S, K):
    import torch
    import paper_1407_2343_amd as snlm
    sigma = 20.0
    x = torch.from_numpy(_noisy(90, 77, sigma, 40 + S)).to("cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    y, theta, _ = ctx.denoise_full(x, S, K, 7.5 * sigma, sigma, kernel)
    torch.cuda.synchronize()
    ref = oracle.full(x.cpu().numpy().astype(np.float64), S, K, 7.5 * sigma, sigma, kernel)
    err = max_abs(y.cpu().numpy(), ref["snlm"])
    say("full", kernel, S, K, "theta", np.round(theta, 4), "max-abs %.2e" % err)
    assert err <= TOL
    ctx.close()


def test_bilateral_errors():
    import torch
    import paper_1407_2343_amd as snlm
    x = torch.zeros((16, 16), device="cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    for ss, sr in ((0.0, 10.0), (3.0, 10.0), (1.0, 0.0), (float("nan"), 10.0)):
        with pytest.raises(snlm.SnlmError) as e:
            ctx.bilateral(x, ss, sr)
        assert e.value.status == snlm.EINVAL
    with pytest.raises(snlm.SnlmError):
        ctx.bilateral(x, 1.0, 10.0, out=x)  # overlap
    ctx.close()
