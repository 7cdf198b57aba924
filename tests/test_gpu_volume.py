"""Separable NLM of volumes on the GPU (the 1D pass along x, y and z in turn)
against the FP64 oracle, within 1e-3 max-abs."""
import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, max_abs, say
from paper_1407_2343_amd.synth import noisy_volume

pytestmark = pytest.mark.gpu


def _vol(D, H, W, seed, sigma=20.0):
    return noisy_volume(D, H, W, sigma, seed)


@pytest.mark.parametrize("shape", [(6, 40, 33), (3, 17, 70), (20, 9, 12), (1, 1, 1), (70, 3, 5)])
@pytest.mark.parametrize("axes", ["xyz", "zyx", "yzx"])
def test_volume_parity(shape, axes):
    import torch
    import paper_1407_2343_amd as snlm
    D, H, W = shape
    x = torch.from_numpy(_vol(D, H, W, D * 100 + H + W)).to("cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    y = ctx.denoise3d(x, 5, 2, 150.0, "box", axes)
    torch.cuda.synchronize()
    ref = oracle.snlm3d(x.cpu().numpy().astype(np.float64), 5, 2, 150.0, "box", axes)
    err = max_abs(y.cpu().numpy(), ref)
    say("volume", shape, axes, "max-abs %.2e" % err)
    assert err <= TOL
    ctx.close()


@pytest.mark.parametrize("kernel,S,K", [("gauss", 8, 3), ("box", 15, 4), ("box", 16, 8), ("gauss", 16, 8)])
def test_volume_kernels_f16(kernel, S, K):
    import torch
    import paper_1407_2343_amd as snlm
    x = torch.from_numpy(_vol(12, 31, 47, 5).astype(np.float16)).to("cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    y = ctx.denoise3d(x, S, K, 180.0, kernel, "zxy")
    torch.cuda.synchronize()
    ref = oracle.snlm3d(x.cpu().numpy().astype(np.float64), S, K, 180.0, kernel, "zxy")
    assert max_abs(y.cpu().numpy(), ref) <= TOL
    ctx.close()


def test_volume_slice_matches_2d():
    import torch
    import paper_1407_2343_amd as snlm
    x = torch.from_numpy(_vol(1, 50, 61, 8)).to("cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    y3 = ctx.denoise3d(x, 6, 2, 120.0, "box", "xyz")
    y2 = ctx.denoise(x[0], 6, 2, 120.0, "box", "row_col", sync=True)
    # the z pass over one sample averages 2S+1 copies of it: within FP32 rounding
    assert float((y3[0] - y2).abs().max()) <= 1e-4 * float(y2.abs().max())
    ctx.close()


def test_volume_errors():
    import ctypes
    import torch
    import paper_1407_2343_amd as snlm
    x = torch.zeros((2, 8, 8), device="cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    with pytest.raises(snlm.SnlmError) as e:
        ctx.denoise3d(x, 3, 2, 10.0, "box", "xxz")
    assert e.value.status == snlm.EINVAL
    o = torch.empty_like(x)
    bad = (ctypes.c_int * 3)(0, 0, 2)
    rc = snlm.lib().snlm_denoise3d(ctx.handle, ctypes.c_void_p(x.data_ptr()), 8, 0, ctypes.c_void_p(o.data_ptr()),
                                   8, 2, 8, 8, 3, 2, 10.0, 0, bad)
    assert rc == snlm.EINVAL
    small = snlm.Context(arena_bytes=256)
    ok = (ctypes.c_int * 3)(0, 1, 2)
    rc = snlm.lib().snlm_denoise3d(small.handle, ctypes.c_void_p(x.data_ptr()), 8, 0, ctypes.c_void_p(o.data_ptr()),
                                   8, 2, 8, 8, 3, 2, 10.0, 0, ok)
    assert rc == snlm.ENOMEM
    small.close()
    ctx.close()


@pytest.mark.parametrize("axes", ["xyz", "zyx"])
def test_volume_bench_whole(axes):
    """The volume workload as the benchmark times it: 256 x 256 x 256 FP32
    (the benchmark's seed), S=10, K=3, box, h = 10 sigma, both axis orders;
    every voxel within 1e-3 of the FP64 oracle."""
    import torch
    import paper_1407_2343_amd as snlm
    v = noisy_volume(256, 256, 256, 20.0, 9001)
    x = torch.from_numpy(v).to("cuda:0")
    ctx = snlm.Context(arena_bytes=1 << 16)
    y = ctx.denoise3d(x, 10, 3, 200.0, "box", axes)
    torch.cuda.synchronize()
    ref = oracle.snlm3d(v.astype(np.float64), 10, 3, 200.0, "box", axes)
    err = max_abs(y.cpu().numpy(), ref)
    say("bench volume", axes, "whole max-abs %.2e" % err)
    assert err <= TOL
    ctx.close()


@pytest.mark.parametrize("axes", ["xyz", "zyx"])
def test_volume_largest(axes):
    """A volume at the 2 GiB limit (511 x 1024 x 1024 FP32): its z lines
    reach byte offsets near 2^31.  Every z line carries the same signal f(z),
    so the x and y passes see constant lines and leave them as they are
    (every weight is 1), and every (y, x) line of the output must be the 1D
    NLM of f: checked on the device against the FP64 oracle's 1D result."""
    import torch
    import paper_1407_2343_amd as snlm
    D, H, W = 511, 1024, 1024
    assert 0.99 * 2 ** 31 < D * H * W * 4 < 2 ** 31 - 1
    f = (128.0 + 40.0 * np.random.default_rng(511).standard_normal(D)).astype(np.float32)
    x = torch.from_numpy(f).to("cuda:0").view(D, 1, 1).expand(D, H, W).contiguous()
    ctx = snlm.Context(arena_bytes=1 << 16)
    y = ctx.denoise3d(x, 10, 3, 200.0, "box", axes)
    torch.cuda.synchronize()
    g = torch.from_numpy(oracle.nlm1d(f.astype(np.float64), 10, 3, 200.0).astype(np.float32)).to("cuda:0")
    err = float((y - g.view(D, 1, 1)).abs().max())
    say("largest volume", axes, "max-abs %.2e" % err)
    assert err <= TOL
    del x, y
    ctx.close()
