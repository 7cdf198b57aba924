"""The recursive-Gaussian patch kernel (Young & van Vliet, the recursive
Gaussian Sec. 2.2 points to) on the GPU against the FP64 oracle, within 1e-3
max-abs.

Both sides run the same recursion from the same steady-state starts L =
ceil(6 beta) + S + 3 samples beyond each end of the reflected line.  The GPU
lifts in FP32, carries the recursion's state in FP64 (for wide kernels an FP32
state amplifies rounding by up to 1/B, ~2000 at beta = 20) and stores FP32, so
a distance's relative error stays near 3e-7 (three FP32 roundings, none
amplified: the filter has unit gain); with exponents that matter (up to ~20 in
base 2) a weight's relative error stays below ~5e-6, and the output's, weighted
by |x(j) - y(i)| <= 255, below 1e-3.  1e-3 is the bar of every other pass.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, max_abs, run_gpu, say
from paper_1407_2343_amd.synth import clean_image

pytestmark = pytest.mark.gpu


def _noisy(H, W, sigma, seed):
    rng = np.random.default_rng(seed)
    f0 = clean_image(H, W, rng)
    return (f0 + sigma * rng.standard_normal(f0.shape)).astype(np.float32)


def _ctx(arena=1 << 24):
    import paper_1407_2343_amd as snlm
    return snlm.Context(arena_bytes=arena)


def _check(ctx, img, S, beta, h, order="row_col", dtype="f32", seg_len=0):
    y, xr = run_gpu(ctx, img, S, 0, h, "gauss_iir", order, dtype=dtype, beta=beta, seg_len=seg_len)
    ref = oracle.snlm(xr, S, 0, h, "gauss_iir", order, beta=beta)
    err = max_abs(y, ref)
    say("iir", img.shape, "S", S, "beta", beta, "h", h, order, dtype, "seg", seg_len, "max-abs %.2e" % err)
    assert err <= TOL
    return y


@pytest.mark.parametrize("H,W", [(1, 1), (5, 3), (37, 53), (64, 64), (130, 47)])
@pytest.mark.parametrize("S,beta", [(1, 0.5), (5, 1.5), (10, 3.0), (16, 8.0)])
def test_iir_parity(H, W, S, beta):
    ctx = _ctx()
    _check(ctx, _noisy(H, W, 20.0, H * 1000 + W + S), S, beta, 150.0 * math.sqrt(beta))
    ctx.close()


@pytest.mark.parametrize("order", ["row_col", "col_row"])
def test_iir_orders_and_f16(order):
    ctx = _ctx()
    img = _noisy(96, 120, 25.0, 4)
    _check(ctx, img, 7, 2.0, 250.0, order)
    _check(ctx, img, 7, 2.0, 250.0, order, dtype="f16")
    ctx.close()


def test_iir_wide_patch_short_lines():
    """beta far above the exact FIR's reach (K <= 8), with lines shorter than
    the recursion's run-in L: the reflection wraps several periods."""
    ctx = _ctx()
    _check(ctx, _noisy(9, 300, 20.0, 8), 6, 20.0, 600.0)
    _check(ctx, _noisy(48, 40, 20.0, 9), 12, 64.0, 1200.0, "col_row")
    ctx.close()


@pytest.mark.parametrize("W,beta", [(3000, 8.0), (4000, 20.0)])
def test_iir_recursion_in_segments(W, beta):
    """Long lines: the recursions run in several segments, each started W
    samples early from a steady state (rho^W <= 1e-12), and still match the
    oracle's whole-line recursion."""
    ctx = _ctx(1 << 26)
    _check(ctx, _noisy(70, W, 20.0, 17), 6, beta, 150.0 * math.sqrt(beta))
    _check(ctx, _noisy(W, 40, 20.0, 18), 6, beta, 150.0 * math.sqrt(beta), "col_row")
    ctx.close()


def test_iir_segment_length_keeps_bits():
    """The job's seg_len does not reach the recursive kernel: its segments
    are a function of the image shape, S and beta alone, so any seg_len gives
    the same bits."""
    import torch
    ctx = _ctx()
    x = torch.from_numpy(_noisy(70, 333, 20.0, 10)).to("cuda:0")
    outs = [ctx.denoise(x, 9, 0, 300.0, "gauss_iir", "row_col", beta=2.5, seg_len=L, sync=True).cpu()
            for L in (16, 48, 352, 0)]
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    ref = oracle.snlm(x.cpu().numpy().astype(np.float64), 9, 0, 300.0, "gauss_iir", "row_col", beta=2.5)
    assert max_abs(outs[0].numpy(), ref) <= TOL
    ctx.close()


def test_iir_h_inf_is_window_mean():
    import torch
    from scipy.ndimage import uniform_filter1d
    ctx = _ctx()
    img = _noisy(40, 57, 20.0, 11)
    y, xr = run_gpu(ctx, img, 4, 0, math.inf, "gauss_iir", beta=3.0)
    ref = uniform_filter1d(uniform_filter1d(xr, 9, axis=1, mode="reflect"), 9, axis=0, mode="reflect")
    assert max_abs(y, ref) <= TOL
    ctx.close()


def test_iir_pitched():
    import torch
    big = torch.from_numpy(_noisy(50, 80, 15.0, 12)).to("cuda:0")
    x = big[4:44, 3:70]
    out_big = torch.full((45, 72), -7.0, device="cuda:0")
    out = out_big[2:42, 1:68]
    ctx = _ctx()
    ctx.denoise(x, 6, 0, 200.0, "gauss_iir", "col_row", beta=1.0, out=out, sync=True)
    ref = oracle.snlm(x.cpu().numpy().astype(np.float64), 6, 0, 200.0, "gauss_iir", "col_row", beta=1.0)
    assert max_abs(out.cpu().numpy(), ref) <= TOL
    assert float(out_big[0].max()) == -7.0 and float(out_big[:, 0].max()) == -7.0
    ctx.close()


def test_iir_default_beta_from_K():
    ctx = _ctx()
    img = _noisy(33, 65, 20.0, 13)
    y, xr = run_gpu(ctx, img, 5, 4, 220.0, "gauss_iir")  # beta = K / 2 = 2
    ref = oracle.snlm(xr, 5, 0, 220.0, "gauss_iir", beta=2.0)
    assert max_abs(y, ref) <= TOL
    ctx.close()


def test_iir_full_size_image():
    """A 1024 x 1024 image, S = 10, beta = 3, against the whole oracle image
    (the recursive distances cost O(S) per pixel on the CPU too)."""
    ctx = _ctx(1 << 26)
    img = _noisy(1024, 1024, 30.0, 14)
    _check(ctx, img, 10, 3.0, 400.0)
    ctx.close()


@pytest.mark.parametrize("beta", [2.0, 8.0])
def test_iir_bench_image_whole(beta):
    """The recursive-Gaussian workload as the benchmark times it: the 2048 x
    2048 image (sigma 30, the benchmark's seed), S = 10, h = 10 sigma
    sqrt(sqrt(2 pi) beta / 7), row_col, at beta = 2 and 8; every pixel
    against the oracle."""
    from paper_1407_2343_amd.synth import noisy_image
    ctx = _ctx(1 << 26)
    img = noisy_image(2048, 2048, 30.0, seed=7001)
    _check(ctx, img, 10, beta, 300.0 * math.sqrt(math.sqrt(2 * math.pi) * beta / 7.0))
    ctx.close()


def test_iir_close_to_exact_fir():
    """Within its approximation error the recursive kernel tracks the exact
    Gaussian FIR whose taps reach 3 beta (K = 6 at beta = 2): far closer than
    the box kernel is."""
    import torch
    ctx = _ctx()
    x = torch.from_numpy(_noisy(128, 128, 25.0, 15)).to("cuda:0")
    yi = ctx.denoise(x, 8, 0, 300.0, "gauss_iir", beta=2.0, sync=True).cpu().numpy()
    yf = ctx.denoise(x, 8, 6, 300.0, "gauss", beta=2.0, sync=True).cpu().numpy()
    yb = ctx.denoise(x, 8, 6, 300.0 * math.sqrt(13 / (math.sqrt(2 * math.pi) * 2.0)), "box", sync=True).cpu().numpy()
    d_if, d_fb = max_abs(yi, yf), max_abs(yf, yb)
    say("iir vs exact fir %.3f, fir vs box %.3f" % (d_if, d_fb))
    assert d_if < 0.5 * d_fb
    ctx.close()


@pytest.mark.parametrize("axes", ["xyz", "zyx"])
def test_iir_volume(axes):
    import torch
    rng = np.random.default_rng(16)
    v = (100.0 + 40.0 * rng.standard_normal((11, 19, 37))).astype(np.float32)
    x = torch.from_numpy(v).to("cuda:0")
    ctx = _ctx()
    y = ctx.denoise3d(x, 5, 3, 250.0, "gauss_iir", axes)  # beta = 1.5
    torch.cuda.synchronize()
    ref = oracle.snlm3d(v.astype(np.float64), 5, 3, 250.0, "gauss_iir", axes)
    err = max_abs(y.cpu().numpy(), ref)
    say("iir volume", axes, "max-abs %.2e" % err)
    assert err <= TOL
    ctx.close()


def test_iir_extremes():
    """The widest kernel (beta = 256: one recursion segment per line, the
    run-in L = 1555 reflecting a 20-sample line many times) at S = 16; S = 0
    (the identity, bitwise); and a tiny h (every weight but the centre's
    underflows: the identity up to rounding)."""
    import torch
    ctx = _ctx()
    _check(ctx, _noisy(20, 300, 20.0, 19), 16, 256.0, 6000.0)
    _check(ctx, _noisy(300, 20, 20.0, 20), 16, 256.0, 6000.0, "col_row")
    x = torch.from_numpy(_noisy(33, 47, 20.0, 21)).to("cuda:0")
    y0 = ctx.denoise(x, 0, 0, 100.0, "gauss_iir", beta=2.0, sync=True)
    assert torch.equal(y0, x)
    _check(ctx, _noisy(33, 47, 20.0, 22), 6, 2.0, 1e-3)
    ctx.close()


def test_iir_largest_buffers():
    """A 9430 x 9430 image at S = 16, beta = 2: each pass stores the forward
    recursion's FP64 state at the start of every block of 16 positions,
    16 * 593 blocks * 3 words per line (2.147 GB, 0.99997 of the 2 GiB limit
    of a region), so the 32-bit offsets of those loads and stores run at
    their limit; one pixel more per side and the job is rejected.  The whole
    output against the oracle."""
    import torch
    import paper_1407_2343_amd as snlm
    n = 9430
    L = 12 + 16 + 3
    nblk = (n + L - 1) // 16 + 2
    assert 0.9999 * 2 ** 31 < 16 * nblk * 3 * 8 * n < 2 ** 31 - 1
    nb = n + 10
    assert 16 * ((nb + L - 1) // 16 + 2) * 3 * 8 * nb > 2 ** 31 - 1
    rng = np.random.default_rng(9430)
    img = (128.0 + 30.0 * rng.standard_normal((n, n))).astype(np.float32)
    ctx = _ctx(snlm.workspace_bytes(n, n) + (1 << 20))
    _check(ctx, img, 16, 2.0, 300.0)
    with pytest.raises(snlm.SnlmError) as e:
        ctx.denoise(torch.zeros((nb, nb), device="cuda:0"), 16, 0, 300.0, "gauss_iir", beta=2.0)
    assert e.value.status == snlm.EINVAL
    ctx.close()


def test_iir_errors():
    import ctypes
    import torch
    import paper_1407_2343_amd as snlm
    x = torch.zeros((32, 32), device="cuda:0")
    ctx = _ctx()
    for beta, K in ((0.4, 2), (300.0, 2), (0.0, 0)):  # K = 0 gives the default beta 0
        with pytest.raises(snlm.SnlmError) as e:
            ctx.denoise(x, 3, K, 10.0, "gauss_iir", beta=beta)
        assert e.value.status == snlm.EINVAL
    with pytest.raises(snlm.SnlmError):
        ctx.denoise_batch([x], 3, 2, [10.0], "gauss_iir")
    with pytest.raises(snlm.SnlmError):
        ctx.denoise_sure(x, 3, 2, 10.0, 5.0, "gauss_iir")
    o = torch.empty_like(x)
    job = ctx.job_for(x, o, 3, 2, 10.0, "gauss_iir")
    t = ctypes.c_uint64(0)
    assert snlm.lib().snlm_submit(ctx.handle, ctypes.byref(job), ctypes.byref(t)) == snlm.EINVAL
    ctx.close()


def test_iir_random_sweep():
    """Seeded random cases over the kernels' block, segment and ring logic:
    shapes from single samples to a few hundred per axis (partial line groups,
    lines shorter than the run-in, several segments), S from 1 to 16, beta from
    0.5 to 64, both orders, FP32 and FP16 input; every pixel against the
    oracle."""
    rng = np.random.default_rng(2024)
    ctx = _ctx(1 << 26)
    for case in range(40):
        H = int(rng.integers(1, 300))
        W = int(rng.integers(1, 300))
        S = int(rng.integers(1, 17))
        beta = float(np.exp(rng.uniform(np.log(0.5), np.log(64.0))))
        order = "row_col" if rng.random() < 0.5 else "col_row"
        dtype = "f16" if rng.random() < 0.25 else "f32"
        h = 150.0 * math.sqrt(beta) * float(rng.uniform(0.5, 2.0))
        say("sweep case", case)
        _check(ctx, _noisy(H, W, 20.0, 7000 + case), S, beta, h, order, dtype)
    ctx.close()
