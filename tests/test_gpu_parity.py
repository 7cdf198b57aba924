"""GPU path (through the C ABI) against the FP64 oracle, element by element,
on the same seeded inputs: max-abs <= 1e-3 on the [0, 255] scale."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, max_abs, run_gpu, say
from paper_1407_2343_amd.synth import noisy_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1407_2343_amd as snlm
    c = snlm.Context(arena_bytes=64 << 20)
    yield c
    c.close()


def check(ctx, img, S, K, h, kernel="box", order="row_col", sum="block", dtype="f32",
          beta=None, seg_len=0, tol=TOL):
    say("case", img.shape, S, K, h, kernel, order, sum, dtype, seg_len)
    y, x_read = run_gpu(ctx, img, S, K, h, kernel, order, sum, dtype, beta, seg_len)
    ref = oracle.snlm(x_read, S, K, h, kernel, order, beta)
    err = max_abs(y, ref)
    say("  max-abs", err)
    assert err <= tol, err
    return y, ref


def test_config_small_64(ctx):
    img = noisy_image(64, 64, 20.0, seed=1000, texture=False)
    check(ctx, img, 5, 2, 200.0)


@pytest.mark.parametrize("kernel", ["box", "gauss"])
@pytest.mark.parametrize("order", ["row_col", "col_row"])
def test_config_512(ctx, kernel, order):
    img = noisy_image(512, 512, 20.0, seed=1001, texture=True)
    check(ctx, img, 10, 3, 200.0, kernel, order)


SHAPES = [(1, 1), (1, 37), (37, 1), (2, 2), (5, 3), (17, 130), (70, 200), (130, 67), (64, 64),
          (65, 129)]


@pytest.mark.parametrize("shape", SHAPES)
def test_ragged_shapes(ctx, shape):
    H, W = shape
    img = noisy_image(H, W, 25.0, seed=7 + H * 1000 + W, texture=True)
    for (S, K, kernel) in [(3, 1, "box"), (10, 3, "gauss"), (16, 8, "box")]:
        check(ctx, img, S, K, 10 * 25.0, kernel, "row_col" if (H + W) % 2 else "col_row")


@pytest.mark.parametrize("S", [1, 2, 4, 7, 11, 13, 15, 16])
@pytest.mark.parametrize("K", [0, 3, 5, 8])
def test_parameter_grid(ctx, S, K):
    img = noisy_image(48, 96, 15.0, seed=S * 31 + K, texture=True)
    check(ctx, img, S, K, 120.0, "box" if (S + K) % 2 else "gauss", "row_col")


def test_f16_input(ctx):
    img = noisy_image(200, 260, 30.0, seed=55, texture=True)
    for kernel in ("box", "gauss"):
        check(ctx, img, 10, 3, 300.0, kernel, "col_row", dtype="f16")


@pytest.mark.parametrize("sum", ["plain", "kahan"])
def test_whole_line_sums(ctx, sum):
    img = noisy_image(300, 520, 20.0, seed=77, texture=True)
    check(ctx, img, 10, 3, 200.0, "box", "row_col", sum=sum)


@pytest.mark.parametrize("sum", ["plain", "kahan"])
def test_whole_line_sums_in_segments_keep_bits(ctx, sum):
    """Whole-line (plain / Kahan) running sums cut into segments that start
    from the scanned states give bitwise the one-segment result, in both
    passes (rows 333 long, columns 150 long), FP32 and FP16 input."""
    img = noisy_image(150, 333, 20.0, seed=14, texture=True)
    for dtype in ("f32", "f16"):
        base, _ = run_gpu(ctx, img, 10, 3, 200.0, "box", "row_col", sum=sum, dtype=dtype,
                          seg_len=1 << 20)
        for seg in (16, 48, 64, 176):
            y, _ = run_gpu(ctx, img, 10, 3, 200.0, "box", "row_col", sum=sum, dtype=dtype, seg_len=seg)
            assert np.array_equal(y, base), (sum, dtype, seg)
        y, _ = run_gpu(ctx, img, 15, 4, 200.0, "box", "col_row", sum=sum, dtype=dtype, seg_len=32)
        b2, _ = run_gpu(ctx, img, 15, 4, 200.0, "box", "col_row", sum=sum, dtype=dtype, seg_len=1 << 20)
        assert np.array_equal(y, b2), (sum, dtype)


def test_h_infinite_is_moving_average(ctx):
    img = noisy_image(50, 70, 20.0, seed=9)
    check(ctx, img, 4, 2, math.inf, "box", "row_col")


def test_h_tiny_is_identity(ctx):
    img = noisy_image(40, 90, 20.0, seed=10)
    y, ref = check(ctx, img, 6, 2, 1e-3, "gauss", "col_row")
    assert max_abs(y, img.astype(np.float32)) <= TOL


def test_s0_is_copy(ctx):
    img = noisy_image(33, 47, 20.0, seed=11)
    y, _ = run_gpu(ctx, img, 0, 3, 100.0)
    assert np.array_equal(y, img.astype(np.float32).astype(np.float64))


def test_constant_image(ctx):
    img = np.full((90, 110), 123.5)
    y, _ = run_gpu(ctx, img, 10, 3, 200.0, "box", "row_col")
    assert max_abs(y, img) <= 1e-4


def test_segment_length_does_not_change_bits(ctx):
    """Segment boundaries repeat the previous chunk's arithmetic exactly."""
    img = noisy_image(150, 333, 20.0, seed=12, texture=True)
    base = None
    for seg in (16, 32, 48, 64, 128, 336):
        for kernel in ("box", "gauss"):
            y, _ = run_gpu(ctx, img, 10, 3, 200.0, kernel, "row_col", seg_len=seg)
            if kernel == "box":
                if base is None:
                    base = y
                assert np.array_equal(y, base), seg


def test_transpose_relation(ctx):
    """RC(X) = CR(X^T)^T bitwise: both passes run the same per-line code."""
    img = noisy_image(77, 141, 20.0, seed=13, texture=True)
    a, _ = run_gpu(ctx, img, 7, 2, 150.0, "gauss", "row_col")
    b, _ = run_gpu(ctx, np.ascontiguousarray(img.T), 7, 2, 150.0, "gauss", "col_row")
    assert np.array_equal(a, b.T)


def _strided(img, pad, offset=0):
    """A device view of img inside a wider buffer: row pitch W + pad, first
    column at `offset` (offsets that are not a multiple of 4 floats make the
    base address unaligned for 16-byte accesses)."""
    import torch
    H, W = img.shape
    buf = torch.zeros((H, W + pad), dtype=torch.float32, device="cuda:0")
    view = buf[:, offset:offset + W]
    view.copy_(torch.from_numpy(img.astype(np.float32)).to("cuda:0"))
    return view


@pytest.mark.parametrize("pad,offset", [(3, 0), (5, 1), (8, 4), (1, 0)])
@pytest.mark.parametrize("order", ["row_col", "col_row"])
def test_pitched_and_unaligned_views(ctx, pad, offset, order):
    """Row pitches that are not multiples of 4 and unaligned base addresses
    (the vector-load tiles of the row pass must handle or avoid them)."""
    import torch
    img = noisy_image(70, 203, 20.0, seed=21 + pad, texture=True)
    x = _strided(img, pad, offset)
    out_buf = torch.zeros((70, 203 + pad + 2), dtype=torch.float32, device="cuda:0")
    out = out_buf[:, 1:204]
    say("case pitched", pad, offset, order, x.stride(), out.stride())
    ctx.denoise(x, 10, 3, 200.0, "box", order, out=out, sync=True)
    ref = oracle.snlm(img.astype(np.float32).astype(np.float64), 10, 3, 200.0, "box", order)
    err = max_abs(out.cpu().numpy(), ref)
    say("  max-abs", err)
    assert err <= TOL
    # nothing outside the output view was written
    assert float(out_buf[:, 0].abs().max()) == 0.0
    assert float(out_buf[:, 204:].abs().max()) == 0.0


def test_largest_image():
    """The largest square image the library accepts (23168 x 23168 FP32: the
    padded FP32 intermediate just below 2 GiB, every byte offset of the
    32-bit buffer addressing in use), S=10, K=3, both orders: pixels at the
    corners, on the borders and inside, against the oracle run on crops that
    hold each pixel's whole reach (S + K in both directions, so the crop's
    own edges are never reflected into the result)."""
    import torch
    import paper_1407_2343_amd as snlm
    n = 23168
    rc, why = snlm.validate(snlm.make_job(1 << 20, (1 << 20) + 4 * n * n + 4096, n, n, 10, 3, 200.0))
    assert rc == snlm.OK, why
    rng = np.random.default_rng(23168)
    img = (128.0 + 30.0 * rng.standard_normal((n, n), dtype=np.float32)).astype(np.float32)
    x = torch.from_numpy(img).to("cuda:0")
    ctx = snlm.Context(arena_bytes=snlm.workspace_bytes(n, n) + (1 << 20))
    R = 13  # S + K
    pts = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (n // 2, 0), (0, n // 2), (n - 1, n // 3),
           (n // 3, n - 1), (n // 2, n // 2), (12345, 20000), (n - 14, n - 14), (R, R)]
    for order in ("row_col", "col_row"):
        y = ctx.denoise(x, 10, 3, 200.0, "box", order, sync=True)
        rows = torch.tensor([p[0] for p in pts], device="cuda:0")
        cols = torch.tensor([p[1] for p in pts], device="cuda:0")
        got = y[rows, cols].cpu().numpy()
        worst = 0.0
        for k, (r, c) in enumerate(pts):
            r0, c0 = max(0, r - R), max(0, c - R)
            r1, c1 = min(n, r + R + 1), min(n, c + R + 1)
            # a crop touching an image border must start (or end) there so
            # that the reflection at that border is the image's own
            crop = img[r0:r1, c0:c1].astype(np.float64)
            assert (r0 == 0 or r - r0 == R) and (r1 == n or r1 - 1 - r == R)
            ref = oracle.pixel(crop, r - r0, c - c0, 10, 3, 200.0, "box", order)
            worst = max(worst, abs(float(got[k]) - ref))
        say("largest image", order, "sampled max-abs %.2e" % worst)
        assert worst <= TOL
        del y
    ctx.close()
