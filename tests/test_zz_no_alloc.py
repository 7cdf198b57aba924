"""snlm_enqueue_static (the entry point for callers that cannot allocate)
against snlm_enqueue_ex of the same jobs, through the C ABI: bitwise equal
outputs on two calls in a row, the second with a smaller image (the static
intermediate keeps the first call's contents), no device memory taken by the
call, and its error cases."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import TOL, max_abs, say

pytestmark = pytest.mark.gpu


def _call_static(snlm, torch, job):
    rc = snlm.lib().snlm_enqueue_static(ctypes.byref(job),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc


def test_static_matches_enqueue_ex(oracle_mod):
    import torch
    import paper_1407_2343_amd as snlm
    from paper_1407_2343_amd.synth import noisy_image
    torch.cuda.set_device(0)
    ctx = snlm.Context(arena_bytes=snlm.workspace_bytes(700, 900) + (1 << 20))
    cases = [(700, 900, 10, 3, "box", "row_col", "block", "f32"),
             (333, 257, 5, 2, "gauss", "col_row", "block", "f16"),
             (129, 65, 15, 4, "box", "row_col", "kahan", "f32")]
    for H, W, S, K, kernel, order, sm, dt in cases:
        say("static vs enqueue_ex", H, W, S, K, kernel, order, sm, dt)
        img = noisy_image(H, W, 20.0, seed=9100 + H)
        x = torch.from_numpy(img.astype(np.float16 if dt == "f16" else np.float32)).to("cuda:0")
        y_static = torch.full((H, W), -1.0, device="cuda:0")
        y_ref = torch.full((H, W), -2.0, device="cuda:0")
        torch.cuda.synchronize()
        j = ctx.job_for(x, y_static, S, K, 200.0, kernel, order, sm)
        # the process's first launch of a kernel may load its code object
        assert _call_static(snlm, torch, j) == snlm.OK
        free0 = torch.cuda.mem_get_info()[0]
        assert _call_static(snlm, torch, j) == snlm.OK
        assert torch.cuda.mem_get_info()[0] == free0  # the call took no device memory
        ctx.denoise_job_sync(ctx.job_for(x, y_ref, S, K, 200.0, kernel, order, sm))
        assert torch.equal(y_static, y_ref)
        ref = oracle_mod.snlm(x.cpu().numpy().astype(np.float64), S, K, 200.0, kernel, order)
        assert max_abs(y_static.cpu().numpy(), ref) <= TOL
    ctx.close()


def test_static_errors():
    import torch
    import paper_1407_2343_amd as snlm
    torch.cuda.set_device(0)
    x = torch.zeros((64, 64), device="cuda:0")
    y = torch.empty_like(x)
    ok = snlm.make_job(x.data_ptr(), y.data_ptr(), 64, 64, 5, 2, 100.0, "box", "row_col", ld_in=64, ld_out=64)
    assert _call_static(snlm, torch, ok) == snlm.OK
    iir = snlm.make_job(x.data_ptr(), y.data_ptr(), 64, 64, 5, 0, 100.0, "gauss_iir", "row_col",
                        ld_in=64, ld_out=64)
    assert _call_static(snlm, torch, iir) == snlm.EINVAL
    bad = snlm.make_job(x.data_ptr(), y.data_ptr(), 64, 64, 17, 2, 100.0, "box", "row_col", ld_in=64, ld_out=64)
    assert _call_static(snlm, torch, bad) == snlm.EINVAL
    # an image whose FP32 intermediate exceeds the static array (shape only:
    # the size check comes before any launch)
    big = torch.empty((4097, 4096), device="cuda:0")
    out = torch.empty_like(big)
    j = snlm.make_job(big.data_ptr(), out.data_ptr(), 4097, 4096, 5, 2, 100.0, "box", "row_col",
                      ld_in=4096, ld_out=4096)
    assert _call_static(snlm, torch, j) == snlm.ENOMEM
