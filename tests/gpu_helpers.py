"""Helpers shared by the GPU tests: run the HIP path through the binding and
the FP64 oracle on exactly the values the GPU read."""
from __future__ import annotations

import sys

import numpy as np

TOL = 1e-3  # max-abs on the [0, 255] scale


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray, dtype="f32"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a.astype(np.float16 if dtype == "f16" else np.float32)))
    return t.to("cuda:0")


def run_gpu(ctx, img: np.ndarray, S, K, h, kernel="box", order="row_col", sum="block",
            dtype="f32", beta=None, seg_len=0):
    x = to_dev(img, dtype)
    y = ctx.denoise(x, S, K, h, kernel, order, sum, beta, seg_len, sync=True)
    return y.cpu().numpy().astype(np.float64), x.cpu().numpy().astype(np.float64)


def max_abs(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))))
