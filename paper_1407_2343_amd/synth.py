"""Seeded synthetic inputs for separable non-local means.

This module only draws numbers: it holds none of the denoiser's arithmetic, so
both the GPU library's tests and the FP64 oracle can take their inputs from it.

Image family (stand-in for the natural test images the paper uses, which are not
available here):

1. background uniform in [0, 255];
2. ``8 + H*W // 16384`` shapes, alternating axis-aligned rectangles and discs,
   placed uniformly, painted in order with intensities uniform in [0, 255];
   rectangle half-sides log-uniform in [2, max(H,W)/4] per axis, disc radii
   log-uniform in [2, max(H,W)/6];
3. a linear gradient with random direction and total excursion uniform in
   [-64, 64];
4. optionally a fine sinusoidal texture ``12*sin(2*pi*(x cos phi + y sin phi)/p + psi)``
   with period p uniform in [4, 16] px;
5. clipped to [0, 255];
6. additive white Gaussian noise of standard deviation sigma, not clipped
   (the noise model f = f0 + sigma*w of Sec. 3.1, eq. noise);
7. cast to the stored dtype.
"""
from __future__ import annotations

import math

import numpy as np


def clean_image(H: int, W: int, rng: np.random.Generator, texture: bool = True) -> np.ndarray:
    """Piecewise-constant shapes + gradient (+ texture), clipped to [0, 255], float64."""
    img = np.full((H, W), rng.uniform(0.0, 255.0), dtype=np.float64)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    n_shapes = 8 + (H * W) // 16384
    big = max(H, W)
    for s in range(n_shapes):
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        val = rng.uniform(0.0, 255.0)
        if s % 2 == 0:
            hy = math.exp(rng.uniform(math.log(2.0), math.log(max(2.0, big / 4.0))))
            hx = math.exp(rng.uniform(math.log(2.0), math.log(max(2.0, big / 4.0))))
            y0, y1 = int(max(0, cy - hy)), int(min(H, cy + hy + 1))
            x0, x1 = int(max(0, cx - hx)), int(min(W, cx + hx + 1))
            img[y0:y1, x0:x1] = val
        else:
            r = math.exp(rng.uniform(math.log(2.0), math.log(max(2.0, big / 6.0))))
            y0, y1 = int(max(0, cy - r - 1)), int(min(H, cy + r + 2))
            x0, x1 = int(max(0, cx - r - 1)), int(min(W, cx + r + 2))
            if y1 > y0 and x1 > x0:
                sub_y = yy[y0:y1, x0:x1]
                sub_x = xx[y0:y1, x0:x1]
                mask = (sub_y - cy) ** 2 + (sub_x - cx) ** 2 <= r * r
                img[y0:y1, x0:x1][mask] = val
    ang = rng.uniform(0.0, 2.0 * math.pi)
    excursion = rng.uniform(-64.0, 64.0)
    proj = xx * math.cos(ang) + yy * math.sin(ang)
    span = max(proj.max() - proj.min(), 1.0)
    img += excursion * (proj - proj.min()) / span
    if texture:
        period = rng.uniform(4.0, 16.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        psi = rng.uniform(0.0, 2.0 * math.pi)
        img += 12.0 * np.sin(2.0 * math.pi * (xx * math.cos(phi) + yy * math.sin(phi)) / period + psi)
    np.clip(img, 0.0, 255.0, out=img)
    return img


def noisy_image(H: int, W: int, sigma: float, seed: int, texture: bool = True,
                dtype=np.float32) -> np.ndarray:
    """Clean image plus N(0, sigma^2) noise (unclipped), cast to ``dtype``."""
    rng = np.random.default_rng(seed)
    f0 = clean_image(H, W, rng, texture)
    f = f0 + sigma * rng.standard_normal((H, W))
    return f.astype(dtype)


def noisy_volume(D: int, H: int, W: int, sigma: float, seed: int) -> np.ndarray:
    """A smooth D x H x W pattern (a sinusoid in x and y, a ramp in z) plus
    N(0, sigma^2) noise, float32."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    clean = 128 + 60 * np.sin(x / 7.0) * np.cos(y / 5.0) + 3.0 * z
    return (clean + sigma * rng.standard_normal(clean.shape)).astype(np.float32)


def noisy_line(N: int, sigma: float, seed: int) -> np.ndarray:
    """A 1D piecewise-constant signal in [0, 1] plus N(0, sigma^2) noise, float64."""
    rng = np.random.default_rng(seed)
    x = np.empty(N)
    pos = 0
    while pos < N:
        run = int(rng.integers(8, 64))
        x[pos:pos + run] = rng.uniform(0.0, 1.0)
        pos += run
    return x + sigma * rng.standard_normal(N)


def batch_shapes(n: int, lo: int, hi: int, seed: int):
    """n (H, W) pairs, each axis drawn log-uniform in [lo, hi] independently."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        H = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        W = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append((H, W))
    return out


def batch_workload(n: int = 64, lo: int = 128, hi: int = 1024, seed: int = 2000,
                   sigmas=(10.0, 20.0, 30.0, 40.0), texture: bool = True):
    """Ragged batch: list of (image float32, sigma).  Shapes log-uniform per axis,
    sigma drawn from ``sigmas`` per image."""
    rng = np.random.default_rng(seed)
    shapes = batch_shapes(n, lo, hi, seed + 1)
    out = []
    for i, (H, W) in enumerate(shapes):
        sigma = float(sigmas[int(rng.integers(0, len(sigmas)))])
        out.append((noisy_image(H, W, sigma, seed * 1000 + i, texture), sigma))
    return out


def serving_requests(n: int = 2000, seed: int = 4000, lo: int = 64, hi: int = 2048,
                     rate_per_s: float = 1000.0):
    """Request descriptors for the serving workload (no pixels): arrival time
    (Poisson process of the given rate), H, W, sigma ~ U[10, 40], S in {5,10,15},
    K in {2,3,4}, kernel box/gauss 50/50, order row_col/col_row 50/50, image seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        H = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        W = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        reqs.append(dict(
            arrival=t, H=H, W=W,
            sigma=float(rng.uniform(10.0, 40.0)),
            S=int(rng.choice([5, 10, 15])),
            K=int(rng.choice([2, 3, 4])),
            kernel="gauss" if rng.random() < 0.5 else "box",
            order="col_row" if rng.random() < 0.5 else "row_col",
            seed=seed * 10000 + i,
        ))
    return reqs
