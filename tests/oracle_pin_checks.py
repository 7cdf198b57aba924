"""Checks that tie the FP64 oracle to things other than itself.

Each ``check_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with what the paper or the mathematics fixes.  They are run
against the real oracle (tests/test_oracle_pins.py) and against copies of it
with planted mistakes (tests/test_oracle_mutants.py), which must each fail at
least one check.
"""
from __future__ import annotations

import math
import os

import numpy as np
from scipy.ndimage import uniform_filter1d

import patchlift_ref as pl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_MATH = {k: getattr(math, k) for k in ("exp", "log", "sqrt")}
_MATH["e"] = math.e


def _eval(expr: str, env: dict) -> float:
    return float(eval(expr, {"__builtins__": {}}, {**_MATH, **env}))


def _parse_blocks(path: str):
    blocks, cur = [], None
    for raw in open(path):
        line = raw.strip()
        if not line or line.startswith("#"):
            continue
        key, _, val = line.partition(":")
        val = val.strip()
        if key == "case":
            cur = {"case": val, "define": []}
            blocks.append(cur)
        elif key == "define":
            cur["define"].append(val)
        elif key != "why":
            cur[key] = val
    return blocks


def _params(s: str) -> dict:
    out = {}
    for tok in s.split():
        k, v = tok.split("=")
        out[k] = v if k == "kernel" else float(v)
    return out


def check_worked_examples_1d(orc):
    for b in _parse_blocks(os.path.join(GOLDEN, "worked_examples.txt")):
        x = [float(v) for v in b["x"].split()]
        p = _params(b["params"])
        want = [_eval(e, {}) for e in b["expect"].split(";")]
        got = orc.nlm1d(x, int(p["S"]), int(p["K"]), p["h"], p["kernel"], p.get("beta"))
        assert np.allclose(got, want, rtol=0, atol=1e-13), (b["case"], got, want)


def check_separable_2x2(orc):
    path = os.path.join(GOLDEN, "separable_2x2.txt")
    text = {}
    defs = []
    for raw in open(path):
        line = raw.strip()
        if not line or line.startswith("#"):
            continue
        key, _, val = line.partition(":")
        if key == "define":
            defs.append(val.strip())
        else:
            text[key] = val.strip()
    env = {}
    for d in defs:
        name, expr = d.split("=", 1)
        env[name.strip()] = _eval(expr, env)
    f = np.array([[float(v) for v in row.split()] for row in text["f"].split(";")])
    p = _params(text["params"])
    for order in ("row_col", "col_row"):
        want = np.array([[_eval(e, env) for e in row.split(",")]
                         for row in text["expect_" + order].split(";")])
        got = orc.snlm(f, int(p["S"]), int(p["K"]), p["h"], p["kernel"], order)
        assert np.allclose(got, want, rtol=0, atol=1e-13), (order, got, want)


def check_alg1_distances(orc, seed: int = 7):
    """Alg. 1 + eq. dist (zero extension) == direct distances, exactly, on
    integer signals with the box kernel; the oracle sees the signal embedded in
    zeros so that no reflection is involved."""
    rng = np.random.default_rng(seed)
    for (N, S, K) in [(8, 2, 1), (13, 4, 3), (20, 5, 2), (9, 3, 0)]:
        x = rng.integers(-9, 10, N).astype(np.float64)
        d = pl.alg1_distances(x, S, K, "box")
        big = np.concatenate([np.zeros(K), x, np.zeros(K)])
        for (i, j), v in d.items():
            assert orc.patch_d2(big, i + K, j + K, K, "box") == v, (N, S, K, i, j)
    # Gaussian taps: agreement to rounding
    x = rng.normal(size=15)
    d = pl.alg1_distances(x, 4, 3, "gauss", 1.5)
    big = np.concatenate([np.zeros(3), x, np.zeros(3)])
    for (i, j), v in d.items():
        ref = orc.patch_d2(big, i + 3, j + 3, 3, "gauss", 1.5)
        assert abs(ref - v) <= 1e-12 * max(1.0, abs(ref)), (i, j, ref, v)


def check_difference_lift(orc, seed: int = 11):
    """Difference-lift prefix sums (eq. recursion) on the reflected extension ==
    direct distances: exact for integer signals and the box kernel."""
    rng = np.random.default_rng(seed)
    for (N, S, K) in [(1, 3, 2), (2, 4, 1), (7, 5, 3), (16, 6, 4), (25, 3, 0)]:
        x = rng.integers(-20, 21, N).astype(np.float64)
        d = pl.difference_lift_distances(x, S, K, "box")
        for s in range(S + 1):
            for t in range(-S, N):
                assert orc.patch_d2(x, t, t + s, K, "box") == d[s, t + S], (N, S, K, s, t)
    x = rng.normal(size=12) * 50
    d = pl.difference_lift_distances(x, 4, 3, "gauss", 1.5)
    for s in range(5):
        for t in range(-4, 12):
            ref = orc.patch_d2(x, t, t + s, 3, "gauss", 1.5)
            assert abs(ref - d[s, t + 4]) <= 1e-11 * max(1.0, ref), (s, t)


def check_patchlift_nlm(orc, seed: int = 3):
    """PatchLift-NLM (Alg. 2, symmetric pair weights) and direct NLM agree to
    rounding; on the setting of the paper's 1D experiment (sigma = 0.2, S = 10,
    K = 5, h = 1) their mean squared difference is of order 1e-17 or below."""
    rng = np.random.default_rng(seed)
    for kernel in ("box", "gauss"):
        x = rng.normal(size=40) * 30 + 100
        a = orc.nlm1d(x, 6, 2, 40.0, kernel)
        b = pl.patchlift_nlm1d(x, 6, 2, 40.0, kernel)
        assert np.max(np.abs(a - b)) <= 1e-11, kernel
    from paper_1407_2343_amd.synth import noisy_line
    x = noisy_line(400, 0.2, seed)
    a = orc.nlm1d(x, 10, 5, 1.0, "box")
    b = pl.patchlift_nlm1d(x, 10, 5, 1.0, "box")
    assert np.mean((a - b) ** 2) < 1e-17


def _img(seed, H=23, W=31):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(H, W)) * 25 + 120


def check_constant(orc):
    f = np.full((9, 14), 77.25)
    for kernel in ("box", "gauss"):
        for order in ("row_col", "col_row"):
            assert np.array_equal(orc.snlm(f, 3, 2, 10.0, kernel, order), f)


def check_h_inf_box_average(orc):
    """h = inf: all weights are 1, so each pass is a (2S+1)-tap moving average of
    the symmetric extension (scipy's 'reflect' mode is that extension)."""
    f = _img(1)
    for S in (1, 4):
        want = uniform_filter1d(uniform_filter1d(f, 2 * S + 1, axis=1, mode="reflect"),
                                2 * S + 1, axis=0, mode="reflect")
        got = orc.snlm(f, S, 2, math.inf, "box", "row_col")
        assert np.max(np.abs(got - want)) < 1e-10
        got = orc.snlm(f, S, 3, math.inf, "gauss", "col_row")
        want = uniform_filter1d(uniform_filter1d(f, 2 * S + 1, axis=0, mode="reflect"),
                                2 * S + 1, axis=1, mode="reflect")
        assert np.max(np.abs(got - want)) < 1e-10


def check_h_zero_identity(orc):
    f = _img(2)
    for kernel in ("box", "gauss"):
        got = orc.snlm(f, 4, 2, 1e-4, kernel, "row_col")
        assert np.max(np.abs(got - f)) < 1e-12


def check_s0_identity(orc):
    f = _img(3)
    assert np.array_equal(orc.snlm(f, 0, 3, 50.0, "box", "row_col"), f)


def check_flips(orc):
    f = _img(4)
    for kernel in ("box", "gauss"):
        base = orc.snlm(f, 4, 2, 60.0, kernel, "row_col")
        for ax in ((0,), (1,), (0, 1)):
            got = orc.snlm(np.flip(f, ax), 4, 2, 60.0, kernel, "row_col")
            assert np.max(np.abs(got - np.flip(base, ax))) < 1e-10, (kernel, ax)


def check_transpose(orc):
    f = _img(5)
    a = orc.snlm(f, 3, 2, 50.0, "gauss", "row_col")
    b = orc.snlm(f.T, 3, 2, 50.0, "gauss", "col_row").T
    assert np.array_equal(a, b)


def check_affine(orc):
    """NLM(a X + b; |a| h) = a NLM(X; h) + b, since d2 scales by a^2."""
    f = _img(6)
    for a_, b_ in ((2.5, -7.0), (-0.5, 3.0)):
        lhs = orc.snlm(a_ * f + b_, 3, 2, 55.0 * abs(a_), "box", "row_col")
        rhs = a_ * orc.snlm(f, 3, 2, 55.0, "box", "row_col") + b_
        assert np.max(np.abs(lhs - rhs)) < 1e-9


def check_k0_pixel_filter(orc):
    """K = 0: d2 = (x_i - x_j)^2, the neighbourhood (Yaroslavsky) filter."""
    rng = np.random.default_rng(8)
    x = rng.normal(size=30) * 20
    S, h = 4, 15.0
    idx = np.arange(-S, x.size + S)
    m = np.mod(idx, 2 * x.size)
    xe = x[np.where(m < x.size, m, 2 * x.size - 1 - m)]
    want = np.empty_like(x)
    for i in range(x.size):
        win = xe[i:i + 2 * S + 1]
        w = np.exp(-(x[i] - win) ** 2 / h ** 2)
        want[i] = np.sum(w * win) / np.sum(w)
    assert np.max(np.abs(orc.nlm1d(x, S, 0, h, "box") - want)) < 1e-12


def check_pixel_matches_full(orc):
    f = _img(9, 17, 12)
    for order in ("row_col", "col_row"):
        full = orc.snlm(f, 5, 2, 40.0, "gauss", order)
        for (r, c) in ((0, 0), (16, 11), (8, 3), (1, 10)):
            assert orc.pixel(f, r, c, 5, 2, 40.0, "gauss", order) == full[r, c]


# ---- SURE combination (Sec. 3.1, Alg. 3, Alg. 4) ----------------------------
def _fd_derivative(orc, x, i, S, K, h, kernel, eps):
    """Central difference of the 1D NLM output at i with respect to x(i)."""
    xp, xm = x.copy(), x.copy()
    xp[i] += eps
    xm[i] -= eps
    return (orc.nlm1d(xp, S, K, h, kernel)[i] - orc.nlm1d(xm, S, K, h, kernel)[i]) / (2 * eps)


def check_div_finite_difference(orc):
    """eq. div against the derivative taken numerically from eq. 1dNLM itself,
    at samples whose whole reach lies inside the line (no reflection)."""
    rng = np.random.default_rng(21)
    x = rng.normal(size=70) * 20 + 100
    for kernel, S, K, h in (("box", 5, 2, 30.0), ("gauss", 6, 3, 40.0), ("box", 3, 0, 12.0)):
        _, d = orc.nlm1d_div(x, S, K, h, kernel)
        for i in range(S + 2 * K, x.size - S - 2 * K, 7):
            fd = _fd_derivative(orc, x, i, S, K, h, kernel, 1e-4)
            assert abs(fd - d[i]) < 1e-7 * max(1.0, abs(d[i])), (kernel, i, fd, d[i])


def check_div_line_ends(orc):
    """eq. div at every sample, line ends included.  The formula differentiates
    with respect to x(i) alone and takes every other sample x(j), j != i, as a
    separate variable, even where the reflection maps j onto i.  That is the
    derivative of eq. 1dNLM on the explicitly extended line (NumPy's
    'symmetric' padding, the half-sample reflection) with only the centre copy
    of x(i) perturbed: the filter at an interior position of the padded array
    never reflects."""
    rng = np.random.default_rng(23)
    x = rng.normal(size=24) * 20 + 100
    for kernel, S, K, h in (("box", 5, 3, 35.0), ("gauss", 4, 3, 30.0), ("box", 2, 2, 25.0)):
        _, d = orc.nlm1d_div(x, S, K, h, kernel)
        R = S + K
        xe = np.pad(x, R, mode="symmetric")
        eps = 1e-4
        for i in list(range(0, R + 1)) + list(range(x.size - R - 1, x.size)):
            xp, xm = xe.copy(), xe.copy()
            xp[R + i] += eps
            xm[R + i] -= eps
            fd = (orc.nlm1d(xp, S, K, h, kernel)[R + i] - orc.nlm1d(xm, S, K, h, kernel)[R + i]) / (2 * eps)
            assert abs(fd - d[i]) < 1e-7 * max(1.0, abs(d[i])), (kernel, i, fd, d[i])


def check_div_limits(orc):
    """h = inf: y is a (2S+1)-tap average, whose derivative at the centre is
    1/(2S+1); a tiny h makes y the identity (derivative 1); the divergence is
    carried linearly through din."""
    rng = np.random.default_rng(22)
    x = rng.normal(size=40) * 30
    y, d = orc.nlm1d_div(x, 4, 2, math.inf, "box")
    assert np.max(np.abs(d - 1.0 / 9.0)) < 1e-15
    y, d = orc.nlm1d_div(x, 4, 2, 1e-3, "gauss")
    assert np.max(np.abs(y - x)) < 1e-12 and np.max(np.abs(d - 1.0)) < 1e-12
    din = rng.uniform(0.5, 2.0, size=x.size)
    _, d1 = orc.nlm1d_div(x, 4, 2, 25.0, "box")
    _, d2 = orc.nlm1d_div(x, 4, 2, 25.0, "box", din=din)
    assert np.max(np.abs(d2 - din * d1)) < 1e-14


def _sure_phi(f, r, sigma, th):
    """SURE of the combination (eq. sure with eq. linear), from its definition."""
    out = th[0] * r["f_rc"] + th[1] * r["f_cr"]
    n = f.size
    return (np.mean((out - f) ** 2) - sigma ** 2
            + 2 * sigma ** 2 / n * (th[0] * r["d_rc"].sum() + th[1] * r["d_cr"].sum()))


def check_sure_minimiser(orc):
    """theta from A theta = b (eqs. A, bb) is where the SURE of eq. sure, written
    out directly, is stationary, and it is a minimum."""
    f = _img(23, 29, 37)
    sigma = 20.0
    for kernel in ("box", "gauss"):
        r = orc.sure(f, 4, 2, 60.0, sigma, kernel)
        th = r["theta"]
        assert np.max(np.abs(r["out"] - (th[0] * r["f_rc"] + th[1] * r["f_cr"]))) < 1e-9
        e = 1e-4
        for k in range(2):
            tp, tm = th.copy(), th.copy()
            tp[k] += e
            tm[k] -= e
            g = (_sure_phi(f, r, sigma, tp) - _sure_phi(f, r, sigma, tm)) / (2 * e)
            assert abs(g) < 1e-6 * np.mean(f ** 2), (kernel, k, g)
        base = _sure_phi(f, r, sigma, th)
        for other in ((1.0, 0.0), (0.0, 1.0), (0.5, 0.5)):
            assert base <= _sure_phi(f, r, sigma, np.array(other)) + 1e-9


def check_sure_chain_and_orders(orc):
    """delta_rc is the product of the row-pass divergence of f and the
    column-pass divergence of the row-filtered image (eqs. partialrc,
    partialcr), and f_rc / f_cr are the two orders of Sec. 3."""
    f = _img(24, 19, 26)
    S, K, h = 3, 2, 45.0
    r = orc.sure(f, S, K, h, 10.0, "box")
    assert np.max(np.abs(r["f_rc"] - orc.snlm(f, S, K, h, "box", "row_col"))) < 1e-10
    assert np.max(np.abs(r["f_cr"] - orc.snlm(f, S, K, h, "box", "col_row"))) < 1e-10
    fr = np.empty_like(f)
    dr = np.empty_like(f)
    for i in range(f.shape[0]):
        fr[i], dr[i] = orc.nlm1d_div(f[i], S, K, h, "box")
    dc = np.empty_like(f)
    for j in range(f.shape[1]):
        _, dc[:, j] = orc.nlm1d_div(fr[:, j], S, K, h, "box")
    assert np.max(np.abs(r["d_rc"] - dr * dc)) < 1e-12


def check_sure_transpose(orc):
    """Transposing the image swaps the two orders, their divergences and theta."""
    f = _img(25, 21, 30)
    a = orc.sure(f, 3, 2, 50.0, 15.0, "gauss")
    b = orc.sure(f.T, 3, 2, 50.0, 15.0, "gauss")
    assert np.max(np.abs(a["f_rc"] - b["f_cr"].T)) < 1e-10
    assert np.max(np.abs(a["d_cr"] - b["d_rc"].T)) < 1e-12
    assert np.max(np.abs(a["theta"] - b["theta"][::-1])) < 1e-8


def check_sure_tracks_mse(orc):
    """With a known clean image and seeded Gaussian noise (eq. noise), the SURE
    combination is no worse than either order (within 1 %), and SURE stays
    close to the true MSE on average (it is unbiased up to the chain-rule
    approximation of eqs. partialrc / partialcr)."""
    from paper_1407_2343_amd.synth import clean_image
    rel = []
    for seed in (1, 2, 3):
        rng = np.random.default_rng(seed)
        f0 = clean_image(96, 96, rng).astype(np.float64)
        sigma = 20.0
        f = f0 + sigma * rng.standard_normal(f0.shape)
        r = orc.sure(f, 5, 2, 150.0, sigma, "box")
        mse = np.mean((r["out"] - f0) ** 2)
        best = min(np.mean((r["f_rc"] - f0) ** 2), np.mean((r["f_cr"] - f0) ** 2))
        assert mse <= 1.01 * best, (seed, mse, best)
        rel.append((_sure_phi(f, r, sigma, r["theta"]) - mse) / mse)
    assert abs(np.mean(rel)) < 0.1, rel


# ---- volumes ----------------------------------------------------------------
def _vol(seed, D=5, H=9, W=13):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(D, H, W)) * 25 + 120


def check_3d_box_average(orc):
    """h = inf: a (2S+1)-tap moving average along each axis (scipy's 'reflect'
    mode is the half-sample symmetric extension)."""
    f = _vol(41)
    want = f
    for ax in (2, 0, 1):  # axes "xzy"
        want = uniform_filter1d(want, 2 * 3 + 1, axis=ax, mode="reflect")
    got = orc.snlm3d(f, 3, 2, math.inf, "box", "xzy")
    assert np.max(np.abs(got - want)) < 1e-10


def check_3d_transpose_and_slices(orc):
    """Permuting the axes of the volume permutes the filtered volume when the
    pass order follows them; one slice (D = 1) is the 2D row_col filter, the
    z pass on a single sample being the identity."""
    f = _vol(42)
    a = orc.snlm3d(f, 3, 2, 40.0, "gauss", "xyz")
    # volume (z, y, x) -> (x, y, z): its x axis is the original z
    b = orc.snlm3d(np.ascontiguousarray(f.transpose(2, 1, 0)), 3, 2, 40.0, "gauss", "zyx")
    assert np.max(np.abs(a - b.transpose(2, 1, 0))) < 1e-10
    s = _vol(43, 1, 11, 14)
    got = orc.snlm3d(s, 4, 2, 35.0, "box", "xyz")[0]
    assert np.max(np.abs(got - orc.snlm(s[0], 4, 2, 35.0, "box", "row_col"))) < 1e-10
    c = np.full((3, 4, 6), -3.5)
    assert np.array_equal(orc.snlm3d(c, 2, 1, 10.0, "box", "zxy"), c)


# ---- bilateral post-processing (Sec. 3.2 eq. BF, Sec. 4.1 rules) -----------
def check_bf_rules(orc):
    for b in _parse_blocks(os.path.join(GOLDEN, "bilateral_rules.txt")):
        ss, sr = orc.bf_params(float(b["sigma"]))
        if "sigma_s" in b:
            want, tol = (float(v) for v in b["sigma_s"].split())
            assert abs(ss - want) <= tol, (b["case"], ss)
        want, tol = (float(v) for v in b["sigma_r"].split())
        assert abs(sr - want) <= tol, (b["case"], sr)


def check_bf_gaussian_limit(orc):
    """sigma_r = inf: a normalised Gaussian blur over the truncated square,
    which is scipy's gaussian_filter with the same radius in 'reflect' mode."""
    from scipy.ndimage import gaussian_filter
    f = _img(31, 20, 27)
    for ss in (0.7, 1.0):  # radius floor(3 ss) = round(3 ss) for these
        got = orc.bilateral(f, ss, math.inf)
        want = gaussian_filter(f, ss, mode="reflect", truncate=3.0)
        assert np.max(np.abs(got - want)) < 1e-10, ss


def check_bf_limits_and_invariants(orc):
    f = _img(32, 18, 23)
    # a tiny range width keeps every pixel (distinct values)
    assert np.max(np.abs(orc.bilateral(f, 1.0, 1e-6) - f)) < 1e-12
    c = np.full((7, 9), 42.5)
    assert np.array_equal(orc.bilateral(c, 0.9, 30.0), c)
    base = orc.bilateral(f, 1.2, 40.0)
    for ax in ((0,), (1,), (0, 1)):
        assert np.max(np.abs(orc.bilateral(np.flip(f, ax), 1.2, 40.0) - np.flip(base, ax))) < 1e-10
    # range kernel on differences: BF(a f + b; |a| sigma_r) = a BF(f; sigma_r) + b
    assert np.max(np.abs(orc.bilateral(-2.0 * f + 5.0, 1.2, 80.0) - (-2.0 * base + 5.0))) < 1e-9
    # sigma_s below 1/3: only the centre tap
    assert np.array_equal(orc.bilateral(f, 0.3, 40.0), f)


# ---- recursive Gaussian patch kernel (Young & van Vliet, cited in Sec. 2.2) ----
def _yvv_poles(beta):
    # The published q(sigma) fit and the cubic of the filter's denominator,
    # b0 z^3 - b1 z^2 - b2 z - b3, whose roots are the causal poles.
    q = 0.98711 * beta - 0.96330 if beta >= 2.5 else 3.97156 - 4.14554 * math.sqrt(1 - 0.26891 * beta)
    b0 = 1.57825 + 2.44413 * q + 1.4281 * q * q + 0.422205 * q ** 3
    b1 = 2.44413 * q + 2.85619 * q * q + 1.26661 * q ** 3
    b2 = -(1.4281 * q * q + 1.26661 * q ** 3)
    b3 = 0.422205 * q ** 3
    return np.roots([b0, -b1, -b2, -b3])


def check_iir_filter(orc):
    """The forward-backward recursion against its closed forms: unit gain
    (constants and, away from the ends, ramps pass unchanged), a symmetric
    impulse response whose variance is the poles' 2 sum p / (1 - p)^2 (a causal
    cascade of geometric responses, run forward and backward), and a shape
    within the approximation error of the sampled Gaussian."""
    for beta in (0.5, 1.0, 2.0, 3.0, 8.0):
        c = orc.yvv(np.full(64, -3.25), beta)
        assert np.max(np.abs(c + 3.25)) < 1e-12, beta
        n, mid = 1201, 600
        imp = np.zeros(n)
        imp[mid] = 1.0
        r = orc.yvv(imp, beta)
        k = np.arange(n) - mid
        assert np.max(np.abs(r - r[::-1])) < 1e-12, beta
        assert abs(r.sum() - 1.0) < 1e-10, beta
        p = _yvv_poles(beta)
        var = 2.0 * float(np.sum(p / (1 - p) ** 2).real)
        assert abs(float(np.sum(r * k * k)) - var) < 1e-8 * var, (beta, var)
        g = np.exp(-k * k / (2 * beta * beta))
        g /= g.sum()
        assert np.max(np.abs(r - g)) < (0.06 if beta >= 2 else 0.10) * g.max(), beta
        ramp = 0.75 * np.arange(n) - 40.0
        rr = orc.yvv(ramp, beta)
        assert np.max(np.abs(rr[300:900] - ramp[300:900])) < 1e-9, beta


def check_iir_distances(orc, seed: int = 21):
    """Distances of the recursive kernel: on a ramp of slope a, away from the
    ends, every lifted difference is a^2 s^2 and the distance is sqrt(2 pi) beta
    a^2 s^2 (the untruncated Gaussian's mass times it); on a noisy line they
    stay within the approximation error of the exact FIR distance with the
    kernel's tails kept (K = 6 beta), and the 1D NLM built on them stays
    much closer to the exact Gaussian NLM than the box NLM is."""
    n = 400
    for beta in (1.0, 3.0):
        a = -1.7
        x = a * np.arange(n) + 12.0
        d = orc.iir_d2(x, 5, beta)
        for s in range(1, 6):
            want = math.sqrt(2 * math.pi) * beta * a * a * s * s
            got = d[s - 1, 5 + 150:5 + 250]
            assert np.max(np.abs(got - want)) < 1e-9 * want, (beta, s)
    rng = np.random.default_rng(seed)
    n = 160
    t = np.arange(n)
    x = 100.0 * np.sin(t / 9.0) + 20.0 * rng.standard_normal(n)
    for beta, S, tol in ((1.0, 4, 0.12), (2.0, 6, 0.05), (4.0, 3, 0.04)):
        K = int(math.ceil(6 * beta))
        d = orc.iir_d2(x, S, beta)
        ref = np.array([[orc.patch_d2(x, u, u + s, K, "gauss", beta) for u in range(-S, n)]
                        for s in range(1, S + 1)])
        assert np.max(np.abs(d - ref)) < tol * ref.max(), beta
        h = 150.0 * math.sqrt(beta)
        yi = orc.nlm1d(x, S, 0, h, "gauss_iir", beta)
        yf = orc.nlm1d(x, S, K, h, "gauss", beta)
        yb = orc.nlm1d(x, S, K, h, "box")
        assert np.max(np.abs(yi - yf)) < 0.2 * np.max(np.abs(yf - yb)), beta
    # h = inf: the window mean, whatever the distances; S = 0: identity
    assert np.max(np.abs(orc.nlm1d(x, 3, 0, math.inf, "gauss_iir", 2.0)
                         - uniform_filter1d(x, 7, mode="reflect"))) < 1e-10
    assert np.array_equal(orc.nlm1d(x, 0, 0, 50.0, "gauss_iir", 2.0), x)


ALL_CHECKS = [
    check_worked_examples_1d, check_separable_2x2, check_alg1_distances,
    check_difference_lift, check_patchlift_nlm, check_constant, check_h_inf_box_average,
    check_h_zero_identity, check_s0_identity, check_flips, check_transpose, check_affine,
    check_k0_pixel_filter, check_pixel_matches_full, check_div_finite_difference,
    check_div_line_ends, check_div_limits, check_sure_minimiser, check_sure_chain_and_orders, check_sure_transpose,
    check_sure_tracks_mse, check_bf_rules, check_bf_gaussian_limit, check_bf_limits_and_invariants,
    check_3d_box_average, check_3d_transpose_and_slices, check_iir_filter, check_iir_distances,
]
