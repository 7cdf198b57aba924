"""Independent lifted computations of patch distances, used to pin the oracle.

The oracle computes every patch distance literally from eq. distanceSquared.
The two routines here reach the same numbers by the other route the paper
describes, PatchLift (Sec. 2.1-2.2), so that a dropped tap, a wrong index or a
wrong sign in either shows up as a mismatch:

* ``alg1_distances`` computes what Alg. 1 and eq. dist compute: the products
  f(i)f(j) of the band B sit at the positions eq. packing_1 gives them in the
  packed sequence (subdiagonals with K zeros between them), the sequence is
  filtered with the patch kernel, and d2 is read off as Vbar(l_ii) + Vbar(l_jj)
  - 2 Vbar(l_ij) (eqs. lift and dist).  Samples outside [1, N] do not exist in this layout,
  which amounts to zero extension of the signal.
* ``difference_lift_distances`` lifts each offset-s diagonal as
  (x(t) - x(t+s))^2 on the reflected extension and sums it over the patch with
  prefix sums (box, the recursion of eq. recursion) or an explicit FIR
  (Gaussian).

Both are written in float64 NumPy for tiny inputs; neither touches the oracle.
"""
from __future__ import annotations

import numpy as np


def kernel_taps(K: int, kernel: str, beta: float | None) -> np.ndarray:
    """g(k) for k = -K..K: box ones, or exp(-k^2/(2 beta^2)) with g(0) = 1."""
    k = np.arange(-K, K + 1, dtype=np.float64)
    if kernel == "box" or K == 0:
        return np.ones(2 * K + 1)
    b = K / 2.0 if beta is None else beta
    return np.exp(-k * k / (2.0 * b * b))


def packed_length(N: int, S: int, K: int) -> int:
    """Length L of V stated under eq. packing_1."""
    num = (S + 1) * (2 * N - S) + 2 * K * S
    assert num % 2 == 0
    return num // 2


def l_index(i: int, j: int, N: int, S: int, K: int) -> int:
    """1-based position of F(i, j), i >= j, in V (eq. packing_1)."""
    num = (S - i + j) * (2 * N + 2 * K - S - 1 - i + j)
    assert num % 2 == 0
    return num // 2 + j


def band(N: int, S: int):
    """The band B of Sec. 2.1 (eq. band): 1-based pairs (i, j), i >= j,
    i - j <= S, both inside [1, N]."""
    return [(j + d, j) for d in range(S + 1) for j in range(1, N - d + 1)]


def alg1_vbar(f1: np.ndarray, S: int, K: int, g: np.ndarray):
    """The packed sequence V of Sec. 2.2 and its filtered version Vbar = V * g.

    Each product F(i, j) = f(i) f(j) of the band B is written at the position
    eq. packing_1 assigns to it; every other position of the length-L sequence
    (the K-sample gaps between subdiagonals) stays zero.  ``f1`` is the signal;
    returns (V, Vbar, positions) with V/Vbar 1-based (index 0 unused) and
    positions[(i, j)] = l."""
    N = f1.size
    L = packed_length(N, S, K)
    V = np.zeros(L + 1)
    pos = {}
    for (i, j) in band(N, S):
        l = l_index(i, j, N, S, K)
        V[l] = f1[i - 1] * f1[j - 1]
        pos[(i, j)] = l
    # Vbar(t) = sum_k g(k) V(t + k), V zero outside [1, L]: entry t - 1 + K
    # of the full convolution of V(1..L) with the reversed taps
    Vbar = np.zeros_like(V)
    Vbar[1:] = np.convolve(V[1:], g[::-1])[K:K + L]
    return V, Vbar, pos


def alg1_distances(x: np.ndarray, S: int, K: int, kernel: str = "box", beta=None) -> dict:
    """d2 for all in-range pairs with |i-j| <= S via Alg. 1 + eq. dist,
    keyed by 0-based (i, j)."""
    N = x.size
    g = kernel_taps(K, kernel, beta)
    _, Vbar, _ = alg1_vbar(np.asarray(x, dtype=np.float64), S, K, g)
    d = {}
    for i in range(1, N + 1):
        for j in range(max(1, i - S), min(N, i + S) + 1):
            a, b = (i, j) if i >= j else (j, i)
            lii = l_index(i, i, N, S, K)
            ljj = l_index(j, j, N, S, K)
            lij = l_index(a, b, N, S, K)
            d[(i - 1, j - 1)] = Vbar[lii] + Vbar[ljj] - 2.0 * Vbar[lij]
    return d


def _refl(t: np.ndarray, n: int) -> np.ndarray:
    m = np.mod(t, 2 * n)
    return np.where(m < n, m, 2 * n - 1 - m)


def difference_lift_distances(x: np.ndarray, S: int, K: int, kernel: str = "box",
                              beta=None) -> np.ndarray:
    """d2[s, t] = d2(t, t+s) for s in 0..S, t in [-S, N) on the reflected
    extension, via the difference lift and prefix sums (box) or an FIR (Gauss)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.size
    g = kernel_taps(K, kernel, beta)
    lo, hi = -S - K - 1, N + K  # lifted samples needed: v in [lo, hi)
    v = np.arange(lo, hi)
    out = np.zeros((S + 1, N + S))
    t = np.arange(-S, N)
    for s in range(S + 1):
        D = (x[_refl(v, N)] - x[_refl(v + s, N)]) ** 2  # lifted diagonal, offset s
        if kernel == "box":
            C = np.cumsum(D)  # C[m] = sum D[0..m]
            # window sum over v in [t-K, t+K] = C(t+K) - C(t-K-1)
            out[s] = C[t + K - lo] - C[t - K - 1 - lo]
        else:
            acc = np.zeros(t.size)
            for k in range(-K, K + 1):
                acc += g[k + K] * D[t + k - lo]
            out[s] = acc
    return out


def patchlift_nlm1d(x: np.ndarray, S: int, K: int, h: float, kernel: str = "box",
                    beta=None) -> np.ndarray:
    """Alg. 2 (PatchLift-NLM) on the reflected extension, using the
    difference-lift distances; each unordered pair's weight is used for both
    centres (the symmetry of the band B)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.size
    d = difference_lift_distances(x, S, K, kernel, beta)  # d[s, t + S]
    y = np.empty(N)
    for i in range(N):
        P, Q = 0.0, 0.0
        for s in range(-S, S + 1):
            u = i if s >= 0 else i + s  # pair (u, u+|s|)
            d2 = d[abs(s), u + S]
            w = 1.0 if d2 == 0 else np.exp(-d2 / (h * h))
            P += w * x[_refl(np.array(i + s), N)]
            Q += w
        y[i] = P / Q
    return y
