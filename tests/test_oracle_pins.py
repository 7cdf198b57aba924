"""The FP64 oracle against hand-derived values, the PatchLift identity computed
another way, and invariants (see oracle_pin_checks.py)."""
import numpy as np
import pytest

import oracle_pin_checks as pc
import patchlift_ref as pl


@pytest.mark.parametrize("check", pc.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(oracle_mod, check):
    check(oracle_mod.load())


@pytest.mark.parametrize("N,S,K", [(8, 2, 1), (13, 4, 3), (20, 5, 2), (6, 5, 0), (7, 0, 2)])
def test_packing_layout(N, S, K):
    """eq. packing_1 lays the band out as Sec. 2.2 describes it: the
    subdiagonals stacked farthest first (mu = 1 is i - j = S, eq.
    correspondence), each one contiguous, with exactly K zeros between
    successive ones, and the last sample (i = j = N) at L = (S+1)(N - S/2) + K S
    (N = 8, S = 2, K = 1 gives 23).  The simplified formula also equals the
    unsimplified sum it comes from."""
    if (N, S, K) == (8, 2, 1):
        assert pl.packed_length(N, S, K) == 23
    L = pl.packed_length(N, S, K)
    pos = {(i, j): pl.l_index(i, j, N, S, K) for (i, j) in pl.band(N, S)}
    assert len(set(pos.values())) == len(pos)
    assert min(pos.values()) == 1 and max(pos.values()) == L == pos[(N, N)]
    runs = []
    for d in range(S, -1, -1):  # farthest subdiagonal first
        ls = [pos[(j + d, j)] for j in range(1, N - d + 1)]
        assert ls == list(range(ls[0], ls[0] + len(ls))), d  # contiguous, in nu order
        runs.append((ls[0], ls[-1]))
    for (a0, a1), (b0, b1) in zip(runs, runs[1:]):
        assert b0 - a1 - 1 == K  # the zero gap between successive subdiagonals
    holes = set(range(1, L + 1)) - set(pos.values())
    assert len(holes) == K * S
    for (i, j), l in pos.items():
        mu, nu = S + 1 - i + j, j  # eq. correspondence
        assert l == (mu - 1) * K + sum(N - S - 1 + t for t in range(1, mu)) + nu
    V, _, _ = pl.alg1_vbar(np.arange(1.0, N + 1), S, K, np.ones(2 * K + 1))
    for (i, j), l in pos.items():
        assert V[l] == i * j
    assert all(V[t] == 0.0 for t in holes)
