"""The FP64 oracle against hand-derived values, the PatchLift identity computed
another way, and invariants (see oracle_pin_checks.py)."""
import pytest

import oracle_pin_checks as pc
import patchlift_ref as pl


@pytest.mark.parametrize("check", pc.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(oracle_mod, check):
    check(oracle_mod.load())


def test_packed_length_matches_alg1_layout():
    # Length of V stated under eq. packing_1: L = (S+1)(N - S/2) + K S, e.g.
    # N=8, S=2, K=1 gives 23.
    assert pl.packed_length(8, 2, 1) == 23
    for (N, S, K) in [(8, 2, 1), (13, 4, 3), (20, 5, 2), (6, 5, 0)]:
        import numpy as np
        _, _, pos = pl.alg1_vbar(np.arange(1.0, N + 1), S, K, np.ones(2 * K + 1))
        assert max(pos.values()) == pl.packed_length(N, S, K)
        for (i, j), l in pos.items():
            assert pl.l_index(i, j, N, S, K) == l
