"""Pins of the drift-rate search oracle (oracle/drift.py): the rounding rule by hand, brute
force on small inputs, a drifting line's closed form, and white-noise variance (no GPU)."""
import math

import numpy as np
import pytest

from oracle import drift as odr


def test_shift_rule_by_hand():
    # S = 5 sub-integrations (4 steps): d = 3 -> 0, 0.75, 1.5, 2.25, 3 -> 0, 1, 2, 2, 3
    assert [odr.shift(3, s, 5) for s in range(5)] == [0, 1, 2, 2, 3]
    assert [odr.shift(-3, s, 5) for s in range(5)] == [0, -1, -2, -2, -3]
    # S = 3 (2 steps): d = 1 -> 0, 0.5, 1 -> halves away from zero: 0, 1, 1 and 0, -1, -1
    assert [odr.shift(1, s, 3) for s in range(3)] == [0, 1, 1]
    assert [odr.shift(-1, s, 3) for s in range(3)] == [0, -1, -1]
    assert all(odr.shift(d, s, 1) == 0 for d in range(-3, 4) for s in range(1))
    assert odr.trial_order(2) == [0, -1, 1, -2, 2]


def test_brute_force_small():
    rng = np.random.default_rng(2)
    S, C, P, D = 4, 30, 3, 5
    r = rng.standard_normal((S, C, P))
    best, drift = odr.dedoppler(r, D)
    for c in range(C):
        for p in range(P):
            bv, bd = -math.inf, 0
            for d in odr.trial_order(D):
                if not (0 <= c + d < C):
                    continue
                tot = 0.0
                for s in range(S):
                    k = c + odr.shift(d, s, S)
                    assert 0 <= k < C
                    tot += float(r[s, k, p])
                v = tot / math.sqrt(S)
                if v > bv:
                    bv, bd = v, d
            assert best[c, p] == pytest.approx(bv, abs=1e-12) and drift[c, p] == bd


@pytest.mark.parametrize("d0", [-7, -2, 0, 3, 9])
def test_drifting_line_closed_form(d0):
    # a unit line along the track of drift d0 starting at channel 40, zero elsewhere:
    # D_d0[40] = S / sqrt(S) = sqrt(S), the maximum over all voxels and trials
    S, C = 6, 100
    r = np.zeros((S, C, 1))
    for s in range(S):
        r[s, 40 + odr.shift(d0, s, S), 0] = 1.0
    best, drift = odr.dedoppler(r, 10)
    assert best[40, 0] == pytest.approx(math.sqrt(S), rel=1e-12)
    assert drift[40, 0] == d0
    assert best.max() == pytest.approx(math.sqrt(S), rel=1e-12)


def test_unit_variance_per_trial_on_white_noise():
    rng = np.random.default_rng(8)
    r = rng.standard_normal((8, 300, 400))
    for d in (0, -5, 12):
        # a single trial: the channels valid for it, that trial alone
        S, C = 8, 300
        lo, hi = max(0, -d), min(C, C - d)
        acc = sum(r[s, lo + odr.shift(d, s, S):hi + odr.shift(d, s, S)] for s in range(S)) / math.sqrt(S)
        assert np.var(acc) == pytest.approx(1.0, abs=0.02)
