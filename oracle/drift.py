"""Oracle for the drift-rate search (test infrastructure only).

The paper's Doppler-drift discussion (Sec. 2, "Doppler drift") leaves drift correction to future
work and asks for a modest drift search, at least tens of Hz over the 30 s dump, for
transmitters on close-in planets.  Reading used here: the dump is split into S
sub-integrations, each channelised, correlated, imaged and standardised on its own (the same
hot path with fewer spectra per integration), giving residual cubes r_s[c][y][x].  A line that
starts at channel c and drifts by d channels over the dump sits at c + shift(d, s) in
sub-integration s, shift(d, s) = round(d s / (S - 1)) with halves rounded away from zero
(shift = 0 when S = 1).  Its de-Dopplered SNR is the unit-energy sum
    D_d[c] = (1 / sqrt(S)) * sum_s r_s[c + shift(d, s)],
defined when the whole track lies in the band (0 <= c + d < C, the shift being monotone in s).
Drift trials are the integers -D..D; per voxel the largest D_d and its drift are kept, trials
visited in the order 0, -1, +1, -2, +2, ... with a strict comparison (ties keep the smaller
|d|, then the negative one).
"""
from __future__ import annotations

import math

import numpy as np


def shift(d: int, s: int, n_sub: int) -> int:
    """round(d s / (n_sub - 1)) with halves away from zero, in integer arithmetic."""
    if n_sub <= 1 or d == 0 or s == 0:
        return 0
    num, den = 2 * abs(d) * s + (n_sub - 1), 2 * (n_sub - 1)
    mag = num // den
    return mag if d > 0 else -mag


def trial_order(max_drift: int) -> list[int]:
    out = [0]
    for k in range(1, max_drift + 1):
        out += [-k, k]
    return out


def dedoppler(r_sub: np.ndarray, max_drift: int) -> tuple[np.ndarray, np.ndarray]:
    """(best, drift): r_sub [S][C][...] -> highest de-Dopplered SNR per voxel [C][...] and its
    total drift in channels (0 where no trial fits, with best = -inf)."""
    r = np.asarray(r_sub, dtype=np.float64)
    n_sub, n_chan = r.shape[0], r.shape[1]
    flat = r.reshape(n_sub, n_chan, -1)
    best = np.full(flat.shape[1:], -np.inf)
    drift = np.zeros(flat.shape[1:], dtype=np.int32)
    for d in trial_order(max_drift):
        c_lo, c_hi = max(0, -d), min(n_chan, n_chan - d)      # 0 <= c + d < C
        if c_hi <= c_lo:
            continue
        acc = np.zeros((c_hi - c_lo, flat.shape[2]))
        for s in range(n_sub):                                 # the track, sub-integration by sub-integration
            k = shift(d, s, n_sub)
            acc += flat[s, c_lo + k:c_hi + k]
        acc /= math.sqrt(n_sub)
        upd = acc > best[c_lo:c_hi]
        best[c_lo:c_hi][upd] = acc[upd]
        drift[c_lo:c_hi][upd] = d
    return best.reshape(r.shape[1:]), drift.reshape(r.shape[1:])
