"""Oracle for the full Stage I search (test infrastructure only).

The paper's Stage I (Sec. 2.4) on a standardised residual cube r[c][y][x] (the SNR cube of the
width-1 detector: unit-variance noise, spectral median removed):

1. Matched filtering across frequency with unit-normalised boxcars of 1 to 100 fine channels,
   densely sampled at the narrowest widths and coarser towards 100.  Reading of the width set
   (the paper gives only its shape): 1..10 in steps of 1, 12..48 in steps of 4, 50..100 in steps
   of 10 (26 widths).  "Unit-normalised" is read as unit energy, so unit-variance white noise
   gives unit-variance filtered output:
       S_w[c] = (1/sqrt(w)) * sum_{j=0}^{w-1} r[c - floor(w/2) + j],
   evaluated only where the window lies inside the band.  When the channels of the noise are
   correlated (rho_l = correlation at a lag of l channels, l = 1..L), unit-normalised is read
   as unit variance under that correlation: the window sum is divided by
       sigma_w = sqrt(w + 2 sum_{l=1}^{min(w-1, L)} (w - l) rho_l)
   (the standard deviation of a sum of w consecutive unit-variance samples), which is sqrt(w)
   for white noise.  The paper does not say how its SNRs treat the correlation that its window
   puts between adjacent fine channels; without it the bank's noise is not unit-normal.
2. For every pixel and channel the highest SNR over the widths and its width are kept (on ties
   the narrower width).
3. SNR -> p-value under the standardised (unit normal) noise model, one-sided:
   p = Q(S) = erfc(S / sqrt 2) / 2.  Benjamini-Hochberg at level q over all m searched voxels
   (in-horizon pixels x channels): k* = max{k : p_(k) <= k q / m}; the voxels with the k*
   smallest p-values (equivalently the k* largest S) are provisional detections; none if no k.
   The BH decision threshold in SNR units is S* = the k*-th largest S.  Every one of the m
   in-horizon voxels takes part in the step-up comparison.
4. Non-maximum suppression along frequency at each pixel: a provisional detection survives if no
   other provisional detection at that pixel within its exclusion region, of half-width
   max(floor(w/2), 1) channels around its channel, has a higher SNR (on ties the lower channel
   survives).
5. Local re-evaluation (reading: the baseline is re-estimated from the flanks next to the
   detection and the SNR recomputed against it): with the detection's window [s, s + w),
   s = c - floor(w/2), guard g = w and flank length L = max(16, 2 w), the flanks
   [s - g - L, s - g) and [s + w + g, s + w + g + L) inside the band give a baseline b (median)
   and noise sigma = 1.482602218505602 * MAD; the re-evaluated SNR is
   sum_{window}(r - b) / (sigma_w sigma).  The detection is kept when that is >= S*; with
   fewer than 8 flank channels or sigma = 0 it is discarded.

Medians of even counts are the mean of the two central order statistics.  Output records
(x, y, c, width, snr = the matched-filter S) sorted by (y, x, c).
"""
from __future__ import annotations

import math

import numpy as np

from .detect import MAD_K, horizon_mask, median_even_mean

WIDTHS = tuple(list(range(1, 11)) + list(range(12, 49, 4)) + list(range(50, 101, 10)))

# Channel correlations of the imaged cube's noise.  The periodic Hann window is the three-tap
# kernel (-1/4, 1/2, -1/4) over the bins of the unwindowed spectrum, so windowed white noise has
# correlation (-1/4 * 1/2 + 1/2 * -1/4) / (1/16 + 1/4 + 1/16) = -2/3 at a lag of one channel and
# (1/16) / (3/8) = 1/6 at two; a cross-correlation product of two independent inputs then has
# the squared magnitudes, 4/9 and 1/36, and so do the images built from such products.
HANN_CROSS_RHO = (4.0 / 9.0, 1.0 / 36.0)
REEVAL_MIN_FLANK = 8


def boxcar_sigma(w: int, rho=()) -> float:
    """Standard deviation of the sum of w consecutive unit-variance samples whose correlation at
    a lag of l channels is rho[l - 1] (zero beyond len(rho)): sqrt(w) for white noise."""
    var = float(w)
    for l in range(1, min(w - 1, len(rho)) + 1):
        var += 2.0 * (w - l) * float(rho[l - 1])
    return math.sqrt(var)


def boxcar_bank(r: np.ndarray, widths=WIDTHS, rho=()) -> tuple[np.ndarray, np.ndarray]:
    """(S, W): highest unit-variance boxcar SNR over the widths and its width, for r [C][...]
    (noise channel correlations rho, see boxcar_sigma)."""
    r = np.asarray(r, dtype=np.float64)
    n_chan = r.shape[0]
    flat = r.reshape(n_chan, -1)
    best = np.full(flat.shape, -np.inf)
    wbest = np.zeros(flat.shape, dtype=np.int32)
    for w in sorted(widths):
        h = w // 2
        c0, c1 = h, n_chan - w + h           # channels whose window [c - h, c - h + w) fits
        if c1 < c0:
            continue
        sw = np.zeros((c1 - c0 + 1, flat.shape[1]))
        for j in range(w):                   # the window sum, term by term
            sw += flat[c0 - h + j:c1 - h + j + 1]
        sw /= boxcar_sigma(w, rho)
        upd = sw > best[c0:c1 + 1]           # strict: the narrower width wins ties
        best[c0:c1 + 1][upd] = sw[upd]
        wbest[c0:c1 + 1][upd] = w
    return best.reshape(r.shape), wbest.reshape(r.shape)


def q_value(s) -> np.ndarray:
    """One-sided standard-normal tail Q(S) = erfc(S / sqrt 2) / 2 (libm erfc, float64)."""
    s = np.asarray(s, dtype=np.float64)
    return np.vectorize(lambda v: 0.5 * math.erfc(v / math.sqrt(2.0)), otypes=[np.float64])(s)


def bh_threshold(s_values: np.ndarray, m: int, q: float) -> tuple[int, float]:
    """(k*, S*) of Benjamini-Hochberg at level q over m tests whose SNRs include s_values (every
    voxel not listed has a lower SNR than all listed ones and is never rejected); (0, inf) when
    nothing is rejected."""
    s = np.sort(np.asarray(s_values, dtype=np.float64))[::-1]     # descending SNR = ascending p
    if s.size == 0:
        return 0, math.inf
    p = q_value(s)
    k = np.arange(1, s.size + 1, dtype=np.float64)
    ok = np.flatnonzero(p <= k * q / m)
    if ok.size == 0:
        return 0, math.inf
    kstar = int(ok[-1]) + 1
    return kstar, float(s[kstar - 1])


def nms(S: np.ndarray, W: np.ndarray, accepted: np.ndarray) -> np.ndarray:
    """Survivors of the width-aware non-maximum suppression along axis 0 of [C][P] arrays."""
    n_chan = S.shape[0]
    keep = accepted.copy()
    half = np.maximum(W // 2, 1)
    for d in range(1, int(half[accepted].max(initial=1)) + 1):
        reach = accepted & (half >= d)
        # neighbour below (c - d): beats c when higher, or equal (the lower channel wins ties)
        lo = np.zeros_like(keep)
        lo[d:] = accepted[:-d] & (S[:-d] >= S[d:])
        # neighbour above (c + d): beats c only when strictly higher
        hi = np.zeros_like(keep)
        hi[:-d] = accepted[d:] & (S[d:] > S[:-d])
        keep &= ~(reach & (lo | hi))
    return keep


def reevaluate(r_pix: np.ndarray, c: int, w: int, rho=()) -> float:
    """Re-evaluated SNR of a detection at channel c with width w in one pixel's spectrum."""
    n_chan = r_pix.shape[0]
    s = c - w // 2
    g, L = w, max(16, 2 * w)
    idx = [j for j in range(s - g - L, s - g) if 0 <= j < n_chan]
    idx += [j for j in range(s + w + g, s + w + g + L) if 0 <= j < n_chan]
    if len(idx) < REEVAL_MIN_FLANK:
        return -math.inf
    flank = r_pix[idx]
    b = float(median_even_mean(flank, axis=0))
    mad = float(median_even_mean(np.abs(flank - b), axis=0))
    if mad <= 0.0:
        return -math.inf
    return float(np.sum(r_pix[s:s + w] - b) / (boxcar_sigma(w, rho) * MAD_K * mad))


def search(r: np.ndarray, q: float = 0.01, widths=WIDTHS, valid: np.ndarray | None = None, rho=()):
    """Stage I over r [C][N][N]: (records, S, W, k*, S*).  valid [N][N] marks searched pixels
    (default: the visible hemisphere); rho the noise's channel correlations (white: empty)."""
    r = np.asarray(r, dtype=np.float64)
    n_chan, n_pix, _ = r.shape
    if valid is None:
        valid = horizon_mask(n_pix)
    S, W = boxcar_bank(r, widths, rho)
    Sv = S[:, valid]
    m = int(valid.sum()) * n_chan
    kstar, sstar = bh_threshold(Sv.ravel(), m, q)
    flatS, flatW = S.reshape(n_chan, -1), W.reshape(n_chan, -1)
    acc = (flatS >= sstar) & valid.ravel()[None, :]
    surv = nms(flatS, flatW, acc)
    c_idx, p_idx = np.nonzero(surv)
    keep = []
    rf = r.reshape(n_chan, -1)
    for c, p in zip(c_idx, p_idx):
        keep.append(reevaluate(rf[:, p], int(c), int(flatW[c, p]), rho) >= sstar)
    keep = np.asarray(keep, dtype=bool)
    c_idx, p_idx = c_idx[keep], p_idx[keep]
    y, x = p_idx // n_pix, p_idx % n_pix
    order = np.lexsort((c_idx, x, y))
    rec = np.zeros(len(order), dtype=[("x", np.int32), ("y", np.int32), ("c", np.int32),
                                      ("width", np.int32), ("snr", np.float64)])
    rec["x"], rec["y"], rec["c"] = x[order], y[order], c_idx[order]
    rec["width"] = flatW[c_idx[order], p_idx[order]]
    rec["snr"] = flatS[c_idx[order], p_idx[order]]
    return rec, S, W, kstar, sstar
