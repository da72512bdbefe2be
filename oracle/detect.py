"""Oracle for the narrowband detection pass (test infrastructure only).

Follows the paper's Stage I (Sec. 2.4) reduced to the width-1 matched filter:

1. Noise model.  The paper standardises every channel image by its median absolute
   deviation (MAD) so the maps have about unit variance, then removes broad spectral
   structure by subtracting a running median along frequency at each pixel, with a window
   wider than 5 kHz.  Every configured band here is narrower than that window, so the
   running median is the median of the whole spectrum of the pixel.
   Two modes:
   * "per_pixel": SNR_p[c] = (I_p[c] - med_c I_p) / (k * MAD_c I_p)   (the default)
   * "per_image": z = (I - med) / (k * MAD) over the in-horizon pixels of each channel image,
                  then SNR_p[c] = z_p[c] - med_c z_p.
   k = 1 / Phi^-1(3/4) = 1.482602218505602 makes k * MAD the standard deviation of Gaussian
   noise.  The median of an even count is the mean of the two central order statistics.
2. Width-1 boxcar: the unit-normalised boxcar of one channel is the SNR itself.
3. Threshold: a voxel is a provisional detection when SNR >= tau.
4. Non-maximum suppression along frequency (Sec. 2.4): a detection survives when it has the
   highest SNR within its exclusion region of half-width max(floor(w/2), 1) = 1 channel;
   on ties the lower channel survives.
5. Only pixels inside the visible hemisphere, l^2 + m^2 < 1, are searched; with
   l = (x - N/2) 2/N this is the integer test (x - N/2)^2 + (y - N/2)^2 < (N/2)^2.
   Pixels whose MAD is zero give no detections.
6. Non-finite input (reading; the paper's images are finite): a pixel whose spectrum holds a
   non-finite value cannot be standardised and is not searched, like a pixel below the
   horizon; in per_image mode each channel's statistics use its finite in-horizon pixels.

Output: records (x, y, c, snr, width) sorted by (y, x, c).
"""
from __future__ import annotations

import numpy as np

MAD_K = 1.482602218505602


def horizon_mask(n_pix: int) -> np.ndarray:
    y, x = np.mgrid[0:n_pix, 0:n_pix]
    h = n_pix // 2
    return (x - h) ** 2 + (y - h) ** 2 < h * h


def median_even_mean(a: np.ndarray, axis: int) -> np.ndarray:
    """Median along an axis; for an even count, the mean of the two central order statistics."""
    s = np.sort(a, axis=axis)
    n = a.shape[axis]
    lo = np.take(s, (n - 1) // 2, axis=axis)
    hi = np.take(s, n // 2, axis=axis)
    return 0.5 * (lo + hi)


def per_pixel_snr(flat: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """SNR of spectra flat [C][P] under the per-pixel noise model, and the pixels with MAD > 0."""
    med = median_even_mean(flat, axis=0)                  # per pixel
    mad = median_even_mean(np.abs(flat - med[None, :]), axis=0)
    good = mad > 0
    snr = np.zeros_like(flat)
    snr[:, good] = (flat[:, good] - med[None, good]) / (MAD_K * mad[None, good])
    return snr, good


def snr_cube(cube: np.ndarray, mode: str = "per_pixel") -> tuple[np.ndarray, np.ndarray]:
    """SNR for every voxel of cube [C][N][N] (float64) and the boolean searchable-pixel mask."""
    cube = np.asarray(cube, dtype=np.float64)
    n_chan, n_pix, _ = cube.shape
    mask = horizon_mask(n_pix)
    flat = cube.reshape(n_chan, -1)[:, mask.ravel()]          # [C][P_in]
    fin = np.isfinite(flat)
    fin_pix = fin.all(axis=0)                                 # searchable: whole spectrum finite
    if mode == "per_pixel":
        snr = np.zeros_like(flat)
        snr[:, fin_pix], good = per_pixel_snr(flat[:, fin_pix])
        good_all = np.zeros(flat.shape[1], dtype=bool)
        good_all[fin_pix] = good
        good = good_all
    elif mode == "per_image":
        z = np.zeros_like(flat)
        for c in range(n_chan):                               # per channel image, finite pixels
            vals = flat[c, fin[c]]
            if vals.size == 0:
                continue
            med_c = float(median_even_mean(vals, axis=0))
            mad_c = float(median_even_mean(np.abs(vals - med_c), axis=0))
            if mad_c > 0:
                z[c, fin[c]] = (vals - med_c) / (MAD_K * mad_c)
        snr = np.zeros_like(flat)
        zf = z[:, fin_pix]
        snr[:, fin_pix] = zf - median_even_mean(zf, axis=0)[None, :]
        good = fin_pix
    else:
        raise ValueError(mode)
    out = np.zeros((n_chan, n_pix * n_pix), dtype=np.float64)
    idx = np.flatnonzero(mask.ravel())
    out[:, idx[good]] = snr[:, good]
    valid = np.zeros(n_pix * n_pix, dtype=bool)
    valid[idx[good]] = True
    return out.reshape(n_chan, n_pix, n_pix), valid.reshape(n_pix, n_pix)


def nms_keep(snr: np.ndarray, tau: float) -> np.ndarray:
    """Boolean [C][...] of surviving detections (threshold + width-1 NMS, ties -> lower channel)."""
    keep = snr >= tau
    prev_lower = np.ones_like(keep)
    prev_lower[1:] = snr[1:] > snr[:-1]          # strictly above the lower neighbour
    next_not_higher = np.ones_like(keep)
    next_not_higher[:-1] = snr[:-1] >= snr[1:]   # not below the upper neighbour
    return keep & prev_lower & next_not_higher


def detect(cube: np.ndarray, tau: float = 5.0, mode: str = "per_pixel"):
    """Candidate records sorted by (y, x, c): structured array with x, y, c, snr, width."""
    snr, valid = snr_cube(cube, mode)
    keep = nms_keep(snr, tau) & valid[None, :, :]
    c, y, x = np.nonzero(keep)
    order = np.lexsort((c, x, y))
    rec = np.zeros(len(c), dtype=[("x", np.int32), ("y", np.int32), ("c", np.int32),
                                  ("snr", np.float64), ("width", np.int32)])
    rec["x"] = x[order]
    rec["y"] = y[order]
    rec["c"] = c[order]
    rec["snr"] = snr[c[order], y[order], x[order]]
    rec["width"] = 1
    return rec, snr, valid
