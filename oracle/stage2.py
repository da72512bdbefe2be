"""Oracle for the Stage II automated cuts (test infrastructure only).

The paper's Stage II (Sec. 2.4) keeps candidates consistent with narrowband point sources:
detections with extended morphology are rejected, images whose noise deviates from
expectations are flagged, and candidate positions come from Gaussian centroid fits with 1-sigma
errors from the fit covariance rescaled by sqrt(reduced chi-square).  Readings used here:

* Fit: the (2h+1) x (2h+1) cutout of the candidate's channel image around its pixel (h = 4;
  h = 2 for the synthesized-beam fit), model f = B + A exp(-Q/2) with
  Q = a dx^2 + 2 b dx dy + c dy^2, dx = x - x0, dy = y - y0 (seven parameters, Q positive
  definite), least squares with unit weights started from A = peak - B, (x0, y0) = the pixel,
  a = c = 1/sigma^2 (sigma from the beam's FWHM, or 1 pixel), b = 0, B = the median of the
  cutout's border ring.  The minimiser is SciPy's MINPACK Levenberg-Marquardt.
* Errors: cov = (J^T J)^-1 RSS / (n - 7) at the solution; with weights 1/sigma^2 the scaling by
  chi^2_red = RSS / (sigma^2 (n - 7)) gives exactly this, whatever sigma.  chi^2_red itself is
  reported with sigma = the channel image's 1.4826 MAD.
* Shape: FWHM = 2 sqrt(2 ln 2) / sqrt(eigenvalue) of [[a, b], [b, c]], major from the smaller
  eigenvalue; position angle of the major axis from the +x axis, in [0, pi).
* Synthesized beam: the fit (h = 2) to the point-spread function (the image of unit
  visibilities) at the image centre.
* Cuts (flags): fit failed (no positive-definite Q or A <= 0) 1; extended, either FWHM above
  ext_factor (1.5) times the beam's 2; the channel's image noise (1.4826 MAD over the visible
  hemisphere) outside [median / k, k * median] over channels, k = 1.5, 4; cutout not inside the
  image (or channel outside the cube, then alone) 8.  A candidate is kept when no flag is set.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import least_squares

from .detect import MAD_K, horizon_mask, median_even_mean

FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))
HALF = 4
BEAM_HALF = 2
EXT_FACTOR = 1.5
NOISE_K = 1.5
FIT_FAILED, EXTENDED, NOISY_CHANNEL, EDGE = 1, 2, 4, 8


def _grid(h):
    yy, xx = np.mgrid[-h:h + 1, -h:h + 1]
    return xx.astype(np.float64), yy.astype(np.float64)


def model(p, xx, yy):
    A, x0, y0, a, b, c, B = p
    dx, dy = xx - x0, yy - y0
    return B + A * np.exp(-0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy))


def jacobian(p, xx, yy):
    A, x0, y0, a, b, c, B = p
    dx, dy = xx - x0, yy - y0
    E = np.exp(-0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy))
    return np.stack([E.ravel(), (A * E * (a * dx + b * dy)).ravel(), (A * E * (b * dx + c * dy)).ravel(),
                     (-0.5 * A * E * dx * dx).ravel(), (-A * E * dx * dy).ravel(), (-0.5 * A * E * dy * dy).ravel(),
                     np.ones(dx.size)], axis=1)


def initial(cut, sigma):
    n = cut.shape[0]
    ring = np.concatenate([cut[0, :], cut[-1, :], cut[1:-1, 0], cut[1:-1, -1]])
    B = float(median_even_mean(ring, axis=0))
    h = n // 2
    return np.array([cut[h, h] - B, 0.0, 0.0, 1.0 / sigma ** 2, 0.0, 1.0 / sigma ** 2, B])


def shape(a, b, c):
    """(FWHM major, FWHM minor, position angle of the major axis in [0, pi))."""
    tr, det = a + c, a * c - b * b
    disc = math.sqrt(max(0.0, 0.25 * (a - c) ** 2 + b * b))
    l_small, l_big = 0.5 * tr - disc, 0.5 * tr + disc
    if l_small <= 0.0 or det <= 0.0:
        return math.nan, math.nan, math.nan
    # eigenvector of the smaller eigenvalue: (b, l_small - a) or (l_small - c, b)
    vx, vy = (b, l_small - a) if abs(b) + abs(l_small - a) >= abs(l_small - c) + abs(b) else (l_small - c, b)
    pa = math.atan2(vy, vx) % math.pi
    return FWHM_PER_SIGMA / math.sqrt(l_small), FWHM_PER_SIGMA / math.sqrt(l_big), pa


def fit(cut: np.ndarray, sigma: float):
    """Least-squares Gaussian fit of a square cutout centred on its middle pixel: dict with the
    parameters (offsets relative to the middle pixel), errors and RSS."""
    cut = np.asarray(cut, dtype=np.float64)
    h = cut.shape[0] // 2
    xx, yy = _grid(h)
    p0 = initial(cut, sigma)
    res = least_squares(lambda p: (model(p, xx, yy) - cut).ravel(), p0,
                        jac=lambda p: jacobian(p, xx, yy), method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15,
                        max_nfev=2000)
    p = res.x
    J = jacobian(p, xx, yy)
    rss = float(np.sum((model(p, xx, yy) - cut) ** 2))
    dof = cut.size - 7
    ok = p[0] > 0.0 and p[3] > 0.0 and p[5] > 0.0 and p[3] * p[5] - p[4] ** 2 > 0.0
    err = np.full(7, math.nan)
    if ok:
        try:
            cov = np.linalg.inv(J.T @ J) * rss / dof
            err = np.sqrt(np.maximum(np.diag(cov), 0.0))
        except np.linalg.LinAlgError:
            ok = False
    maj, mnr, pa = shape(p[3], p[4], p[5]) if ok else (math.nan,) * 3
    return {"p": p, "ok": ok, "rss": rss, "dof": dof, "err": err, "fwhm_maj": maj, "fwhm_min": mnr, "pa": pa}


def beam(psf: np.ndarray):
    """Synthesized beam (FWHM major, minor in pixels, position angle) from a point-spread
    function image [N][N] with its peak at the centre pixel."""
    n = psf.shape[0]
    h = n // 2
    f = fit(psf[h - BEAM_HALF:h + BEAM_HALF + 1, h - BEAM_HALF:h + BEAM_HALF + 1], 1.0)
    return f["fwhm_maj"], f["fwhm_min"], f["pa"]


def channel_noise(img: np.ndarray) -> np.ndarray:
    """1.4826 MAD of every channel image over the visible hemisphere."""
    img = np.asarray(img, dtype=np.float64)
    mask = horizon_mask(img.shape[1])
    vals = img[:, mask]
    med = median_even_mean(vals, axis=1)
    return MAD_K * median_even_mean(np.abs(vals - med[:, None]), axis=1)


def stage2(img: np.ndarray, cands, beam_fwhm, ext_factor: float = EXT_FACTOR, noise_k: float = NOISE_K,
           half: int = HALF):
    """Flags and fits for candidate records (fields x, y, c) on image cube img [C][N][N];
    beam_fwhm is one (major, minor, position angle) triple or one per channel [C][3]."""
    img = np.asarray(img, dtype=np.float64)
    n_chan, n_pix, _ = img.shape
    bm = np.asarray(beam_fwhm, dtype=np.float64)
    if bm.ndim == 1:
        bm = np.broadcast_to(bm, (n_chan, 3))
    sig = channel_noise(img)
    med = float(median_even_mean(sig, axis=0))
    out = []
    for r in cands:
        x, y, c = int(r["x"]), int(r["y"]), int(r["c"])
        if not 0 <= c < n_chan:                     # no such channel: only the outside flag
            out.append({"flags": EDGE, "fit": None})
            continue
        bmaj, bmin = float(bm[c, 0]), float(bm[c, 1])
        sigma0 = bmaj / FWHM_PER_SIGMA if math.isfinite(bmaj) and bmaj > 0 else 1.0
        flags = 0
        if not (med / noise_k <= sig[c] <= noise_k * med):
            flags |= NOISY_CHANNEL
        if x < half or y < half or x + half >= n_pix or y + half >= n_pix:
            out.append({"flags": flags | EDGE, "fit": None})
            continue
        f = fit(img[c, y - half:y + half + 1, x - half:x + half + 1], sigma0)
        if not f["ok"]:
            flags |= FIT_FAILED
        elif f["fwhm_maj"] > ext_factor * bmaj or f["fwhm_min"] > ext_factor * bmin:
            flags |= EXTENDED
        f["chi2_red"] = f["rss"] / (sig[c] ** 2 * f["dof"]) if sig[c] > 0 else math.inf
        f["x0"], f["y0"] = x + f["p"][1], y + f["p"][2]
        out.append({"flags": flags, "fit": f})
    return out
