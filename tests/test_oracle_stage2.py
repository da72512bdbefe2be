"""Pins of the Stage II oracle (Sec. 2.4 automated cuts, Gaussian centroid fits) against closed
forms, an independently parametrised generator, finite differences and Monte Carlo statistics."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
import oracle
from oracle import stage2 as s2

K = 2.0 * math.sqrt(2.0 * math.log(2.0))


def _cut(img, x, y, h=s2.HALF):
    return img[y - h:y + h + 1, x - h:x + h + 1]


@pytest.mark.parametrize("dx,dy,smaj,smin,th", [(0.3, -0.2, 1.6, 1.2, 0.5), (0.0, 0.0, 1.5, 1.5, 0.0),
                                               (-0.45, 0.4, 2.0, 1.0, 0.0), (0.1, 0.35, 2.2, 1.1, math.pi / 2),
                                               (0.2, 0.1, 1.8, 0.9, 2.6)])
def test_noise_free_blob_recovered(dx, dy, smaj, smin, th):
    """A blob drawn from (sigma_maj, sigma_min, rotation) plus a constant background is fitted
    exactly: amplitude, centroid, FWHM = 2 sqrt(2 ln 2) sigma along both axes, position angle."""
    img = synth.elliptical_blob(41, 20 + dx, 20 + dy, 7.5, smaj, smin, th) + 0.25
    f = s2.fit(_cut(img, 20, 20), 1.0)
    A, x0, y0, a, b, c, B = f["p"]
    assert f["ok"] and f["rss"] < 1e-20
    assert abs(A - 7.5) < 1e-9 and abs(B - 0.25) < 1e-9
    assert abs(x0 - dx) < 1e-9 and abs(y0 - dy) < 1e-9
    assert abs(f["fwhm_maj"] - K * smaj) < 1e-8 and abs(f["fwhm_min"] - K * smin) < 1e-8
    if smaj != smin:
        d = (f["pa"] - th) % math.pi
        assert min(d, math.pi - d) < 1e-8


def test_shape_closed_forms():
    # circular: both FWHM = K sigma
    maj, mnr, _ = s2.shape(1 / 4.0, 0.0, 1 / 4.0)
    assert maj == pytest.approx(2 * K) and mnr == pytest.approx(2 * K)
    # axis-aligned, wider along y: major along +y (angle pi/2)
    maj, mnr, pa = s2.shape(1.0, 0.0, 0.25)
    assert maj == pytest.approx(2 * K) and mnr == pytest.approx(K) and pa == pytest.approx(math.pi / 2)
    # wider along x
    maj, mnr, pa = s2.shape(0.25, 0.0, 1.0)
    assert maj == pytest.approx(2 * K) and pa == pytest.approx(0.0)
    # not positive definite
    assert math.isnan(s2.shape(1.0, 2.0, 1.0)[0])


def test_solution_is_stationary():
    """At the returned parameters the finite-difference gradient of the residual sum of squares
    vanishes (a wrong Jacobian term would stop MINPACK elsewhere) and the RSS is a minimum."""
    rng = np.random.default_rng(5)
    img = synth.elliptical_blob(41, 20.3, 19.8, 9.0, 1.7, 1.1, 0.8) + rng.standard_normal((41, 41))
    cut = _cut(img, 20, 20)
    f = s2.fit(cut, 1.4)
    xx, yy = np.meshgrid(np.arange(-4, 5.0), np.arange(-4, 5.0))

    def rss(p):
        A, x0, y0, a, b, c, B = p
        u, v = xx - x0, yy - y0
        return float(np.sum((B + A * np.exp(-0.5 * (a * u * u + 2 * b * u * v + c * v * v)) - cut) ** 2))

    p = f["p"]
    assert rss(p) == pytest.approx(f["rss"], rel=1e-12)
    for i in range(7):
        h = 1e-6 * max(1.0, abs(p[i]))
        e = np.zeros(7)
        e[i] = h
        g = (rss(p + e) - rss(p - e)) / (2 * h)
        assert abs(g) < 1e-4
        assert rss(p + 100 * e) > f["rss"] and rss(p - 100 * e) > f["rss"]


def test_covariance_errors_match_scatter():
    """Over noise realisations the scatter of the fitted centroid and amplitude matches the
    reported errors (covariance x RSS / (n - 7)), and RSS / (n - 7) averages the noise variance."""
    rng = np.random.default_rng(11)
    clean = synth.elliptical_blob(41, 20.2, 19.7, 10.0, 1.6, 1.2, 0.5)
    xs, amps, ex, ea, chi = [], [], [], [], []
    for _ in range(300):
        f = s2.fit(_cut(clean + rng.standard_normal((41, 41)), 20, 20), 1.4)
        assert f["ok"]
        xs.append(f["p"][1])
        amps.append(f["p"][0])
        ex.append(f["err"][1])
        ea.append(f["err"][0])
        chi.append(f["rss"] / f["dof"])
    assert 0.85 < np.std(xs) / np.median(ex) < 1.15
    assert 0.85 < np.std(amps) / np.median(ea) < 1.15
    assert 0.95 < np.mean(chi) < 1.05
    assert abs(np.mean(xs) - 0.2) < 3 * np.std(xs) / math.sqrt(len(xs))


def test_absorption_fails_fit():
    img = 0.5 - synth.elliptical_blob(41, 20.0, 20.0, 6.0, 1.5, 1.5, 0.0)
    assert not s2.fit(_cut(img, 20, 20), 1.0)["ok"]


def test_beam_of_gaussian_psf():
    psf = synth.elliptical_blob(64, 32, 32, 1.0, 1.3, 0.9, 1.1)
    maj, mnr, pa = s2.beam(psf)
    assert maj == pytest.approx(K * 1.3, rel=1e-9) and mnr == pytest.approx(K * 0.9, rel=1e-9)
    assert pa == pytest.approx(1.1, abs=1e-9)


def _psf_centre(xyz, freq, n_pix):
    n_in = 2 * xyz.shape[0]
    vis = np.zeros((len(freq), n_in * (n_in + 1) // 2, 2))
    vis[..., 0] = 1.0
    h = n_pix // 2
    pix = np.array([(x, y) for y in range(h - 2, h + 3) for x in range(h - 2, h + 3)])
    vals = oracle.image_dft_pixels(vis, xyz, freq, n_pix, pix, grid_n_pix=n_pix)
    out = np.zeros((len(freq), n_pix, n_pix))
    for c in range(len(freq)):
        out[c, pix[:, 1], pix[:, 0]] = vals[c]
    return out


def test_beam_of_array_orientation_and_frequency():
    """An array twice as long east-west (x) as north-south has a beam twice as narrow in l:
    major axis along m (position angle pi/2), axis ratio near 2; the beam shrinks as 1/nu."""
    xyz = synth.antenna_layout(128, 60.0, 3)
    xyz[:, 0] *= 2.0
    nu = 60.0e6
    psf = _psf_centre(xyz, np.array([nu, 1.3 * nu]), 512)
    b0, b1 = s2.beam(psf[0]), s2.beam(psf[1])
    assert abs(b0[2] - math.pi / 2) < 0.1 and abs(b1[2] - math.pi / 2) < 0.1
    assert 1.7 < b0[0] / b0[1] < 2.3
    assert 1.3 * 0.97 < b0[0] / b1[0] < 1.3 * 1.03 and 1.3 * 0.97 < b0[1] / b1[1] < 1.3 * 1.03


def test_channel_noise_and_flags():
    rng = np.random.default_rng(2)
    cube, _ = synth.stage2_scene(rng, 12, 128, n_point=0, n_ext=0, noisy=(3, -8))
    sig = s2.channel_noise(cube)
    want = np.ones(12)
    want[3], want[7] = 3.0, 0.3
    np.testing.assert_allclose(sig, want, rtol=0.04)
    cands = [{"x": 40, "y": 50, "c": c} for c in range(12)]
    res = s2.stage2(cube, cands, (3.0, 3.0, 0.0))
    noisy = [bool(r["flags"] & s2.NOISY_CHANNEL) for r in res]
    assert noisy == [c in (3, 7) for c in range(12)]


def test_stage2_scene():
    """Beam-shaped blobs are kept with centroids within their errors; blobs 2.5-4 times the
    beam are rejected as extended; candidates whose cutout leaves the image are flagged."""
    rng = np.random.default_rng(8)
    bs = (1.6, 1.2, 0.5)
    cube, blobs = synth.stage2_scene(rng, 16, 96, beam_sigma=bs, n_point=20, n_ext=8)
    beam = (K * bs[0], K * bs[1], bs[2])
    cands = [{"x": int(round(b.x)), "y": int(round(b.y)), "c": b.c} for b in blobs]
    cands += [{"x": 2, "y": 40, "c": 0}, {"x": 50, "y": 93, "c": 1}]
    res = s2.stage2(cube, cands, beam)
    pulls = []
    for b, r in zip(blobs, res):
        if b.extended:
            assert r["flags"] & s2.EXTENDED
        else:
            assert r["flags"] == 0
            f = r["fit"]
            pulls += [(f["x0"] - b.x) / f["err"][1], (f["y0"] - b.y) / f["err"][2]]
            assert 0.5 < f["chi2_red"] < 1.6
    assert max(abs(p) for p in pulls) < 4.5
    assert 0.6 < np.std(pulls) < 1.4
    assert res[-2]["flags"] & s2.EDGE and res[-1]["flags"] & s2.EDGE


def test_errors_equal_curve_fit_covariance():
    """The 1-sigma errors equal the square roots of SciPy curve_fit's covariance diagonal
    (absolute_sigma=False: inverse normal matrix scaled by RSS / (n - p), computed by curve_fit
    from MINPACK's factorisation)."""
    from scipy.optimize import curve_fit
    rng = np.random.default_rng(21)
    img = synth.elliptical_blob(41, 20.1, 20.3, 6.0, 1.5, 1.0, 2.2) + 0.7 * rng.standard_normal((41, 41))
    cut = _cut(img, 20, 20)
    f = s2.fit(cut, 1.2)
    xx, yy = np.meshgrid(np.arange(-4, 5.0), np.arange(-4, 5.0))

    def g(xy, A, x0, y0, a, b, c, B):
        u, v = xy[0] - x0, xy[1] - y0
        return B + A * np.exp(-0.5 * (a * u * u + 2 * b * u * v + c * v * v))

    popt, pcov = curve_fit(g, np.stack([xx.ravel(), yy.ravel()]), cut.ravel(), p0=f["p"], method="lm")
    np.testing.assert_allclose(popt, f["p"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(np.sqrt(np.diag(pcov)), f["err"], rtol=1e-5)


def test_channel_noise_ignores_pixels_below_horizon():
    rng = np.random.default_rng(4)
    cube, _ = synth.stage2_scene(rng, 4, 64, n_point=0, n_ext=0)
    mask = oracle.detect.horizon_mask(64)
    blank = cube.copy()
    blank[:, ~mask] = 0.0
    np.testing.assert_array_equal(s2.channel_noise(cube), s2.channel_noise(blank))
