"""Pins of the oracle detector (Sec. 2.4, Stage I with the width-1 matched filter)."""
import numpy as np
import pytest

from oracle import detect as D


def _cube_with_spectrum(spec, n_pix=8, x=4, y=4, base=None):
    C = len(spec)
    rng = np.random.default_rng(0)
    cube = rng.standard_normal((C, n_pix, n_pix)) if base is None else base.copy()
    cube[:, y, x] = spec
    return cube


def test_median_even_count_is_mean_of_central_pair():
    a = np.array([[4.0, 1.0, 3.0, 2.0], [1.0, 1.0, 5.0, 9.0]])
    np.testing.assert_allclose(D.median_even_mean(a, axis=1), [2.5, 3.0])
    np.testing.assert_allclose(D.median_even_mean(np.array([[3.0, 1.0, 2.0]]), axis=1), [2.0])


def test_mad_constant_normalises_gaussian_noise():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(2_000_000)
    mad = D.median_even_mean(np.abs(x - D.median_even_mean(x[None], 1)[0])[None], 1)[0]
    assert abs(D.MAD_K * mad - 1.0) < 0.003
    # 1/Phi^-1(3/4)
    from scipy.stats import norm
    assert abs(D.MAD_K - 1.0 / norm.ppf(0.75)) < 1e-14


def test_hand_computed_spike_snr():
    # sorted spectrum [-1,-1,-1,1,1,1,1,11]: median = (1 + 1)/2 = 1;
    # |x - 1| sorted [0,0,0,0,2,2,2,10]: MAD = (0 + 2)/2 = 1; spike SNR = (11 - 1)/k
    spec = np.array([1, -1, 1, -1, 1, -1, 1, 11], float)
    rec, snr, valid = D.detect(_cube_with_spectrum(spec), tau=5.0)
    mine = rec[(rec["x"] == 4) & (rec["y"] == 4)]
    assert len(mine) == 1 and mine["c"][0] == 7
    assert abs(mine["snr"][0] - 10 / D.MAD_K) < 1e-12
    np.testing.assert_allclose(snr[:, 4, 4], (spec - 1) / D.MAD_K)


def test_nms_plateau_keeps_lower_channel_and_chain_keeps_top():
    spec = np.zeros(16)
    spec[::2] = 1
    spec[1::2] = -1
    spec[5] = spec[6] = 20           # plateau -> channel 5
    spec[10], spec[11], spec[12] = 12, 15, 18   # rising chain -> channel 12
    rec, snr, _ = D.detect(_cube_with_spectrum(spec), tau=5.0)
    mine = rec[(rec["x"] == 4) & (rec["y"] == 4)]
    assert list(mine["c"]) == [5, 12]


def test_horizon_mask_integer_rule():
    m = D.horizon_mask(8)
    assert m[4, 4] and m[4, 1] and not m[4, 0] and not m[0, 0] and not m[0, 4]
    assert m.sum() == sum(1 for y in range(8) for x in range(8) if (x - 4) ** 2 + (y - 4) ** 2 < 16)


def test_zero_mad_pixel_gives_nothing():
    spec = np.zeros(10)
    spec[3] = 100.0
    rec, _, valid = D.detect(_cube_with_spectrum(spec), tau=5.0)
    assert not valid[4, 4]
    assert len(rec[(rec["x"] == 4) & (rec["y"] == 4)]) == 0


def test_gaussian_noise_false_positive_rate():
    # P(z >= 5) = 2.87e-7; over ~0.8M searchable voxels we expect ~0.2 false positives.
    rng = np.random.default_rng(7)
    cube = rng.standard_normal((4096, 16, 16))
    rec, snr, valid = D.detect(cube, tau=5.0)
    assert len(rec) <= 4
    s = snr[:, valid]
    assert abs(s.std() - 1.0) < 0.01


def test_per_image_mode_recovers_weak_spike():
    rng = np.random.default_rng(3)
    cube = rng.standard_normal((256, 16, 16))
    cube[100, 6, 9] += 8.0
    for mode in ("per_pixel", "per_image"):
        rec, snr, _ = D.detect(cube, tau=5.0, mode=mode)
        hit = rec[(rec["x"] == 9) & (rec["y"] == 6) & (rec["c"] == 100)]
        assert len(hit) == 1 and 6.5 < hit["snr"][0] < 9.5


def test_records_sorted_by_y_x_c():
    rng = np.random.default_rng(4)
    cube = rng.standard_normal((64, 16, 16))
    for (c, y, x) in [(10, 9, 3), (5, 3, 9), (40, 3, 9), (7, 3, 4)]:
        cube[c, y, x] += 30
    rec, _, _ = D.detect(cube, tau=5.0)
    keys = list(zip(rec["y"], rec["x"], rec["c"]))
    assert keys == sorted(keys)
    assert {(3, 4, 7), (3, 9, 5), (3, 9, 40), (9, 3, 10)} <= set(keys)


def test_per_image_mode_hand_computed():
    # A 4 x 4 image has nine pixels in the visible hemisphere, the 3 x 3 block x, y in {1, 2, 3}.
    # Channel c holds m_c + s_c v there, with v = -4..4 in raster order over the block (channel 2
    # reversed); so each channel's in-horizon median is m_c and its MAD 2 s_c, and
    # z = v / (2k) in channels 0 and 1 and -v / (2k) in channel 2.  Per pixel the median of z over
    # the three channels is v / (2k), so the standardised residual is (0, 0, -v / k).
    # A huge value at the below-horizon pixel (0, 0) changes nothing; had it entered the
    # per-image statistics, every median would move.  Had the per-pixel spectral median not
    # been removed, channels 0 and 1 would keep v / (2k).
    k = D.MAD_K
    v = np.arange(-4.0, 5.0).reshape(3, 3)
    m_c, s_c = (10.0, -5.0, 100.0), (1.0, 3.0, 0.5)
    cube = np.zeros((3, 4, 4))
    for c in range(3):
        vc = v if c < 2 else v[::-1, ::-1]
        cube[c, 1:4, 1:4] = m_c[c] + s_c[c] * vc
    cube[:, 0, 0] = 1e6
    rec, snr, valid = D.detect(cube, tau=2.5, mode="per_image")
    expect = np.zeros((3, 4, 4))
    expect[2, 1:4, 1:4] = -v / k
    np.testing.assert_allclose(snr, expect, atol=1e-12)
    assert valid.sum() == 9 and not valid[0, 0]
    # only v = -4 (pixel (1, 1)) reaches 4 / k = 2.698 >= 2.5, in channel 2
    assert [(int(a["x"]), int(a["y"]), int(a["c"])) for a in rec] == [(1, 1, 2)]
    assert rec["snr"][0] == pytest.approx(4.0 / k, rel=1e-12)


def test_non_finite_pixels_are_not_searched():
    # the cube of the per-image hand case with channel 0 of the centre pixel (v = 0) not finite:
    # that pixel is not searched, and channel 0's statistics come from its 8 finite in-horizon
    # pixels, v = -4..-1, 1..4: median 0, MAD 2.5, so z = v / (2.5 k) there; channels 1 and 2
    # keep v / (2k) and -v / (2k).  Per pixel the median over channels is v / (2.5 k), so the
    # standardised residual is (0, v (1/2 - 1/2.5) / k, -v (1/2 + 1/2.5) / k)
    k = D.MAD_K
    v = np.arange(-4.0, 5.0).reshape(3, 3)
    cube = np.zeros((3, 4, 4))
    for c, (m_c, s_c) in enumerate([(10.0, 1.0), (-5.0, 3.0), (100.0, 0.5)]):
        cube[c, 1:4, 1:4] = m_c + s_c * (v if c < 2 else v[::-1, ::-1])
    for bad in (np.nan, np.inf, -np.inf):
        cube[0, 2, 2] = bad
        rec, snr, valid = D.detect(cube, tau=100.0, mode="per_image")
        expect = np.zeros((3, 4, 4))
        expect[1, 1:4, 1:4] = v * (0.5 - 0.4) / k
        expect[2, 1:4, 1:4] = -v * (0.5 + 0.4) / k
        expect[:, 2, 2] = 0.0
        np.testing.assert_allclose(snr, expect, atol=1e-12)
        assert valid.sum() == 8 and not valid[2, 2]
    # per pixel: every other pixel is scored exactly as in the cube without that value
    rng = np.random.default_rng(6)
    noisy = rng.standard_normal((64, 16, 16))
    noisy[20, 7, 9] += 40.0
    ref_rec, ref_snr, _ = D.detect(noisy, tau=5.0)
    hit = noisy.copy()
    hit[33, 8, 8] = np.nan
    rec, snr, valid = D.detect(hit, tau=5.0)
    assert not valid[8, 8] and (snr[:, 8, 8] == 0).all()
    keep = np.ones((16, 16), bool)
    keep[8, 8] = False
    np.testing.assert_array_equal(snr[:, keep], ref_snr[:, keep])
    assert [tuple(r) for r in rec] == [tuple(r) for r in ref_rec if not (r["x"] == 8 and r["y"] == 8)]
