"""Pins of the full Stage I search oracle (oracle/search.py) against closed forms, brute force,
SciPy's Benjamini-Hochberg routine and hand-worked cases (no GPU)."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
from oracle import search as osr

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_width_set():
    w = osr.WIDTHS
    assert w[:10] == tuple(range(1, 11)) and w[-1] == 100 and len(w) == 26
    assert all(b > a for a, b in zip(w, w[1:]))


@pytest.mark.parametrize("w0", [1, 7, 16, 60])
def test_boxcar_rectangular_pulse_closed_form(w0):
    # a rectangular pulse of amplitude A over [p0, p0 + w0) on zero background: the unit-energy
    # boxcar peaks at A sqrt(w0) with width w0, centred at p0 + floor(w0 / 2)
    n_chan, p0, A = 300, 110, 3.0
    r = np.zeros((n_chan, 1))
    r[p0:p0 + w0, 0] = A
    S, W = osr.boxcar_bank(r)
    c = int(np.argmax(S[:, 0]))
    assert c == p0 + w0 // 2
    assert W[c, 0] == w0
    assert S[c, 0] == pytest.approx(A * math.sqrt(w0), rel=1e-12)
    # a wider window over the whole pulse gives A w0 / sqrt(w) < A sqrt(w0)
    wide = [w for w in osr.WIDTHS if w > w0][0]
    assert A * w0 / math.sqrt(wide) < S[c, 0]


def test_boxcar_brute_force_small():
    rng = np.random.default_rng(3)
    n_chan, widths = 40, (1, 2, 3, 5, 8)
    r = rng.standard_normal((n_chan, 3))
    S, W = osr.boxcar_bank(r, widths)
    for p in range(3):
        for c in range(n_chan):
            best, bw = -math.inf, 0
            for w in widths:
                s = c - w // 2
                if s < 0 or s + w > n_chan:
                    continue
                tot = 0.0
                for j in range(w):
                    tot += float(r[s + j, p])
                v = tot / math.sqrt(w)
                if v > best:
                    best, bw = v, w
            assert S[c, p] == pytest.approx(best, abs=1e-12)
            assert W[c, p] == bw


def test_boxcar_edges_use_fitting_widths_only():
    n_chan = 30
    r = np.ones((n_chan, 1))
    S, W = osr.boxcar_bank(r)
    # at channel 0 only width 1 fits (a wider window would start before the band)
    assert W[0, 0] == 1 and S[0, 0] == 1.0
    # in the middle the widest fitting width wins on a constant spectrum (S = sqrt(w))
    assert W[15, 0] == 30 or W[15, 0] == max(w for w in osr.WIDTHS if w <= 30)


def test_boxcar_unit_variance_on_white_noise():
    rng = np.random.default_rng(11)
    r = rng.standard_normal((400, 500))
    for w in (1, 5, 24, 100):
        S, _ = osr.boxcar_bank(r, (w,))
        h = w // 2
        vals = S[h:400 - w + h + 1].ravel()
        assert np.var(vals) == pytest.approx(1.0, abs=0.03)


def test_q_value_closed_forms():
    assert osr.q_value(0.0) == pytest.approx(0.5, abs=1e-15)
    assert osr.q_value(scipy.stats.norm.isf(0.025)) == pytest.approx(0.025, rel=1e-12)
    assert osr.q_value(8.0) == pytest.approx(scipy.stats.norm.sf(8.0), rel=1e-10)


@pytest.mark.parametrize("q", [0.01, 0.05, 0.2])
def test_bh_matches_scipy(q):
    rng = np.random.default_rng(int(q * 1000))
    s = np.concatenate([rng.standard_normal(3000), rng.uniform(3.0, 6.0, 60)])
    kstar, sstar = osr.bh_threshold(s, s.size, q)
    adj = scipy.stats.false_discovery_control(osr.q_value(s), method="bh")
    rej_scipy = adj <= q
    rej = s >= sstar
    assert rej.sum() == kstar == rej_scipy.sum()
    np.testing.assert_array_equal(rej, rej_scipy)


def test_bh_on_the_top_values_only():
    rng = np.random.default_rng(5)
    s = np.concatenate([rng.standard_normal(20000), rng.uniform(4.0, 7.0, 40)])
    full = osr.bh_threshold(s, s.size, 0.05)
    top = np.sort(s)[-500:]
    assert osr.bh_threshold(top, s.size, 0.05) == full
    assert osr.bh_threshold(rng.standard_normal(100), 10 ** 9, 0.05) == (0, math.inf)


def test_nms_hand_cases():
    n_chan = 40
    S = np.zeros((n_chan, 1))
    W = np.ones((n_chan, 1), dtype=np.int32)
    acc = np.zeros((n_chan, 1), dtype=bool)
    # c = 10 (S 6, w 8: half-width 4) loses to c = 13 (S 7, w 1: half-width 1 sees nothing)
    S[10], W[10], acc[10] = 6.0, 8, True
    S[13], W[13], acc[13] = 7.0, 1, True
    # equal SNR at 20 and 21 (w 2: half-width 1): the lower channel survives
    S[20], W[20], acc[20] = 6.0, 2, True
    S[21], W[21], acc[21] = 6.0, 2, True
    # 30 (S 9, w 2) and 33 (S 5, w 9: half-width 4): 33 loses to 30, 30 does not reach 33
    S[30], W[30], acc[30] = 9.0, 2, True
    S[33], W[33], acc[33] = 5.0, 9, True
    # a higher value that is not a provisional detection does not suppress
    S[36], acc[36] = 6.5, True
    S[37] = 50.0
    keep = osr.nms(S, W, acc)
    assert sorted(np.flatnonzero(keep[:, 0]).tolist()) == [13, 20, 30, 36]


def test_reevaluate_closed_form():
    # flanks alternate b - 1, b + 1 (median b, MAD 1); a window of w channels at b + A
    n_chan, b, A, w, c = 400, 2.5, 0.7, 6, 200
    r = np.where(np.arange(n_chan) % 2 == 0, b - 1.0, b + 1.0)
    s = c - w // 2
    r[s:s + w] = b + A
    got = osr.reevaluate(r, c, w)
    assert got == pytest.approx(A * w / (math.sqrt(w) * osr.MAD_K * 1.0), rel=1e-12)
    # constant flanks: MAD 0, cannot be re-evaluated
    assert osr.reevaluate(np.full(n_chan, 1.0), c, w) == -math.inf
    # a band of 8 channels leaves 3 + 2 flank channels around channel 4 (guard 1): too few
    assert osr.reevaluate(np.random.default_rng(1).standard_normal(8), 4, 1) == -math.inf
    assert math.isfinite(osr.reevaluate(np.random.default_rng(1).standard_normal(12), 6, 1))


def test_search_finds_injected_line_and_nothing_in_noise():
    rng = np.random.default_rng(21)
    n_chan, n = 512, 16
    r = rng.standard_normal((n_chan, n, n))
    rec0, _, _, k0, _ = osr.search(r, q=0.01)
    assert len(rec0) == 0 and k0 == 0
    # a 12-channel line of total SNR 14 at (x, y) = (9, 7)
    w0, p0, snr = 12, 300, 14.0
    r[p0:p0 + w0, 7, 9] += snr / math.sqrt(w0)
    rec, S, W, kstar, sstar = osr.search(r, q=0.01)
    assert kstar >= 1 and math.isfinite(sstar)
    hit = rec[(rec["x"] == 9) & (rec["y"] == 7)]
    assert len(hit) == 1
    assert abs(int(hit["c"][0]) - (p0 + w0 // 2)) <= 2
    assert hit["width"][0] in (8, 9, 10, 12, 16)
    assert hit["snr"][0] > 10.0
    # the line's own correlated voxels (neighbouring channels and widths) make up most of the
    # k* provisional detections and lower the BH threshold; the few other survivors are noise
    # voxels just above it (false discoveries, a small fraction of k*)
    others = rec[(rec["x"] != 9) | (rec["y"] != 7)]
    assert len(others) <= max(1, 0.05 * kstar)
    assert (others["snr"] < sstar + 0.5).all()


@pytest.mark.parametrize("sigma,q", [(1.4, 0.05), (1.0, 0.2), (1.0, 0.6)])
def test_search_bh_over_every_searched_voxel(sigma, q):
    # Benjamini-Hochberg over all m in-horizon voxels (Sec. 2.4), pinned to SciPy's adjusted
    # p-values over the same voxels.  Noise wider than the unit-normal model (sigma = 1.4, as
    # Hann-correlated channels give) or a lenient level puts the threshold well below 3 SNR; at
    # q = 0.6 the step-up reaches voxels with S < 0 (p > 1/2)
    rng = np.random.default_rng(int(sigma * 100 + q * 1000))
    n_chan, n = 96, 12
    r = sigma * rng.standard_normal((n_chan, n, n))
    r[40:46, 5, 6] += 3.0
    rec, S, W, kstar, sstar = osr.search(r, q=q)
    valid = oracle.detect.horizon_mask(n)
    sv = S[:, valid].ravel()
    rej = scipy.stats.false_discovery_control(osr.q_value(sv), method="bh") <= q
    assert kstar == int(rej.sum()) > 0
    assert sstar == sv[rej].min() and sstar < 3.0
    if q == 0.6:
        assert sstar < 0.0
    # suppression and re-evaluation see exactly the accepted voxels
    assert all(S[int(a["c"]), int(a["y"]), int(a["x"])] >= sstar for a in rec)


def test_search_accepts_every_voxel_when_all_are_significant():
    # every searched voxel far above any threshold: BH accepts all m of them; constant flanks
    # (MAD 0) then discard every survivor at the re-evaluation
    r = np.full((64, 8, 8), 4.0)
    rec, S, _, kstar, sstar = osr.search(r, q=0.05)
    m = int(oracle.detect.horizon_mask(8).sum()) * 64
    assert kstar == m and sstar == S[:, oracle.detect.horizon_mask(8)].min()
    assert len(rec) == 0


# ---- correlated channels (unit-variance boxcars under a channel correlation) ----

@pytest.mark.parametrize("a", [(1.0, 0.8, 0.3), (1.0, -0.5, 0.2)])
def test_boxcar_sigma_unit_variance_of_ma2_noise(a):
    """Monte Carlo: an MA(2) process x_k = a0 e_k + a1 e_{k-1} + a2 e_{k-2} has correlations
    rho1 = (a0 a1 + a1 a2) / sum a^2, rho2 = a0 a2 / sum a^2; its window sums divided by
    boxcar_sigma have unit variance, while sqrt(w) (the white-noise scale) does not."""
    a0, a1, a2 = a
    var = a0 * a0 + a1 * a1 + a2 * a2
    rho = ((a0 * a1 + a1 * a2) / var, a0 * a2 / var)
    rng = np.random.Generator(np.random.PCG64(11))
    e = rng.standard_normal((1 << 21) + 2)
    x = (a0 * e[2:] + a1 * e[1:-1] + a2 * e[:-2]) / math.sqrt(var)
    for w in (1, 2, 3, 10, 50):
        n = x.size // w
        sums = x[:n * w].reshape(n, w).sum(axis=1)
        v = float(np.var(sums / osr.boxcar_sigma(w, rho)))
        assert abs(v - 1.0) < 0.04, (w, v)
        if w > 1:
            assert abs(float(np.var(sums / math.sqrt(w))) - 1.0) > 0.15
    assert osr.boxcar_sigma(7, ()) == math.sqrt(7)


def test_hann_cross_product_channel_correlations():
    """The cross-correlation products of two independent white inputs, windowed with the periodic
    Hann window and transformed (numpy FFT), have the channel correlations HANN_CROSS_RHO."""
    rng = np.random.Generator(np.random.PCG64(12))
    n = 4096
    win = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n) / n)
    acc = np.zeros(3)
    for _ in range(64):
        z = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
        X = np.fft.fft(z * win, axis=1)
        v = (X[0] * np.conj(X[1])).real
        v = v / v.std()
        acc += [np.mean(v * v), np.mean(v[:-1] * v[1:]), np.mean(v[:-2] * v[2:])]
    acc /= 64
    assert abs(acc[1] / acc[0] - osr.HANN_CROSS_RHO[0]) < 0.01
    assert abs(acc[2] / acc[0] - osr.HANN_CROSS_RHO[1]) < 0.01


def test_search_with_channel_correlation_keeps_noise_unit_normal():
    """A noise-only cube with the Hann cross-product correlations: under the matching rho the
    best-over-widths statistic of a single width is unit normal, and BH admits nothing at
    q = 0.01; with the white-noise scale the same cube overflows BH."""
    # an MA(2) process with rho = HANN_CROSS_RHO: a0 a2 / S = 1/36, (a0 + a2) a1 / S = 4/9
    from scipy.optimize import fsolve

    def eq(v):
        a0, a1, a2 = v
        S = a0 * a0 + a1 * a1 + a2 * a2
        return [a0 * a2 / S - osr.HANN_CROSS_RHO[1], (a0 * a1 + a1 * a2) / S - osr.HANN_CROSS_RHO[0], S - 1.0]

    a = fsolve(eq, [0.8, 0.5, 0.05])
    rng = np.random.Generator(np.random.PCG64(13))
    n_chan, n_pix = 600, 8
    e = rng.standard_normal((n_chan + 2, n_pix, n_pix))
    r = a[0] * e[2:] + a[1] * e[1:-1] + a[2] * e[:-2]
    valid = np.ones((n_pix, n_pix), dtype=bool)
    S1, _ = osr.boxcar_bank(r, widths=(20,), rho=osr.HANN_CROSS_RHO)
    s = S1[np.isfinite(S1)]
    assert abs(float(np.var(s)) - 1.0) < 0.1
    rec, _, _, kstar, _ = osr.search(r, q=0.01, widths=(1, 2, 5, 10, 20), valid=valid, rho=osr.HANN_CROSS_RHO)
    assert kstar == 0 and len(rec) == 0
    _, _, _, k_white, _ = osr.search(r, q=0.01, widths=(1, 2, 5, 10, 20), valid=valid)
    assert k_white > 0
