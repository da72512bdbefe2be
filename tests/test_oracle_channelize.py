"""Pins of the oracle channelizer and requantiser against closed forms and brute force.

The channelizer is the paper's upchannelisation (Sec. 2.1): an FFT over the time samples of
a coarse channel, here with a periodic Hann window and fftshifted channel order.
"""
import numpy as np
import pytest


def _tone_volt(n_fft, n_spec, seq):
    """int8 voltages [1][n_spec*n_fft][2] repeating the complex sequence `seq` (period divides n_fft)."""
    seq = np.asarray(seq)
    reps = n_fft * n_spec // len(seq)
    z = np.tile(seq, reps)
    v = np.stack([z.real, z.imag], axis=-1).astype(np.int8)
    return v[None]


@pytest.mark.parametrize("n_fft", [1024, 4096])
def test_on_bin_tone_lands_in_its_bin(orc, n_fft):
    # x[n] = A i^n is a tone at baseband bin +N/4, exactly representable in int8.
    A = 100
    v = _tone_volt(n_fft, 2, [A, 1j * A, -A, -1j * A])
    c_tone = (n_fft // 4 + n_fft // 2) % n_fft          # fftshifted channel of bin +N/4
    out = orc.channelize(v, n_fft, 2, c_tone - 8, 16)   # [16][1][2]
    X = out[:, 0, :]
    # Hann: sum w = N/2 on the bin, -N/4 on each neighbour, zero elsewhere.
    np.testing.assert_allclose(X[8], A * n_fft / 2, atol=1e-7)
    np.testing.assert_allclose(X[7], -A * n_fft / 4, atol=1e-7)
    np.testing.assert_allclose(X[9], -A * n_fft / 4, atol=1e-7)
    others = np.delete(X, [7, 8, 9], axis=0)
    assert np.abs(others).max() < 1e-7


def test_negative_frequency_and_phase(orc):
    n_fft, A = 2048, 90
    # x[n] = i A (-i)^n: bin -N/4 with phase pi/2.
    v = _tone_volt(n_fft, 1, [1j * A, A, -1j * A, -A])
    c = (-n_fft // 4 + n_fft // 2) % n_fft
    X = orc.channelize(v, n_fft, 1, c - 1, 3)[:, 0, 0]
    np.testing.assert_allclose(X[1], 1j * A * n_fft / 2, atol=1e-7)
    np.testing.assert_allclose(X[0], -1j * A * n_fft / 4, atol=1e-7)


def test_dc_lands_in_centre_channel(orc):
    n_fft, A = 512, 7
    v = _tone_volt(n_fft, 3, [A])
    X = orc.channelize(v, n_fft, 3, n_fft // 2 - 2, 5)[:, 0, :]
    np.testing.assert_allclose(X[2], A * n_fft / 2, atol=1e-9)
    np.testing.assert_allclose(X[1], -A * n_fft / 4, atol=1e-9)
    np.testing.assert_allclose(X[3], -A * n_fft / 4, atol=1e-9)
    np.testing.assert_allclose(X[[0, 4]], 0, atol=1e-9)


@pytest.mark.parametrize("n0,wval", [(0, 0.0), (256, 1.0), (128, 0.5), (384, 0.5)])
def test_impulse_samples_the_window(orc, n0, wval):
    # An impulse at n0 gives X[k] = w[n0] x exp(-2 pi i k n0 / N); Hann: w[0]=0, w[N/2]=1, w[N/4]=1/2.
    n_fft = 512
    v = np.zeros((1, n_fft, 2), np.int8)
    v[0, n0] = (3, -5)
    X = orc.channelize(v, n_fft, 1, 0, n_fft)[:, 0, 0]
    k = (np.arange(n_fft) + n_fft // 2) % n_fft
    expect = wval * (3 - 5j) * np.exp(-2j * np.pi * k * n0 / n_fft)
    np.testing.assert_allclose(X, expect, atol=1e-9)


def test_hann_sums(orc):
    for n in (64, 4096):
        w = orc.hann(n)
        assert abs(w.sum() - n / 2) < 1e-9
        assert abs((w * w).sum() - 3 * n / 8) < 1e-9


@pytest.mark.parametrize("n", [8, 256, 4096])
def test_fft_matches_direct_dft_and_numpy(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = orc.fft(x)
    scale = np.abs(X).max()
    assert np.abs(X - orc.dft(x)).max() < 1e-12 * scale * np.log2(n) * 10
    assert np.abs(X - np.fft.fft(x)).max() < 1e-12 * scale * np.log2(n) * 10


def test_parseval(orc):
    n_fft, n_spec = 1024, 3
    rng = np.random.default_rng(5)
    v = rng.integers(-127, 128, size=(2, n_spec * n_fft, 2)).astype(np.int8)
    X = orc.channelize(v, n_fft, n_spec, 0, n_fft)       # all channels
    w = orc.hann(n_fft)
    for i in range(2):
        for s in range(n_spec):
            z = v[i, s * n_fft:(s + 1) * n_fft].astype(np.float64)
            z = (z[:, 0] + 1j * z[:, 1]) * w
            lhs = (np.abs(X[:, i, s]) ** 2).sum()
            rhs = n_fft * (np.abs(z) ** 2).sum()
            assert abs(lhs - rhs) < 1e-9 * rhs


def test_spectra_are_consecutive_blocks(orc):
    # Spectrum s sees only samples [s N, (s+1) N): a tone in block 1 only appears in spectrum 1.
    n_fft = 256
    v = np.zeros((1, 3 * n_fft, 2), np.int8)
    v[0, n_fft:2 * n_fft, 0] = 10
    X = orc.channelize(v, n_fft, 3, n_fft // 2, 1)[0, 0]
    np.testing.assert_allclose(X, [0, 10 * n_fft / 2, 0], atol=1e-9)


def test_requantize_round_half_even_and_clip(orc):
    vals = np.array([2.5, 3.5, -2.5, -3.5, 0.49999997, 126.5, 127.4, 127.6, 400.0, -400.0, -127.5,
                     1e-30, -0.5])
    expect = np.array([2, 4, -2, -4, 0, 126, 127, 127, 127, -127, -127, 0, 0])
    spec = (vals + 1j * vals[::-1]).reshape(1, 1, -1)
    q = orc.requantize(spec, np.array([1.0], np.float32))
    np.testing.assert_array_equal(q[0, 0, 0], expect)
    np.testing.assert_array_equal(q[0, 0, 1], expect[::-1])


def test_requantize_applies_gain_in_float32(orc):
    # g * X is formed in float32: with g = fl32(0.1), 25 g = 2.50000003725 in float64 (which would
    # round to 3) but exactly 2.5 in float32, which rounds half-to-even to 2.
    spec = np.array([[[25.0 + 0j]]])
    q = orc.requantize(spec, np.array([0.1], np.float32))
    assert q[0, 0, 0, 0] == 2 and q[0, 0, 1, 0] == 0
