"""End-to-end pins of the oracle chain channelize -> requantise -> correlate -> image -> detect.

* The tiny configuration (16 antennas, one loud tone from (l, m) = (0.2, -0.1)) must detect the
  tone in its channel at the pixel nearest the source, and nothing away from it.
* A weak on-bin tone must come out at the SNR the radiometer closed form predicts:
  SNR = 2 sqrt(T N_b) A^2 N / (3 sigma^2) for a periodic-Hann channelizer (sum w = N/2,
  sum w^2 = 3N/8), consistent with the paper's scaling sigma_nu ~ (dnu t)^-1/2 (Sec. 3.1).
"""
import numpy as np

import synth


def _chain(orc, volt, cfg_like, xyz, freq, gain, n_pix, grid_n_pix=0):
    X = orc.channelize(volt, cfg_like["n_fft"], cfg_like["n_spec"], cfg_like["chan0"],
                       cfg_like["n_chan"])
    q = orc.requantize(X, gain)
    vis = orc.correlate(q)
    img = orc.image_dft(vis, xyz, freq, n_pix, grid_n_pix)
    return X, q, vis, img


def test_tiny_config_detects_its_tone(orc):
    cfg = synth.make_config(1)
    xyz, volt, freq, gain = synth.config_inputs(cfg)
    d = dict(n_fft=cfg.n_fft, n_spec=cfg.n_spec, chan0=cfg.chan0, n_chan=cfg.n_chan)
    X, q, vis, img = _chain(orc, volt.numpy(), d, xyz, freq, gain, cfg.n_pix)
    c_tone = cfg.n_fft // 2 + 256 - cfg.chan0
    # the tone's channel holds ~107 LSB per component after requantisation
    assert 90 < np.abs(q[c_tone].astype(float)).max() <= 127
    rec, snr, valid = orc.detect.detect(img, tau=5.0)
    assert len(rec) > 0
    at_tone = rec[rec["c"] == c_tone]
    near = at_tone[(at_tone["x"] == 38) & (at_tone["y"] == 29)]   # nearest pixel to (38.4, 28.8)
    assert len(near) == 1 and near["snr"][0] > 1000
    # Away from the tone only noise remains.  With 16 antennas, T = 16 and 64 channels the
    # per-pixel noise is chi^2-like (beamformed power) and the MAD of 64 samples scatters by
    # ~15%, so a handful of 5-6 sigma noise voxels is expected, but nothing strong.
    far = rec[np.abs(rec["c"] - c_tone) > 1]
    assert len(far) < 40 and (len(far) == 0 or far["snr"].max() < 8.0)


def test_weak_tone_snr_matches_closed_form(orc):
    n_ant, n_fft, n_spec, n_chan, n_pix = 16, 1024, 64, 256, 32
    xyz = synth.antenna_layout(n_ant, 100.0, seed=21)
    chan0 = n_fft // 2 - n_chan // 2
    c_rel = 140
    k0 = chan0 + c_rel - n_fft // 2
    dx, dy = 6, -4
    l0, m0 = dx * 2.0 / n_pix, dy * 2.0 / n_pix
    n_b = n_ant * (n_ant - 1) // 2
    sig = synth.SIGMA
    A = synth.tone_amp_for_snr(15.0, n_fft, n_spec, n_b, sig)
    expect = 2 * np.sqrt(n_spec * n_b) * A * A * n_fft / (3 * sig * sig)
    volt = synth.voltages(n_ant, n_fft, n_spec, [synth.Tone(k0, A, l0, m0)], xyz, seed=22)
    freq = synth.channel_freqs(n_fft, chan0, n_chan)
    gain = np.full(2 * n_ant, synth.gain_noise(n_fft, sig), np.float32)
    d = dict(n_fft=n_fft, n_spec=n_spec, chan0=chan0, n_chan=n_chan)
    X, q, vis, img = _chain(orc, volt.numpy(), d, xyz, freq, gain, n_pix)
    assert abs(q.astype(float).std() - 8.0) < 0.2
    rec, snr, valid = orc.detect.detect(img, tau=5.0)
    got = snr[c_rel, n_pix // 2 + dy, n_pix // 2 + dx]
    assert abs(got - expect) < 3.5, (got, expect)
    hit = rec[(rec["c"] == c_rel) & (rec["x"] == n_pix // 2 + dx) & (rec["y"] == n_pix // 2 + dy)]
    assert len(hit) == 1
