"""The instrument-scale step (352 antennas x 2 pol, 65,536-point channelizer keeping 4,096 channels,
T = 32, int8 correlation with Stokes I overlapped with 256 x 256 gridded imaging, 5 sigma
detection) run on the GPU exactly as the benchmark times it, checked against the oracle on the same synthetic voltages:
every requantised code (bit-exact away from rounding ties), the visibilities of sampled channels
(bit-exact), their whole images (within 1e-5 of the peak), the full SNR spectra of the injected
tones' pixels, and every tone loud enough at its nearest pixel detected at its closed-form SNR."""
import math

import numpy as np
import pytest

import synth
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402

DEV = torch.device("cuda", 0)


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)


def test_instrument_step_against_oracle():
    cfg = synth.make_config(2)
    xyz, volt, freq, gain = synth.config_inputs(cfg, device="cuda")
    n_in, C, T, n_pix = cfg.n_in, cfg.n_chan, cfg.n_spec, cfg.n_pix
    _say(f"{cfg.name}: running the step on the GPU")
    ctx = nb.nbsi_create(0)
    g = torch.from_numpy(gain).to(DEV)
    plan = nb.ImagePlan(xyz, freq, n_pix, nb.NBSI_IMAGE_GRID, ctx=ctx)
    spec_q, _ = nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, g, want_q=True, ctx=ctx)
    nprod = n_in * (n_in + 1) // 2
    vis = torch.empty((C, nprod, 2), dtype=torch.int32, device=DEV)
    st = torch.empty((C, plan.n_pairs(), 2), dtype=torch.float32, device=DEV)
    _, _, img = nb.nbsi_correlate_image(spec_q, plan, vis=vis, stokes_i=st)
    rec, snr, n = nb.nbsi_detect(img, thresh=5.0, want_snr=True, ctx=ctx)
    torch.cuda.synchronize()
    q_gpu = spec_q.cpu().numpy()
    v_cpu = volt.cpu().numpy()
    del volt
    _say("oracle channelizer over every input and spectrum")
    X = oracle.channelize(v_cpu, cfg.n_fft, T, cfg.chan0, C)
    del v_cpu
    q_ref = oracle.requantize(X, gain)
    diff = q_gpu.astype(np.int16) - q_ref.astype(np.int16)
    bad = np.argwhere(diff != 0)
    _say(f"codes: {len(bad)} of {q_ref.size} differ")
    assert np.abs(diff).max(initial=0) <= 1
    ref_f = np.stack([X.real, X.imag], axis=2) * gain[None, :, None, None].astype(np.float64)
    tie_tol = 2e-5 * np.abs(ref_f).max()
    for c, i, comp, s in bad[:2000]:
        val = float(np.float32(np.float32(ref_f[c, i, comp, s] / gain[i]) * gain[i]))
        assert abs(abs(val - math.floor(val)) - 0.5) < tie_tol, (c, i, comp, s, val)
    assert len(bad) <= max(2, q_ref.size // 10000)
    del X, ref_f

    # channels of the injected tones, and a few more, whose codes all agree
    tone_ch = sorted({(t.k0 + cfg.n_fft // 2) - cfg.chan0 for t in cfg.tones})
    clean = np.ones(C, bool)
    clean[np.unique(bad[:, 0])] = False
    rng = np.random.default_rng(9)
    sample = [c for c in tone_ch if clean[c]][:3] + [int(c) for c in rng.choice(np.flatnonzero(clean), 3, replace=False)]
    _say(f"visibilities and images of channels {sample}")
    vis_g = vis.cpu().numpy()
    img_g = img.cpu().numpy()
    h = n_pix // 2
    pix = [(int(x), int(y)) for x, y in rng.integers(0, n_pix, (300, 2)) if (x - h) ** 2 + (y - h) ** 2 < h * h]
    for t in cfg.tones:
        pix.append((int(round(t.l0 * h + h)), int(round(t.m0 * h + h))))
    pix = np.array(pix, dtype=np.int32)
    for c in sample:
        v_ref = oracle.correlate(q_ref[c:c + 1])
        np.testing.assert_array_equal(vis_g[c], v_ref[0])
        # the whole image against the direct Fourier sum over the same baseline set
        ref_img = oracle.image_dft(v_ref, xyz, freq[c:c + 1], n_pix, grid_n_pix=n_pix)[0]
        scale = np.abs(ref_img).max()
        d = np.abs(img_g[c].astype(np.float64) - ref_img)
        _say(f"channel {c}: image max-abs/peak {d.max() / scale:.2e}, rms/peak {np.sqrt((d * d).mean()) / scale:.2e}")
        assert d.max() <= 1e-5 * scale and np.sqrt((d * d).mean()) <= 1e-6 * scale, c

    # the tones' pixels: every channel's image value from the oracle's visibilities, then the
    # per-pixel SNR spectrum of the detector's noise model
    _say("oracle visibilities of every channel for the tone pixels' spectra")
    v_all = oracle.correlate(q_ref)
    tone_pix = np.unique(pix[-len(cfg.tones):], axis=0)
    spec = oracle.image_dft_pixels(v_all, xyz, freq, n_pix, tone_pix, grid_n_pix=n_pix)  # [C][P]
    del v_all
    snr_g = snr.cpu().numpy()
    for j, (x, y) in enumerate(tone_pix):
        s = spec[:, j]
        med = oracle.detect.median_even_mean(s, axis=0)
        mad = oracle.detect.median_even_mean(np.abs(s - med), axis=0)
        ref_snr = (s - med) / (oracle.detect.MAD_K * mad)
        assert np.abs(snr_g[:, y, x] - ref_snr).max() <= 1e-3 * max(1.0, np.abs(ref_snr).max()), (x, y)
    _say(f"detections: {n}")
    assert n == len(rec)
    for r in rec:
        assert (r["x"] - h) ** 2 + (r["y"] - h) ** 2 < h * h and r["snr"] >= 5.0
    # every tone whose closed-form SNR at its nearest pixel is >= 8 is detected there, in its
    # channel, with an SNR within 3 of that closed form (unit-variance noise: a 3 sigma band).
    # Closed form at the source: 2 sqrt(T N_b) A^2 N / (3 sigma^2) (periodic Hann, on-bin tone);
    # at the pixel centre it is scaled by the synthesized beam B(l_x - l0, m_y - m0), the image
    # of the noise-free point source there
    a, b_ = np.tril_indices(cfg.n_ant, -1)
    n_checked = 0
    for t in cfg.tones:
        ct = (t.k0 + cfg.n_fft // 2) - cfg.chan0
        xt, yt = int(round(t.l0 * h + h)), int(round(t.m0 * h + h))
        nu = freq[ct:ct + 1]
        n_b = int(oracle.count_baselines(xyz, nu, n_pix)[0])
        u = (xyz[a, 0] - xyz[b_, 0]) * nu[0] / synth.C_LIGHT
        v = (xyz[a, 1] - xyz[b_, 1]) * nu[0] / synth.C_LIGHT
        ph = np.exp(2j * np.pi * (u * t.l0 + v * t.m0))
        vis_pt = np.zeros((1, nprod, 2))
        for pol in (0, 1):
            i, j = 2 * a + pol, 2 * b_ + pol
            vis_pt[0, i * (i + 1) // 2 + j] = np.stack([ph.real, ph.imag], -1)
        beam = oracle.image_dft_pixels(vis_pt, xyz, nu, n_pix, np.array([[xt, yt]]), grid_n_pix=n_pix)[0, 0]
        snr_cf = 2.0 * math.sqrt(T * n_b) * t.amp ** 2 * cfg.n_fft / (3.0 * cfg.sigma ** 2) * beam
        got = float(snr_g[ct, yt, xt])
        hit = any(int(r["c"]) == ct and int(r["x"]) == xt and int(r["y"]) == yt for r in rec)
        _say(f"tone at channel {ct} pixel ({xt}, {yt}): closed form {snr_cf:.2f}, measured {got:.2f}, detected {hit}")
        if snr_cf >= 8.0:
            n_checked += 1
            assert hit and abs(got - snr_cf) <= 3.0, (ct, xt, yt, snr_cf, got)
    assert n_checked >= 1
