"""Precision modes of the imager on the precision workload (352 antennas, 2^18-point
channelizer, 8 spectra, 16,384 channels, 512 x 512 gridded images): visibilities stay exact
int32; the gridding runs in FP32, FP16 or BF16 (FP32 accumulation, FP64 only for uv and
phase terms).  Reported per mode against the FP64 direct-Fourier oracle on 16 channels at
sampled pixels (a patch around the loudest tone plus random in-horizon pixels): max-abs and
RMS error relative to the peak, and the tone's per-pixel spectral SNR over a 64-channel window.

Bars: FP32 1e-5, FP16 2e-3, BF16 1e-2 (max-abs / peak); tone SNR within 1 % of the oracle's.
"""
import json

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402

DEV = torch.device("cuda", 0)
BARS = {nb.NBSI_PREC_FP32: 1e-5, nb.NBSI_PREC_FP16: 2e-3, nb.NBSI_PREC_BF16: 1e-2}
NAMES = {nb.NBSI_PREC_FP32: "fp32", nb.NBSI_PREC_FP16: "fp16", nb.NBSI_PREC_BF16: "bf16"}


def test_precision_modes_against_fp64_oracle():
    print("precision workload: channelize 2^18 x 8 spectra, 16384 channels", flush=True)
    cfg = synth.make_config(4)
    xyz, volt, freq, gain = synth.config_inputs(cfg, device="cuda")
    g = torch.from_numpy(gain).to(DEV)
    q, _ = nb.nbsi_channelize(volt, cfg.n_fft, cfg.n_spec, cfg.chan0, cfg.n_chan, g)
    del volt
    loud = max(cfg.tones, key=lambda t: t.amp)
    c_t = loud.k0 + cfg.n_fft // 2 - cfg.chan0
    c0 = min(max(0, c_t - 32), cfg.n_chan - 64)
    qw = q[c0:c0 + 64].contiguous()
    vis = nb.nbsi_correlate(qw)
    torch.cuda.synchronize()
    # the visibilities are exact: one channel against the oracle's triple loop
    k = c_t - c0
    assert np.array_equal(vis[k:k + 1].cpu().numpy(), oracle.correlate(qw[k:k + 1].cpu().numpy()))
    fw = freq[c0:c0 + 64]
    plan = nb.ImagePlan(xyz, fw, cfg.n_pix, nb.NBSI_IMAGE_GRID)
    imgs = {p: nb.nbsi_image(plan, vis, p).cpu().numpy().astype(np.float64) for p in BARS}
    plan.close()
    # the tone's pixel: the FP32 image's peak within 3 pixels of its sky position
    n = cfg.n_pix
    xt, yt = int(round(n / 2 + loud.l0 * n / 2)), int(round(n / 2 + loud.m0 * n / 2))
    win = imgs[nb.NBSI_PREC_FP32][k, yt - 3:yt + 4, xt - 3:xt + 4]
    dy, dx = np.unravel_index(np.argmax(win), win.shape)
    yt, xt = yt - 3 + dy, xt - 3 + dx
    # sampled pixels: a 24 x 24 patch around the tone and 400 random in-horizon pixels
    rng = np.random.default_rng(4)
    pts = [(x, y) for y in range(yt - 12, yt + 12) for x in range(xt - 12, xt + 12)]
    while len(pts) < 576 + 400:
        x, y = rng.integers(0, n, size=2)
        if (x - n // 2) ** 2 + (y - n // 2) ** 2 < (n // 2) ** 2:
            pts.append((int(x), int(y)))
    pix = np.array(pts, dtype=np.int32)
    chans = sorted(set([k] + list(rng.choice(64, size=15, replace=False))))[:16]
    vis_np = vis.cpu().numpy()
    ref = oracle.image_dft_pixels(vis_np[chans], xyz, fw[chans], n, pix, grid_n_pix=n)    # [16][n_pix]
    spec_ref = oracle.image_dft_pixels(vis_np, xyz, fw, n, np.array([[xt, yt]], np.int32), grid_n_pix=n)[:, 0]
    snr_ref = oracle.detect.per_pixel_snr(spec_ref[:, None])[0][k, 0]
    peak = np.abs(ref).max()
    report = {"workload": "352 ant, 2^18-pt channelizer, T=8, 512^2 GRID; 16 channels x 976 pixels",
              "tone_snr_fp64": round(float(snr_ref), 3)}
    for p, bar in BARS.items():
        got = imgs[p][chans][:, pix[:, 1], pix[:, 0]]
        d = np.abs(got - ref)
        snr = oracle.detect.per_pixel_snr(imgs[p][:, yt, xt][:, None])[0][k, 0]
        report[NAMES[p]] = {"max_abs_over_peak": float(d.max() / peak),
                            "rms_over_peak": float(np.sqrt(np.mean(d * d)) / peak),
                            "tone_snr": round(float(snr), 3),
                            "tone_snr_rel_err": float(abs(snr - snr_ref) / abs(snr_ref))}
    print(json.dumps(report), flush=True)
    assert snr_ref > 8
    for p, bar in BARS.items():
        r = report[NAMES[p]]
        assert r["max_abs_over_peak"] <= bar, (NAMES[p], r)
        assert r["tone_snr_rel_err"] <= 0.01, (NAMES[p], r)
