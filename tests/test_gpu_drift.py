"""Drift-rate search on the GPU (nbsi_dedoppler) against the oracle (oracle/drift.py), and end
to end: a tone drifting across four sub-integrations, each sent through channelize, correlate,
image and the per-pixel standardisation on the GPU, is found at its start channel and drift."""
import math

import numpy as np
import pytest

import synth
from oracle import drift as odr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("n_sub,n_chan,n_pix,max_drift", [(1, 70, 16, 3), (3, 200, 24, 5), (8, 333, 16, 16),
                                                           (5, 64, 32, 0)])
def test_dedoppler_matches_oracle(n_sub, n_chan, n_pix, max_drift):
    print(f"dedoppler S={n_sub} C={n_chan} n_pix={n_pix} D={max_drift}", flush=True)
    rng = np.random.default_rng(n_sub * 100 + n_chan)
    r = rng.standard_normal((n_sub, n_chan, n_pix, n_pix)).astype(np.float32)
    best, drift = nb.nbsi_dedoppler(torch.from_numpy(r).to(DEV), max_drift)
    torch.cuda.synchronize()
    ref, dref = odr.dedoppler(r.astype(np.float64), max_drift)
    b = best.cpu().numpy().astype(np.float64)
    d = drift.cpu().numpy().astype(np.int32)
    assert np.abs(b - ref).max() <= 2e-6
    bad = np.argwhere(d != dref)
    flat = r.astype(np.float64).reshape(n_sub, n_chan, -1)
    for c, y, x in bad[:1000]:  # only near-ties may pick another drift, and it must achieve the best
        dd = int(d[c, y, x])
        assert 0 <= c + dd < n_chan
        v = sum(flat[s, c + odr.shift(dd, s, n_sub), y * n_pix + x] for s in range(n_sub)) / math.sqrt(n_sub)
        assert abs(v - ref[c, y, x]) <= 2e-6


def test_drifting_tone_end_to_end():
    n_ant, n_fft, t_sub, n_sub, n_chan, n_pix, d0 = 16, 4096, 8, 4, 64, 64, 6
    xyz = synth.antenna_layout(n_ant, 100.0, 1001)
    chan0 = n_fft // 2 + 256 - 24
    freq = synth.channel_freqs(n_fft, chan0, n_chan)
    plan = nb.nbsi_image_plan_create(xyz, freq, n_pix, nb.NBSI_IMAGE_DFT)
    gain = torch.full((2 * n_ant,), float(synth.gain_loud_tone(n_fft, 1.5, synth.SIGMA)), device=DEV)
    cubes = []
    for s in range(n_sub):
        k0 = 256 + odr.shift(d0, s, n_sub)  # the tone moves d0 channels over the dump
        tone = synth.Tone(k0=k0, amp=1.5, l0=0.2, m0=-0.1)
        v = synth.voltages(n_ant, n_fft, t_sub, [tone], xyz, 4000 + s, device="cuda")
        q, _ = nb.nbsi_channelize(v, n_fft, t_sub, chan0, n_chan, gain)
        vis = nb.nbsi_correlate(q)
        img = nb.nbsi_image(plan, vis)
        _, snr, _ = nb.nbsi_detect(img, want_snr=True)
        cubes.append(snr)
    stack = torch.stack(cubes).contiguous()
    best, drift = nb.nbsi_dedoppler(stack, 10)
    b = best.cpu().numpy()
    dr = drift.cpu().numpy()
    c, y, x = np.unravel_index(int(np.argmax(np.where(np.isfinite(b), b, -np.inf))), b.shape)
    c_tone = 256 + n_fft // 2 - chan0
    print(f"  peak at c={c} (x, y)=({x}, {y}) drift {int(dr[c, y, x])} SNR {b[c, y, x]:.1f}", flush=True)
    # the brightest track starts at the tone's first channel with the tone's drift (its pixel may
    # be a sidelobe: the 200 m array's beam is narrower than a 64^2 pixel, and the source lies
    # 0.4 pixel from the nearest pixel centre)
    assert c == c_tone and int(dr[c, y, x]) == d0
    # at the pixel nearest the source the same track is found, far above the zero-drift sum
    assert int(dr[c_tone, 29, 38]) == d0
    zero = stack[:, c_tone, 29, 38].sum().item() / math.sqrt(n_sub)
    assert b[c_tone, 29, 38] > 1.5 * zero
