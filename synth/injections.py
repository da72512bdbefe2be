"""Classifier training data built through the library's own pipeline: noise visibilities from
synthetic voltages (channelize, correlate), sky tones, horizon RFI and broadband spikes added to
them as visibilities, imaging, and the threshold detector; every detector candidate becomes a
stamp of the SNR cube labelled 1 when it sits on an injected sky tone (within one channel and
1.5 pixels) and 0 otherwise.  Input generation for tests and benchmarks (the classifier's
inputs); the imaging, detection and stamps run in libnbsi.
"""
from __future__ import annotations

import numpy as np

import synth
from paper_2606_04304_amd import (NBSI_DETECT_PER_PIXEL, NBSI_IMAGE_GRID, ImagePlan, nbsi_channelize,
                                  nbsi_correlate, nbsi_detect, nbsi_image, nbsi_stamps)


def _torch():
    import torch
    return torch


def noise_visibilities(n_ant: int, radius_m: float, n_fft: int, n_spec: int, chan0: int, n_chan: int, seed: int,
                       ctx=None):
    """Antenna layout, channel frequencies and int32 noise visibilities of one synthetic dump."""
    torch = _torch()
    xyz = synth.antenna_layout(n_ant, radius_m, seed)
    volt = synth.voltages(n_ant, n_fft, n_spec, [], xyz, seed + 1, device="cuda")
    gain = torch.full((2 * n_ant,), float(synth.gain_noise(n_fft, synth.SIGMA)), dtype=torch.float32,
                      device=volt.device)
    q, _ = nbsi_channelize(volt, n_fft, n_spec, chan0, n_chan, gain, ctx=ctx)
    del volt
    vis = nbsi_correlate(q, ctx=ctx)
    return xyz, synth.channel_freqs(n_fft, chan0, n_chan), vis


def image_sigma(img) -> float:
    """Robust noise level of an image cube: the median over channels of 1.4826 MAD of the
    in-horizon pixels (used only to set injection amplitudes)."""
    torch = _torch()
    C, N, _ = img.shape
    yy, xx = torch.meshgrid(torch.arange(N, device=img.device), torch.arange(N, device=img.device), indexing="ij")
    inside = ((xx - N // 2) ** 2 + (yy - N // 2) ** 2) < (N // 2) ** 2
    v = img[:, inside]
    med = v.median(dim=1, keepdim=True).values
    mad = (v - med).abs().median(dim=1).values
    return float((1.482602218505602 * mad).median().item())


def build_dataset(xyz, freq, vis_noise, n_pix: int, n_sets: int, seed: int, n_tone: int = 150, n_rfi: int = 50,
                  n_spike: int = 20, thresh: float = 5.0, ctx=None, log=None):
    """Stamps, labels and bookkeeping of n_sets injection sets over one noise dump."""
    torch = _torch()
    dev = vis_noise.device
    plan = ImagePlan(xyz, freq, n_pix, NBSI_IMAGE_GRID, ctx=ctx)
    img = nbsi_image(plan, vis_noise)
    sigma = image_sigma(img)
    stamps, labels, kinds, tone_ids = [], [], [], []
    n_tones, n_found = 0, 0
    rng = np.random.Generator(np.random.PCG64(seed))
    vis_f = torch.empty(vis_noise.shape, dtype=torch.float32, device=dev)
    for s in range(n_sets):
        scene = synth.classifier_scene(rng, len(freq), n_pix, sigma, n_tone, n_rfi, n_spike)
        vis_f.copy_(vis_noise)
        synth.add_sources(vis_f, xyz, freq, [src for _, _, srcs in scene for src in srcs])
        nbsi_image(plan, vis_f, img=img)
        rec, snr, n = nbsi_detect(img, NBSI_DETECT_PER_PIXEL, thresh, want_snr=True, ctx=ctx)
        if n == 0:
            continue
        cands = torch.from_numpy(np.ascontiguousarray(rec).view(np.int32).reshape(-1, 5)).to(dev)
        stamps.append(nbsi_stamps(snr, cands, ctx=ctx))
        lab, kind, tid = _label(rec, scene)
        labels.append(lab)
        kinds.append(kind)
        tone_ids.append(np.where(tid >= 0, tid + n_tones, -1))
        n_tones += sum(1 for k, _, _ in scene if k == synth.KIND_TONE)
        n_found += len(np.unique(tid[tid >= 0]))
        if log:
            log(f"set {s + 1}/{n_sets}: {len(rec)} candidates, {int(lab.sum())} on tones")
    plan.close()
    return {"stamps": torch.cat(stamps), "labels": np.concatenate(labels).astype(np.float32),
            "kinds": np.concatenate(kinds), "tone_ids": np.concatenate(tone_ids), "tones_injected": n_tones,
            "tones_found": n_found, "sigma": sigma}


def _label(rec, scene):
    """1 for candidates on a sky tone; the kind of injection each candidate lies near (or noise)
    and the index of its tone among the scene's tones (-1 when none)."""
    lab = np.zeros(len(rec), dtype=np.float32)
    kind = np.full(len(rec), synth.KIND_NOISE, dtype=np.int32)
    tid = np.full(len(rec), -1, dtype=np.int64)
    cx, cy, cc = rec["x"].astype(np.float64), rec["y"].astype(np.float64), rec["c"]
    t = 0
    for k, (c0, x0, y0), srcs in scene:
        c_lo = min(s.c for s in srcs) - 1
        c_hi = max(s.c for s in srcs) + 1
        if k == synth.KIND_TONE:
            hit = (np.abs(cc - c0) <= 1) & (np.abs(cx - x0) <= 1.5) & (np.abs(cy - y0) <= 1.5)
            lab[hit] = 1.0
            kind[hit] = k
            tid[hit] = t
            t += 1
        else:
            near = (cc >= c_lo) & (cc <= c_hi) & (np.abs(cx - x0) <= 12) & (np.abs(cy - y0) <= 12)
            kind[near & (kind == synth.KIND_NOISE)] = k
    return lab, kind, tid


