"""Throughput of the hot path on one MI355X: channelize -> correlate -> image -> detect.

Workload: 352 dual-polarisation antennas (704 inputs, 248,160 correlation products) in a
1.5 km disk, complex int8 voltages (sigma = 8) with 8 injected tones, a 65,536-point Hann
channelizer keeping 4,096 channels, 32 spectra integrated, int8 -> int32 correlation, FP32
gridding + 2D FFT to 256 x 256 all-sky images, 5 sigma per-pixel spectral detection.
Inputs are synthetic (seeded) and resident in HBM before timing starts.

A step is one pass of all four stages over one dump; the correlator writes every visibility and,
from the same sums, Stokes I of the imager's candidate pairs, which the imager grids (the
separate gather from the visibilities gives the same image bit for bit).  The JSON line reports
  value = useful correlation ops of the step / step time (TOPS, 8 ops per complex MAC),
and, in "components", the correlator-only TOPS, the imaged channels/s (imager only and end
to end), and the same figures for the plain FP32 path (float32 spectra, FP32 correlator,
float32 visibilities into the same imager) timed on the same GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0
FP16_PEAK_TFLOPS = 2500.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-path", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the uneven-sub-band leg (batched graph vs per-sub-band launches)")
    ap.add_argument("--batch-only", action="store_true",
                    help="profiling aid: run only the uneven-sub-band leg and print its figures")
    ap.add_argument("--no-deep", action="store_true", help="skip the long-integration correlator leg")
    ap.add_argument("--no-classifier", action="store_true", help="skip the classifier leg")
    ap.add_argument("--no-search", action="store_true", help="skip the full Stage I search leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the C4 precision leg")
    ap.add_argument("--no-c5", action="store_true", help="skip the C5 classifier leg (10^5 injections)")
    ap.add_argument("--leg", default=None,
                    choices=["deep_correlator", "classifier", "stage1_search", "dedoppler", "stage2", "precision",
                             "c5"],
                    help="with --legs-only: run this leg alone")
    ap.add_argument("--step-only", action="store_true",
                    help="profiling aid: only the timed step (no legs, no FP32 path, no batch)")
    ap.add_argument("--legs-only", action="store_true",
                    help="profiling aid: run only the long-integration correlator, classifier and search legs")
    ap.add_argument("--stages", default="all", help="profiling aid: all | correlate")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str, source: str):
    """HBM bytes per launch of `kernel` from the committed counter summary (profiles/traffic.json:
    FETCH_SIZE and WRITE_SIZE scaled by a plain copy's counts), or None when the summary was taken
    on other source code than the current `source` file."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    ent = d.get("kernels", {}).get(kernel)
    if not ent or ent.get("source_sha") != source_digest([source]):
        return None
    return int(ent["hbm_bytes_per_launch"])


def cpu_baseline(cfg, xyz, freq, volt_dev, gain, q_dev, img_dev):
    """Time the oracle on a bounded sample of the same workload and extrapolate to one step."""
    import torch

    import oracle
    n_in, n_fft, T, C, n_pix = cfg.n_in, cfg.n_fft, cfg.n_spec, cfg.n_chan, cfg.n_pix
    threads = oracle.num_threads()
    t = {}
    # channelize: 2 of n_in inputs, every spectrum
    v = volt_dev[:2].cpu().numpy()
    t0 = time.perf_counter()
    oracle.channelize(v, n_fft, T, cfg.chan0, C)
    t["channelize"] = (time.perf_counter() - t0) * n_in / 2
    # correlate: 32 of C channels
    q = q_dev[:32].cpu().numpy()
    t0 = time.perf_counter()
    oracle.correlate(q)
    t["correlate"] = (time.perf_counter() - t0) * C / 32
    # image: 1 channel, direct Fourier sum over the gridded set B
    vis1 = oracle.correlate(q_dev[:1].cpu().numpy())
    t0 = time.perf_counter()
    oracle.image_dft(vis1, xyz, freq[:1], n_pix, grid_n_pix=n_pix)
    t["image"] = (time.perf_counter() - t0) * C
    # detect: 4 image rows (all channels)
    rows = img_dev[:, n_pix // 2 - 2:n_pix // 2 + 2, :].cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    snr, _ = oracle.detect.per_pixel_snr(rows.reshape(C, -1))
    oracle.detect.nms_keep(snr, 5.0)
    t["detect"] = (time.perf_counter() - t0) * n_pix / 4
    step = sum(t.values())
    ops = 8.0 * cfg.n_in * (cfg.n_in + 1) / 2 * T * C
    # the same oracle on one core, on a smaller sample (extrapolated the same way)
    oracle.set_threads(1)
    t1 = {}
    try:
        v1 = volt_dev[:1].cpu().numpy()
        t0 = time.perf_counter()
        oracle.channelize(v1, n_fft, T, cfg.chan0, C)
        t1["channelize"] = (time.perf_counter() - t0) * n_in
        q1 = q_dev[:2].cpu().numpy()
        t0 = time.perf_counter()
        oracle.correlate(q1)
        t1["correlate"] = (time.perf_counter() - t0) * C / 2
        ys, xs = np.mgrid[0:n_pix:4, 0:n_pix:4]
        pix = np.stack([xs.ravel(), ys.ravel()], axis=1)          # 1/16 of the pixels
        t0 = time.perf_counter()
        oracle.image_dft_pixels(vis1, xyz, freq[:1], n_pix, pix, grid_n_pix=n_pix)
        t1["image"] = (time.perf_counter() - t0) * C * (n_pix * n_pix) / len(pix)
        t0 = time.perf_counter()
        snr1, _ = oracle.detect.per_pixel_snr(rows[:, :1].reshape(C, -1))
        oracle.detect.nms_keep(snr1, 5.0)
        t1["detect"] = (time.perf_counter() - t0) * n_pix
    finally:
        oracle.set_threads(threads)
    step1 = sum(t1.values())
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": ops / step / 1e12, "unit": "TOPS", "cores": threads, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": ("channelize 2/704 inputs x 32 spectra (x352); correlate 32/4096 channels "
                       "(x128); direct-Fourier image 1/4096 channels at 256^2 over the gridded "
                       "baseline set (x4096); detect SNR on 4/256 image rows (x64); summed"),
            "stage_seconds": {k: round(v, 3) for k, v in t.items()}, "step_seconds": round(step, 3),
            "one_core": {"value": ops / step1 / 1e12, "unit": "TOPS", "cores": 1,
                         "sample": ("channelize 1/704 inputs (x704); correlate 2/4096 channels (x2048); "
                                    "direct-Fourier image of 1/4096 channels at every 4th pixel of each "
                                    "4th row (x65536); detect SNR on 1/256 image rows (x256); summed"),
                         "stage_seconds": {k: round(v, 3) for k, v in t1.items()},
                         "step_seconds": round(step1, 3)}}


def batched_leg(args, nb, torch, ctx, dev, synth):
    """Twelve uneven sub-bands of 352 antennas (FFT lengths 2^14..2^18, 8..128 spectra, 1024
    channels each, images 128^2..512^2): channelize + correlate + image of all of them, once as
    per-sub-band library calls and once as one batch (grouped persistent launches replayed from a
    captured hipGraph), with default tiles and with autotuned tiles, then with the sub-bands
    pipelined over two streams (sub-band s + 1 channelized while s is correlated and imaged)."""
    n_ant = 352
    n_in = 2 * n_ant
    nprod = n_in * (n_in + 1) // 2
    xyz = synth.antenna_layout(n_ant, 750.0, 3001)
    subs = []
    for i, c in enumerate(synth.subband_configs(12, 1024, n_ant)):
        tones = synth.random_tones(1, c["n_fft"], c["chan0"], c["n_chan"], 5.0, 20.0, xyz, c["n_spec"],
                                   c["n_pix"], seed=3100 + i)
        v = synth.voltages(n_ant, c["n_fft"], c["n_spec"], tones, xyz, 3200 + i, device="cuda", nu0=c["nu0"])
        g = torch.full((n_in,), float(c["gain"]), dtype=torch.float32, device=dev)
        subs.append(dict(volt=v, gain=g, n_fft=c["n_fft"], n_spec=c["n_spec"], chan0=c["chan0"],
                         n_chan=c["n_chan"], n_pix=c["n_pix"],
                         freq_hz=synth.channel_freqs(c["n_fft"], c["chan0"], c["n_chan"], c["nu0"])))
    log("[bench] sub-band inputs ready")
    plans = [nb.nbsi_image_plan_create(xyz, d["freq_hz"], d["n_pix"], nb.NBSI_IMAGE_GRID, ctx=ctx) for d in subs]
    outs = [(torch.empty((d["n_chan"], n_in, 2, d["n_spec"]), dtype=torch.int8, device=dev),
             torch.empty((d["n_chan"], nprod, 2), dtype=torch.int32, device=dev),
             torch.empty((d["n_chan"], d["n_pix"], d["n_pix"]), dtype=torch.float32, device=dev)) for d in subs]

    def per_subband():
        for d, p, (q, vis, img) in zip(subs, plans, outs):
            nb.nbsi_channelize(d["volt"], d["n_fft"], d["n_spec"], d["chan0"], d["n_chan"], d["gain"],
                               spec_q=q, ctx=ctx)
            nb.nbsi_correlate(q, vis=vis, ctx=ctx)
            nb.nbsi_image(p, vis, img=img)

    def timed(fn, k):
        return _timed(torch, fn, k)

    k = max(2, args.steps // 2)
    ms_per = timed(per_subband, k)
    log(f"[bench] per-sub-band launches: {ms_per:.2f} ms")
    eager = nb.Batch(xyz, subs, graph=False, ctx=ctx)
    ms_eager = timed(eager.run, k)
    log(f"[bench] batched launches without a graph (default tiles): {ms_eager:.2f} ms")
    eager.close()
    batch = nb.Batch(xyz, subs, graph=True, ctx=ctx)
    ms_batch = timed(batch.run, k)
    log(f"[bench] batched graph (default tiles): {ms_batch:.2f} ms")
    same = all(torch.equal(bd["vis"], o[1]) and torch.equal(bd["img"], o[2])
               for bd, o in zip(batch.subbands, outs))
    launches = batch.describe()
    batch.close()
    # the same batch with FP16 / BF16 gridding (FP32 accumulation), against the FP32 batch's images
    reduced = {}
    for prec, name in ((nb.NBSI_PREC_FP16, "fp16"), (nb.NBSI_PREC_BF16, "bf16")):
        bp = nb.Batch(xyz, subs, precision=prec, graph=True, ctx=ctx)
        ms_p = timed(bp.run, k)
        worst = 0.0
        for bd, o in zip(bp.subbands, outs):
            peak = o[2].abs().amax(dim=(1, 2))
            worst = max(worst, float(((bd["img"] - o[2]).abs().amax(dim=(1, 2)) / peak).max()))
        reduced[name] = {"batched_graph_ms": round(ms_p, 3), "vs_fp32_batch_max_abs_over_peak": worst}
        bp.close()
        log(f"[bench] batched graph, {name} gridding: {ms_p:.2f} ms")
    tuned = nb.Batch(xyz, subs, graph=True, autotune=True, ctx=ctx)
    ms_tuned = timed(tuned.run, k)
    desc = json.loads(tuned.describe())
    log(f"[bench] batched graph (autotuned): {ms_tuned:.2f} ms")
    tuned.close()
    # sub-band s + 1 channelized while sub-band s is correlated and imaged on a second stream
    over = nb.Batch(xyz, subs, overlap=True, ctx=ctx)
    ms_over = timed(over.run, k)
    same_over = all(torch.equal(bd["vis"], o[1]) and torch.equal(bd["img"], o[2])
                    for bd, o in zip(over.subbands, outs))
    log(f"[bench] batched, sub-bands overlapped on two streams (default tiles): {ms_over:.2f} ms")
    over.close()
    # the plain FP32 path per sub-band: float spectra, FP32 correlator, FP32 gridding (last: it
    # overwrites the per-sub-band images)
    t_max = max(d["n_spec"] for d in subs)
    spec_f = torch.empty((1024 * n_in * 2 * t_max,), dtype=torch.float32, device=dev)
    vis_f = torch.empty((1024, nprod, 2), dtype=torch.float32, device=dev)

    def per_subband_f32():
        for d, p, (_, _, img) in zip(subs, plans, outs):
            sf = spec_f[:d["n_chan"] * n_in * 2 * d["n_spec"]].view(d["n_chan"], n_in, 2, d["n_spec"])
            nb.nbsi_channelize(d["volt"], d["n_fft"], d["n_spec"], d["chan0"], d["n_chan"], d["gain"],
                               want_q=False, want_f=True, spec_f=sf, ctx=ctx)
            nb.nbsi_correlate_f32(sf, vis=vis_f[:d["n_chan"]], ctx=ctx)
            nb.nbsi_image(p, vis_f[:d["n_chan"]], nb.NBSI_PREC_FP32, img=img)

    ms_plain = timed(per_subband_f32, k)
    log(f"[bench] plain FP32 path per sub-band: {ms_plain:.2f} ms")
    del spec_f, vis_f
    n_ch = sum(d["n_chan"] for d in subs)
    ops = sum(8.0 * nprod * d["n_spec"] * d["n_chan"] for d in subs)
    return {
        "workload": "12 sub-bands x 1024 channels, 352 ant x 2 pol, FFT 2^14..2^18, T 128..8, "
                    "GRID 128^2..512^2 (channelize + correlate + image)",
        "per_subband_ms": round(ms_per, 3), "batched_eager_ms": round(ms_eager, 3),
        "batched_graph_ms": round(ms_batch, 3),
        "batched_graph_autotuned_ms": round(ms_tuned, 3),
        "batched_overlapped_ms": round(ms_over, 3),
        "speedup_batched": round(ms_per / ms_batch, 3), "speedup_autotuned": round(ms_per / ms_tuned, 3),
        "speedup_overlapped": round(ms_per / ms_over, 3),
        "overlapped_equals_per_subband": bool(same_over),
        "fine_channels_per_s_autotuned": round(n_ch / (ms_tuned * 1e-3), 1),
        "correlated_tops_autotuned": round(ops / (ms_tuned * 1e-3) / 1e12, 3),
        "batched_equals_per_subband": bool(same),
        "batched_reduced_precision": reduced,
        "plain_fp32_path_per_subband_ms": round(ms_plain, 3),
        "speedup_vs_plain_fp32_path": {"batched_fp32_graph": round(ms_plain / ms_batch, 3),
                                       **{f"batched_{n}_graph": round(ms_plain / r["batched_graph_ms"], 3)
                                          for n, r in reduced.items()}},
        "launches": json.loads(launches)["launches"],
        "autotuned_choices": [(s["n_fft"], s["n_spec"], s["n_pix"], s["corr_variant"], s["grid_ge"])
                              for s in desc["subbands"]],
    }


def _timed(torch, fn, k):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(k):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / k


def precision_leg(args, nb, torch, ctx, dev, synth):
    """C4 at full size: 352 antennas x 2 pol, 2^18-point channelizer keeping 16,384 channels, T = 8
    spectra, 512 x 512 gridded images.  Channelize (int8 codes) and correlate with the Stokes-I
    epilogue once (exact int32 visibilities), then image every channel from Stokes I by gridding
    in FP32, FP16 and BF16 (FP32 accumulation, float64 uv); and the plain FP32 path on the same
    GPU (float spectra, FP32 correlator, FP32 gridding from float visibilities).  FP16 / BF16
    images are compared with the FP32 ones over every channel (worst channel's max-abs and RMS
    error relative to its peak; the FP64-oracle errors at sampled pixels are the precision test's)."""
    cfg = synth.make_config(4)
    xyz, volt, freq, gain = synth.config_inputs(cfg, device="cuda")
    n_in, C, T, n_pix = 2 * cfg.n_ant, cfg.n_chan, cfg.n_spec, cfg.n_pix
    nprod = n_in * (n_in + 1) // 2
    g = torch.from_numpy(gain).to(dev)
    plan = nb.ImagePlan(xyz, freq, n_pix, nb.NBSI_IMAGE_GRID, ctx=ctx)
    n_pairs = plan.n_pairs()
    k = max(2, args.steps // 4)
    q = torch.empty((C, n_in, 2, T), dtype=torch.int8, device=dev)
    ms_chan = _timed(torch, lambda: nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, g, spec_q=q, ctx=ctx), k)
    vis = torch.empty((C, nprod, 2), dtype=torch.int32, device=dev)
    st = torch.empty((C, n_pairs, 2), dtype=torch.float32, device=dev)
    ms_corr = _timed(torch, lambda: nb.nbsi_correlate_stokes(q, plan, vis=vis, stokes_i=st, ctx=ctx), k)
    del vis
    torch.cuda.empty_cache()
    ref = torch.empty((C, n_pix, n_pix), dtype=torch.float32, device=dev)
    img = torch.empty_like(ref)
    modes = {}
    for prec, name in ((nb.NBSI_PREC_FP32, "fp32"), (nb.NBSI_PREC_FP16, "fp16"), (nb.NBSI_PREC_BF16, "bf16")):
        out = ref if prec == nb.NBSI_PREC_FP32 else img
        ms = _timed(torch, lambda: nb.nbsi_image_stokes(plan, st, prec, img=out), k)
        entry = {"image_ms": round(ms, 3), "imaged_channels_per_s": round(C / (ms * 1e-3), 1)}
        if prec != nb.NBSI_PREC_FP32:
            worst_max = worst_rms = 0.0
            for c0 in range(0, C, 1024):
                r, o = ref[c0:c0 + 1024], img[c0:c0 + 1024]
                peak = r.abs().amax(dim=(1, 2))
                d = (o - r).abs()
                worst_max = max(worst_max, float((d.amax(dim=(1, 2)) / peak).max()))
                worst_rms = max(worst_rms, float((d.pow(2).mean(dim=(1, 2)).sqrt() / peak).max()))
            entry.update({"vs_fp32_max_abs_over_peak": worst_max, "vs_fp32_rms_over_peak": worst_rms})
        modes[name] = entry
        log(f"[bench] C4 gridding {name}: {ms:.2f} ms")
    del st
    torch.cuda.empty_cache()
    # plain FP32 path: float spectra, FP32 correlator, FP32 gridding of float visibilities
    spec_f = torch.empty((C, n_in, 2, T), dtype=torch.float32, device=dev)
    ms_chan_f = _timed(torch, lambda: nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, g, want_q=False,
                                                         want_f=True, spec_f=spec_f, ctx=ctx), k)
    vis_f = torch.empty((C, nprod, 2), dtype=torch.float32, device=dev)
    ms_corr_f = _timed(torch, lambda: nb.nbsi_correlate_f32(spec_f, vis=vis_f, ctx=ctx), k)
    ms_img_f = _timed(torch, lambda: nb.nbsi_image(plan, vis_f, nb.NBSI_PREC_FP32, img=img), k)
    log(f"[bench] C4 plain FP32 path: {ms_chan_f + ms_corr_f + ms_img_f:.2f} ms")
    plan.close()
    del spec_f, vis_f, ref, img, q, volt
    torch.cuda.empty_cache()
    mixed = {n: round(ms_chan + ms_corr + modes[n]["image_ms"], 3) for n in modes}
    plain = round(ms_chan_f + ms_corr_f + ms_img_f, 3)
    return {
        "workload": "C4: 352 ant x 2 pol, 2^18-pt channelizer, T=8, 16384 channels, GRID 512^2",
        "channelize_ms": round(ms_chan, 3), "correlate_stokes_ms": round(ms_corr, 3),
        "gridding": modes,
        "mixed_precision_path_ms": mixed,
        "plain_fp32_path_ms": {"channelize_f32": round(ms_chan_f, 3), "correlate_f32": round(ms_corr_f, 3),
                               "image_fp32_from_f32_vis": round(ms_img_f, 3), "total": plain},
        "speedup_vs_plain_fp32_path": {n: round(plain / v, 3) for n, v in mixed.items()},
    }


def c5_leg(args, nb, torch, ctx, dev, synth):
    """C5: candidate cubes of the instrument configuration (352 antennas, 65,536-point channelizer,
    T = 32, 4,096 channels, 256^2 images) with 10^5 synthetic injections through the library's own
    pipeline: 460 injection sets of 150 sky tones, 50 horizon RFI tracks and 20 broadband spikes,
    over three noise dumps (training 300 sets, operating point 60, test 100).  The network is
    trained on the GPU (the library's forward / backward / Adam kernels) on the training dump's
    candidates, its operating point (95 % of tone candidates kept) set on the second dump, and it
    is scored on the third against the plain 5 sigma detector (every candidate accepted):
    precision over accepted candidates, recall over injected tones."""
    from paper_2606_04304_amd import classifier as cl
    from synth import injections as inj
    splits = {"train": (9400, 300), "operating_point": (9500, 60), "test": (9600, 100)}
    data = {}
    t0 = time.perf_counter()
    for name, (seed, n_sets) in splits.items():
        xyz, freq, vis = inj.noise_visibilities(352, 750.0, 65536, 32, 30720, 4096, seed, ctx=ctx)
        data[name] = inj.build_dataset(xyz, freq, vis, 256, n_sets, seed + 7, ctx=ctx)
        del vis
        torch.cuda.empty_cache()
        log(f"[bench] C5 {name}: {n_sets} injection sets, {len(data[name]['labels'])} candidates")
    build_s = time.perf_counter() - t0
    n_inj = sum(220 * n for _, n in splits.values())
    net = nb.Net(synth.net_init(9700), max_batch=512)
    tr = data["train"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = cl.train(net, tr["stamps"], tr["labels"], epochs=3, batch=512, lr=2e-3, seed=9701)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    cut = cl.operating_point(cl.scores(net, data["operating_point"]["stamps"]),
                             data["operating_point"]["labels"], keep=0.95)
    te = data["test"]
    z = cl.scores(net, te["stamps"]) - cut
    lab, tid, n_t = te["labels"], te["tone_ids"], te["tones_injected"]
    p_thr, r_thr = cl.precision_recall(np.ones(len(lab), bool), lab, tid, n_t)
    p_net, r_net = cl.precision_recall(z > 0, lab, tid, n_t)
    kinds = te["kinds"]
    names = {synth.KIND_TONE: "tone", synth.KIND_RFI: "rfi", synth.KIND_SPIKE: "spike", synth.KIND_NOISE: "noise"}
    rej = {names[k]: round(float(np.mean(z[kinds == k] <= 0)), 4) for k in names if np.any(kinds == k)}
    net.close()
    log(f"[bench] C5: threshold P {p_thr:.3f} R {r_thr:.3f}; network P {p_net:.3f} R {r_net:.3f}")
    return {
        "workload": "C5: instrument-scale candidate cubes, 10^5 injections (tones, horizon RFI, broadband "
                    "spikes), 33-channel x 9x9 FP16 stamps, 3-layer conv net",
        "injections": n_inj,
        "candidates": {k: int(len(d["labels"])) for k, d in data.items()},
        "tone_candidates": {k: int(np.sum(d["labels"] > 0.5)) for k, d in data.items()},
        "tones_injected_test": int(n_t),
        "threshold_detector": {"precision": round(p_thr, 4), "recall": round(r_thr, 4)},
        "with_network": {"precision": round(p_net, 4), "recall": round(r_net, 4)},
        "rejected_fraction_by_kind": rej,
        "train_loss_per_epoch": [round(h, 4) for h in hist],
        "data_build_s": round(build_s, 2), "train_s": round(train_s, 3),
    }


def deep_correlator_leg(args, nb, torch, ctx, dev, synth):
    """The correlator alone at 704 inputs and 1,024 channels for integrations T = 32 (the
    instrument configuration), 298 (the paper's 30 s at ~10 Hz) and 1,024 / 2,048: where the
    output write stops dominating, the int8 matrix cores become the bound."""
    n_in, C = 704, 1024
    nprod = n_in * (n_in + 1) // 2
    vis = torch.empty((C, nprod, 2), dtype=torch.int32, device=dev)
    rows = []
    for T in (32, 298, 1024, 2048):
        q = synth.random_spectra(C, n_in, T, seed=5000 + T, full_range=True, device="cuda")
        ms = _timed(torch, lambda: nb.nbsi_correlate(q, vis=vis, ctx=ctx), max(3, args.steps // 2))
        useful = 8.0 * nprod * T * C
        hbm = C * 2 * n_in * T + C * nprod * 8
        rows.append({"n_spec": T, "kernel": nb.nbsi_correlate_kernel(n_in, T), "ms": round(ms, 4),
                     "useful_tops": round(useful / (ms * 1e-3) / 1e12, 2),
                     "frac_of_int8_mfma_peak": round(useful / (ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4),
                     "hbm_gbs": round(hbm / (ms * 1e-3) / 1e9, 1),
                     "frac_of_hbm": round(hbm / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        log(f"[bench] deep correlator T={T}: {ms:.3f} ms, {rows[-1]['useful_tops']} TOPS")
        del q
    del vis
    torch.cuda.empty_cache()
    return {"workload": "correlator only, 704 inputs x 1024 channels, random int8 spectra", "rows": rows}


def classifier_leg(args, nb, torch, ctx, dev, synth):
    """The candidate classifier on 100,000 stamps (33 channels x 9 x 9, FP16): one training epoch
    in mini-batches of 512 (forward, backward, Adam per step) and inference over all stamps.
    FLOP per stamp: forward 7.52 M; training 21.0 M (forward, weight gradients of the three
    convolutions and data gradients of the upper two)."""
    n, B = 100_000, 512
    g = torch.Generator(device=dev)
    g.manual_seed(6001)
    stamps = torch.randn((n, nb.NBSI_STAMP_CHANNELS, nb.NBSI_STAMP_PIXELS, nb.NBSI_STAMP_PIXELS),
                         generator=g, device=dev).to(torch.float16)
    labels = (torch.rand(n, generator=g, device=dev) < 0.4).to(torch.float32)
    idx = torch.randperm(n, generator=g, device=dev).to(torch.int32)
    net = nb.Net(synth.net_init(6002), max_batch=4096, ctx=ctx)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    n_steps = n // B

    def epoch():
        for s0 in range(0, n_steps * B, B):
            net.train_step(stamps, labels, index=idx[s0:s0 + B], lr=1e-3, loss=loss)

    logits = torch.empty(n, dtype=torch.float32, device=dev)

    def infer():
        for s0 in range(0, n, 4096):
            m = min(4096, n - s0)
            net.forward(stamps[s0:s0 + m], logits=logits[s0:s0 + m])

    ms_train = _timed(torch, epoch, 2)
    ms_inf = _timed(torch, infer, 3)
    net.close()
    fwd, train = 7.52e6, 21.0e6
    tr_rate = n_steps * B / (ms_train * 1e-3)
    inf_rate = n / (ms_inf * 1e-3)
    log(f"[bench] classifier: train {tr_rate:.0f} stamps/s, infer {inf_rate:.0f} stamps/s")
    return {"workload": "100,000 FP16 stamps 33x9x9, batch 512 training, batch 4096 inference",
            "train_epoch_ms": round(ms_train, 3), "train_stamps_per_s": round(tr_rate, 1),
            "train_tflops": round(train * tr_rate / 1e12, 2),
            "train_frac_of_fp16_mfma_peak": round(train * tr_rate / 1e12 / FP16_PEAK_TFLOPS, 4),
            "infer_ms": round(ms_inf, 3), "infer_stamps_per_s": round(inf_rate, 1),
            "infer_tflops": round(fwd * inf_rate / 1e12, 2),
            "infer_frac_of_fp16_mfma_peak": round(fwd * inf_rate / 1e12 / FP16_PEAK_TFLOPS, 4)}


def search_leg(args, nb, torch, ctx, dev, C, n_pix):
    """The full Stage I search (boxcar bank of 26 widths, Benjamini-Hochberg at q = 0.01,
    suppression, re-evaluation) at the instrument's cube size, 4096 channels x 256^2, on a
    standardised residual cube of unit-variance white noise (seeded) with 64 injected lines of
    widths 1..100 and matched-filter SNR 8..30.  The step's own imaged cube, whose channels the
    periodic Hann window correlates, is searched in search_pipeline_leg."""
    g = torch.Generator(device=dev)
    g.manual_seed(7001)
    snr = torch.randn((C, n_pix, n_pix), generator=g, device=dev)
    rng = np.random.Generator(np.random.PCG64(7002))
    widths = (1, 2, 3, 5, 8, 12, 20, 32, 50, 80, 100)
    for i in range(64):
        w = int(widths[i % len(widths)])
        x, y = (int(v) for v in rng.integers(n_pix // 4, 3 * n_pix // 4, 2))
        c0 = int(rng.integers(150, C - 250))
        snr[c0:c0 + w, y, x] += float(rng.uniform(8.0, 30.0)) / math.sqrt(w)
    torch.cuda.synchronize()
    res = nb.nbsi_search(snr, fdr_q=0.01, ctx=ctx)
    reps = max(2, args.steps // 3)
    t0 = time.perf_counter()
    for _ in range(reps):
        res = nb.nbsi_search(snr, fdr_q=0.01, ctx=ctx)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    rec, thr, kprov = res[0], res[1], res[2]
    vox = C * n_pix * n_pix
    # bank: the SNR cube in, best SNR (4 B) and width (1 B) out; accept: the best SNR read again
    algo = vox * 4 + vox * 5 + vox * 4
    log(f"[bench] stage I search: {ms:.3f} ms, k* {kprov}, S* {thr:.3f}, {len(rec)} candidates")
    del snr
    torch.cuda.empty_cache()
    return {"workload": "4096 x 256^2 standardised white-noise cube with 64 injected lines (widths 1..100, "
                        "SNR 8..30), 26 boxcar widths 1..100, BH q = 0.01",
            "ms": round(ms, 3), "voxels_per_s": round(vox / (ms * 1e-3), 1), "provisional": kprov,
            "threshold_snr": round(thr, 4) if math.isfinite(thr) else None, "candidates": int(len(rec)),
            "algorithmic_bytes": algo, "gbs": round(algo / (ms * 1e-3) / 1e9, 1)}


def search_pipeline_leg(args, nb, torch, ctx, img, C, n_pix):
    """The Stage I search on the step's own output: the per-pixel SNR cube of the last step's
    images (nbsi_detect), whose noise the periodic Hann window correlates across channels.  The
    measured lag-1..3 correlations of that cube are reported beside the model's (4/9, 1/36, 0),
    and the search runs with the model's correlations (unit-variance boxcars) and, for
    comparison, with the white-noise scale sqrt(w)."""
    _, snr, _ = nb.nbsi_detect(img, want_snr=True, ctx=ctx)
    hp = n_pix // 2
    yy, xx = torch.meshgrid(torch.arange(n_pix, device=img.device), torch.arange(n_pix, device=img.device),
                            indexing="ij")
    hor = ((xx - hp) ** 2 + (yy - hp) ** 2) < hp * hp
    v = snr[:, hor].double()
    v = v - v.mean(dim=0, keepdim=True)
    var = float((v * v).mean())
    rho_meas = [round(float((v[:-l] * v[l:]).mean()) / var, 4) for l in (1, 2, 3)]
    res = nb.nbsi_search(snr, fdr_q=0.01, ctx=ctx, rho=nb.HANN_CROSS_RHO)
    reps = max(2, args.steps // 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = nb.nbsi_search(snr, fdr_q=0.01, ctx=ctx, rho=nb.HANN_CROSS_RHO)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    white = nb.nbsi_search(snr, fdr_q=0.01, ctx=ctx)
    m = int(hor.sum()) * C
    rec, thr, kprov = res[0], res[1], res[2]
    log(f"[bench] stage I search on the step's SNR cube: {ms:.3f} ms, measured rho {rho_meas}, "
        f"k* {kprov} ({kprov / m:.2e} of voxels), {len(rec)} candidates; white-noise scale: k* {white[2]} "
        f"({white[2] / m:.2e}), {len(white[0])} candidates")
    del snr
    torch.cuda.empty_cache()
    return {"workload": f"the step's per-pixel SNR cube ({C} x {n_pix}^2), 26 boxcar widths 1..100, BH q = 0.01, "
                        "channel correlations (4/9, 1/36) of the Hann-windowed cross-correlations",
            "ms": round(ms, 3), "measured_rho_lag1_3": rho_meas, "model_rho": list(nb.HANN_CROSS_RHO),
            "searched_voxels": m, "provisional": kprov, "provisional_fraction": round(kprov / m, 8),
            "threshold_snr": round(thr, 4) if math.isfinite(thr) else None, "candidates": int(len(rec)),
            "white_scale": {"provisional": white[2], "provisional_fraction": round(white[2] / m, 6),
                            "candidates": int(len(white[0]))}}


def dedoppler_leg(args, nb, torch, ctx, dev, C, n_pix):
    """The drift-rate search at the instrument's cube size: 4 sub-integration residual cubes of
    4096 x 256^2 (seeded unit white noise), total drifts -16..16 channels."""
    g = torch.Generator(device=dev)
    g.manual_seed(7101)
    sub = torch.randn((4, C, n_pix, n_pix), generator=g, device=dev)
    best = torch.empty((C, n_pix, n_pix), dtype=torch.float32, device=dev)
    drift = torch.empty((C, n_pix, n_pix), dtype=torch.int8, device=dev)
    ms = _timed(torch, lambda: nb.nbsi_dedoppler(sub, 16, best=best, drift=drift, ctx=ctx), max(3, args.steps // 2))
    vox = C * n_pix * n_pix
    algo = 4 * vox * 4 + vox * 5  # every sub-integration read once, best SNR and drift written
    log(f"[bench] de-Doppler (4 sub-integrations, 33 drifts): {ms:.3f} ms")
    del sub, best, drift
    torch.cuda.empty_cache()
    return {"workload": "4 x 4096 x 256^2 sub-integration cubes, drifts -16..16 channels", "ms": round(ms, 3),
            "track_sums_per_s": round(33 * vox / (ms * 1e-3), 1), "algorithmic_bytes": algo,
            "gbs": round(algo / (ms * 1e-3) / 1e9, 1), "frac_of_hbm": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def calibrated_leg(args, nb, torch, ctx, dev, spec_q, vis, C, n_in, T, nprod):
    """Calibration applied in the correlator epilogue on the step's spectra (complex factors per
    input and channel, float32 output in place of the int32 visibilities), against the plain call."""
    g = torch.Generator(device=dev)
    g.manual_seed(7003)
    cal = torch.randn((C, n_in, 2), generator=g, device=dev)
    vis_f = vis.view(torch.float32)
    ms_cal = _timed(torch, lambda: nb.nbsi_correlate_cal(spec_q, cal, vis=vis_f, ctx=ctx), max(3, args.steps // 2))
    ms_plain = _timed(torch, lambda: nb.nbsi_correlate(spec_q, vis=vis, ctx=ctx), max(3, args.steps // 2))
    cal_bytes = C * (2 * n_in * T) + C * n_in * 8 + C * nprod * 8
    log(f"[bench] calibrated correlator {ms_cal:.3f} ms (plain {ms_plain:.3f} ms)")
    return {"ms": round(ms_cal, 4), "plain_ms": round(ms_plain, 4),
            "gbs": round(cal_bytes / (ms_cal * 1e-3) / 1e9, 1),
            "frac_of_hbm": round(cal_bytes / (ms_cal * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def stage2_leg(args, nb, torch, ctx, dev, C, n_pix, n_cand=4096):
    """Stage II cuts at the instrument's cube size: 4096 x 256^2 unit white noise with n_cand
    beam-shaped (sigma 1.6 x 1.2 px) blobs at seeded sub-pixel positions, a quarter of them 3x
    wider; every blob is a candidate (9 x 9 cutout fits, noise statistics of every channel)."""
    g = torch.Generator(device=dev)
    g.manual_seed(7201)
    cube = torch.randn((C, n_pix, n_pix), generator=g, device=dev)
    rng = np.random.default_rng(7202)
    xs = rng.integers(8, n_pix - 8, n_cand)
    ys = rng.integers(8, n_pix - 8, n_cand)
    cs = rng.integers(0, C, n_cand)
    off = rng.uniform(-0.5, 0.5, (n_cand, 2))
    yy, xx = torch.meshgrid(torch.arange(-5, 6, device=dev, dtype=torch.float64),
                            torch.arange(-5, 6, device=dev, dtype=torch.float64), indexing="ij")
    K = 2.0 * math.sqrt(2.0 * math.log(2.0))
    for i in range(n_cand):
        f = 3.0 if i % 4 == 3 else 1.0
        u, v = xx - off[i, 0], yy - off[i, 1]
        ct, st = math.cos(0.5), math.sin(0.5)
        a, b = (u * ct + v * st) / (1.6 * f), (-u * st + v * ct) / (1.2 * f)
        amp = 8.0 + 32.0 * ((i * 0.6180339887) % 1.0)
        cube[cs[i], ys[i] - 5:ys[i] + 6, xs[i] - 5:xs[i] + 6] += (amp * torch.exp(-0.5 * (a * a + b * b))).float()
    cands = torch.from_numpy(np.stack([xs, ys, cs, np.ones(n_cand), np.zeros(n_cand)], 1).astype(np.int32)).to(dev)
    beam = torch.tensor([[K * 1.6, K * 1.2, 0.5]] * C, dtype=torch.float64, device=dev)
    out = torch.empty((n_cand, 160), dtype=torch.uint8, device=dev)
    ms = _timed(torch, lambda: nb.nbsi_stage2(cube, cands, beam, out=out, ctx=ctx), max(3, args.steps // 2))
    rec = nb.fits_host(out, n_cand)
    kept = int((rec["flags"] == 0).sum())
    log(f"[bench] Stage II ({n_cand} candidates): {ms:.3f} ms, kept {kept}")
    del cube
    torch.cuda.empty_cache()
    return {"workload": f"{C} x {n_pix}^2 cube, {n_cand} candidates (9 x 9 Gaussian fits, FP64)", "ms": round(ms, 3),
            "candidates_per_s": round(n_cand / (ms * 1e-3), 1), "kept": kept,
            "median_iterations": float(np.median(rec["n_iter"])), "max_iterations": int(rec["n_iter"].max())}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    import torch

    import paper_2606_04304_amd as nb
    import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.batch_only:
        print(json.dumps(batched_leg(args, nb, torch, nb.nbsi_create(0), dev, synth)))
        return
    if args.legs_only:
        c0 = nb.nbsi_create(0)
        legs = {"deep_correlator": lambda: deep_correlator_leg(args, nb, torch, c0, dev, synth),
                "classifier": lambda: classifier_leg(args, nb, torch, c0, dev, synth),
                "stage1_search": lambda: search_leg(args, nb, torch, c0, dev, 4096, 256),
                "dedoppler": lambda: dedoppler_leg(args, nb, torch, c0, dev, 4096, 256),
                "stage2": lambda: stage2_leg(args, nb, torch, c0, dev, 4096, 256),
                "precision": lambda: precision_leg(args, nb, torch, c0, dev, synth),
                "c5": lambda: c5_leg(args, nb, torch, c0, dev, synth)}
        names = [args.leg] if args.leg else list(legs)
        print(json.dumps({k: legs[k]() for k in names}))
        return
    cfg = synth.make_config(2)
    log(f"[bench] generating inputs: {cfg.name}")
    xyz = synth.antenna_layout(cfg.n_ant, cfg.radius_m, cfg.seed_base + 1)
    volt = synth.voltages(cfg.n_ant, cfg.n_fft, cfg.n_spec, cfg.tones, xyz, cfg.seed_base + 2,
                          device="cuda")
    freq = synth.channel_freqs(cfg.n_fft, cfg.chan0, cfg.n_chan)
    gain = torch.full((cfg.n_in,), float(cfg.gain), dtype=torch.float32, device=dev)
    n_in, C, T, n_pix = cfg.n_in, cfg.n_chan, cfg.n_spec, cfg.n_pix
    nprod = n_in * (n_in + 1) // 2
    spec_q = torch.empty((C, n_in, 2, T), dtype=torch.int8, device=dev)
    vis = torch.empty((C, nprod, 2), dtype=torch.int32, device=dev)
    img = torch.empty((C, n_pix, n_pix), dtype=torch.float32, device=dev)
    ctx = nb.nbsi_create(0)
    plan = nb.nbsi_image_plan_create(xyz, freq, n_pix, nb.NBSI_IMAGE_GRID, ctx=ctx)
    n_pairs = plan.n_pairs()
    stokes = torch.empty((C, max(1, n_pairs), 2), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log("[bench] inputs ready")

    stage_names = ["channelize", "correlate", "image", "detect"]
    seg_names = ["channelize", "correlate+image", "detect"]

    def mark(ev, k):
        if ev is not None:
            ev[k].record()

    def step(ev=None):
        mark(ev, 0)
        nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, gain, spec_q=spec_q, ctx=ctx)
        mark(ev, 1)
        # correlate and image overlapped over 16 channel ranges on two streams; the correlator
        # also writes Stokes I of the imaged candidate pairs from its epilogue, so the imager
        # does not re-read the visibilities
        nb.nbsi_correlate_image(spec_q, plan, vis=vis, stokes_i=stokes, img=img)
        mark(ev, 2)
        rec, _, n = nb.nbsi_detect(img, ctx=ctx)
        mark(ev, 3)
        return n

    def stage_step(ev=None):
        """The same kernels one stage at a time (the correlator as one launch over every channel),
        so that events bracket each stage on its own."""
        mark(ev, 0)
        nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, gain, spec_q=spec_q, ctx=ctx)
        mark(ev, 1)
        nb.nbsi_correlate_stokes(spec_q, plan, vis=vis, stokes_i=stokes)
        mark(ev, 2)
        nb.nbsi_image_stokes(plan, stokes, img=img)
        mark(ev, 3)
        rec, _, n = nb.nbsi_detect(img, ctx=ctx)
        mark(ev, 4)
        return n

    def corr_only(ev=None):
        mark(ev, 0)
        nb.nbsi_correlate_stokes(spec_q, plan, vis=vis, stokes_i=stokes)
        mark(ev, 1)

    if args.calibrate:
        # a plain copy kernel of known size: 1 GiB read + 1 GiB written per launch
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration done (3 x 1 GiB)")

    run = step if args.stages == "all" else corr_only
    n_ev = 4 if args.stages == "all" else 2
    for i in range(args.warmup):
        run()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(n_ev)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_cand = 0
    for i in range(args.steps):
        n_cand = run(events[i]) or n_cand
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps: {wall * 1e3 / args.steps:.3f} ms/step")
    per = np.array([[events[i][k].elapsed_time(events[i][k + 1]) for k in range(n_ev - 1)]
                    for i in range(args.steps)])  # ms
    ms_step = wall * 1e3 / args.steps
    ops = 8.0 * nprod * T * C
    if args.stages != "all":
        corr_ms = float(per[:, 0].mean())
        print(json.dumps({"correlate_ms": corr_ms, "tops": ops / corr_ms / 1e9}))
        return
    seg_ms = {n: float(per[:, k].mean()) for k, n in enumerate(seg_names)}

    # per-stage pass after the timed region: the same number of steps, one stage at a time
    stage_step()
    torch.cuda.synchronize()
    ev_s = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    t1 = time.perf_counter()
    for i in range(args.steps):
        stage_step(ev_s[i])
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t1) * 1e3 / args.steps
    per_s = np.array([[ev_s[i][k].elapsed_time(ev_s[i][k + 1]) for k in range(4)] for i in range(args.steps)])
    stage_ms = {n: float(per_s[:, k].mean()) for k, n in enumerate(stage_names)}
    log(f"[bench] per-stage pass: {ms_seq:.3f} ms/step")

    # roofline of the correlator: one kernel per call in the per-stage pass, so the events
    # bracket exactly that launch, on the stream the library launches on (torch's current one)
    corr_kernel = nb.nbsi_correlate_kernel(n_in, T)
    # the correlation itself: int8 spectra in, int32 visibilities out; the same launch also writes
    # float32 Stokes I of the imager's candidate pairs (a side output, counted separately)
    corr_bytes = C * (2 * n_in * T) + C * nprod * 8
    side_bytes = C * n_pairs * 8
    achieved = corr_bytes / (stage_ms["correlate"] * 1e-3) / 1e9
    traffic = traffic_from_profile(corr_kernel, "paper_2606_04304_amd/csrc/correlate.hip")
    roofline = {"kernel": corr_kernel, "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": corr_bytes,
                "side_output_bytes_per_launch": side_bytes,
                "frac_with_side_output": round((corr_bytes + side_bytes) / (stage_ms["correlate"] * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4),
                "launch": f"one launch over all {C} channels, timed in the per-stage pass",
                "mfma_frac": round(ops / (stage_ms["correlate"] * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4)}
    # every stage against the HBM roofline with its algorithmic bytes (reads + writes once)
    stage_bytes = {
        # voltages in, int8 spectra out (the staging through context scratch is not counted)
        "channelize": n_in * T * cfg.n_fft * 2 + C * n_in * T * 2,
        "correlate": corr_bytes,
        # Stokes I of every candidate pair in, the image out
        "image": C * n_pairs * 8 + C * n_pix * n_pix * 4,
        "detect": C * n_pix * n_pix * 4,
    }
    stage_roof = {k: {"algorithmic_bytes": int(v), "gbs": round(v / (stage_ms[k] * 1e-3) / 1e9, 1),
                      "frac_of_hbm": round(v / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                  for k, v in stage_bytes.items()}

    comp = {
        "step_segments_ms": {k: round(v, 4) for k, v in seg_ms.items()},
        "per_stage_pass_ms_per_step": round(ms_seq, 4),
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "correlator_tops": round(ops / stage_ms["correlate"] / 1e9, 2),
        "imaged_channels_per_s_imager": round(C / (stage_ms["image"] * 1e-3), 1),
        "imaged_channels_per_s_end_to_end": round(C / (ms_step * 1e-3), 1),
        "candidates": int(n_cand),
        "stokes_candidate_pairs": int(n_pairs),
        "stage_hbm_roofline": stage_roof,
    }

    if args.step_only:
        args.no_search = args.no_fp32_path = args.no_batch = args.no_deep = args.no_classifier = True
        args.no_precision = args.no_c5 = True
    if not args.no_search:
        comp["stage1_search"] = search_leg(args, nb, torch, ctx, dev, C, n_pix)
        comp["stage1_search_pipeline"] = search_pipeline_leg(args, nb, torch, ctx, img, C, n_pix)
        comp["dedoppler"] = dedoppler_leg(args, nb, torch, ctx, dev, C, n_pix)
        comp["stage2"] = stage2_leg(args, nb, torch, ctx, dev, C, n_pix)
    if not args.step_only:
        comp["calibrated_correlator"] = calibrated_leg(args, nb, torch, ctx, dev, spec_q, vis, C, n_in, T, nprod)

    # ---- plain FP32 path on the same GPU: float spectra, FP32 correlator, float vis ----
    if not args.no_fp32_path:
        del spec_q
        spec_f = torch.empty((C, n_in, 2, T), dtype=torch.float32, device=dev)
        vis_f = torch.empty((C, nprod, 2), dtype=torch.float32, device=dev)
        del vis
        torch.cuda.empty_cache()

        def step_f32(ev=None):
            if ev is not None:
                ev[0].record()
            nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, gain, want_q=False, want_f=True,
                               spec_f=spec_f, ctx=ctx)
            if ev is not None:
                ev[1].record()
            nb.nbsi_correlate_f32(spec_f, vis=vis_f, ctx=ctx)
            if ev is not None:
                ev[2].record()
            nb.nbsi_image(plan, vis_f, img=img)
            if ev is not None:
                ev[3].record()
            nb.nbsi_detect(img, ctx=ctx)
            if ev is not None:
                ev[4].record()

        step_f32()
        torch.cuda.synchronize()
        k2 = max(2, args.steps // 2)
        ev2 = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(k2)]
        t1 = time.perf_counter()
        for i in range(k2):
            step_f32(ev2[i])
        torch.cuda.synchronize()
        wall2 = (time.perf_counter() - t1) * 1e3 / k2
        per2 = np.array([[ev2[i][k].elapsed_time(ev2[i][k + 1]) for k in range(4)] for i in range(k2)])
        s2 = {n: float(per2[:, k].mean()) for k, n in enumerate(stage_names)}
        comp["fp32_path"] = {
            "ms_per_step": round(wall2, 3), "stage_ms": {k: round(v, 4) for k, v in s2.items()},
            "correlator_tops": round(ops / s2["correlate"] / 1e9, 2),
            "imaged_channels_per_s_imager": round(C / (s2["image"] * 1e-3), 1),
            "tops_end_to_end": round(ops / wall2 / 1e9, 3),
        }
        comp["speedup_vs_fp32_path"] = {
            "end_to_end": round(wall2 / ms_step, 3),
            "correlator": round(s2["correlate"] / stage_ms["correlate"], 3),
            "channelize": round(s2["channelize"] / stage_ms["channelize"], 3),
        }
        log("[bench] fp32 path timed")

    if not args.no_batch:
        comp["batched_subbands"] = batched_leg(args, nb, torch, ctx, dev, synth)
        torch.cuda.empty_cache()
    if not args.no_deep:
        comp["deep_correlator"] = deep_correlator_leg(args, nb, torch, ctx, dev, synth)
    if not args.no_classifier:
        comp["classifier"] = classifier_leg(args, nb, torch, ctx, dev, synth)
        torch.cuda.empty_cache()
    if not args.no_precision:
        comp["precision_c4"] = precision_leg(args, nb, torch, ctx, dev, synth)
        torch.cuda.empty_cache()
    if not args.no_c5:
        comp["classifier_c5"] = c5_leg(args, nb, torch, ctx, dev, synth)
        torch.cuda.empty_cache()

    out = {
        "metric": "correlated fine-channel TOPS + imaged channels/s @256^2 vs plain FP32 path",
        "value": round(ops / (ms_step * 1e-3) / 1e12, 4),
        "unit": "TOPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8->int32 correlate, f32 channelize/image/detect",
        "data": "synthetic",
        "config": {"workload": "instrument scale: 352 ant x 2 pol, 65536-pt channelizer, T=32, "
                               "4096 channels, GRID 256^2, 5 sigma per-pixel detect",
                   "n_inputs": n_in, "n_fft": cfg.n_fft, "n_spec": T, "n_chan": C, "n_pix": n_pix,
                   "products": nprod},
        "roofline": roofline,
        "components": comp,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        q_tmp = torch.empty((C, n_in, 2, T), dtype=torch.int8, device=dev)
        nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, gain, spec_q=q_tmp, ctx=ctx)
        torch.cuda.synchronize()
        out["cpu_baseline"] = cpu_baseline(cfg, xyz, freq, volt, cfg.gain, q_tmp, img)
        out["cpu_baseline"]["vs_gpu"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
