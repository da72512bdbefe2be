"""Throughput of the hot path on one MI355X: channelize -> correlate -> image -> detect.

Workload: 352 dual-polarisation antennas (704 inputs, 248,160 correlation products) in a
1.5 km disk, complex int8 voltages (sigma = 8) with 8 injected tones, a 65,536-point Hann
channelizer keeping 4,096 channels, 32 spectra integrated, int8 -> int32 correlation, FP32
gridding + 2D FFT to 256 x 256 all-sky images, 5 sigma per-pixel spectral detection.
Inputs are synthetic (seeded) and resident in HBM before timing starts.

A step is one pass of all four stages over one dump.  The JSON line reports
  value = useful correlation ops of the step / step time (TOPS, 8 ops per complex MAC),
and, in "components", the correlator-only TOPS, the imaged channels/s (imager only and end
to end), and the same figures for the plain FP32 path (float32 spectra, FP32 correlator,
float32 visibilities into the same imager) timed on the same GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-path", action="store_true")
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


def traffic_from_profile(kernel_src, launch_algo_bytes):
    """HBM bytes per launch from the committed counter summary, if it was taken on this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    ent = d.get(kernel_src["name"])
    if not ent or ent.get("source_sha") != source_digest(kernel_src["files"]):
        return None
    return ent.get("hbm_bytes_per_launch")


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
    return {"value": ops / step / 1e12, "unit": "TOPS", "cores": threads, "kind": "oracle",
            "sample": ("channelize 2/704 inputs x 32 spectra (x352); correlate 32/4096 channels "
                       "(x128); direct-Fourier image 1/4096 channels at 256^2 over the gridded "
                       "baseline set (x4096); detect SNR on 4/256 image rows (x64); summed"),
            "stage_seconds": {k: round(v, 3) for k, v in t.items()}, "step_seconds": round(step, 3)}


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
    torch.cuda.synchronize()
    log("[bench] inputs ready")

    stage_names = ["channelize", "correlate", "image", "detect"]

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        nb.nbsi_channelize(volt, cfg.n_fft, T, cfg.chan0, C, gain, spec_q=spec_q, ctx=ctx)
        if ev is not None:
            ev[1].record()
        nb.nbsi_correlate(spec_q, vis=vis, ctx=ctx)
        if ev is not None:
            ev[2].record()
        nb.nbsi_image(plan, vis, img=img)
        if ev is not None:
            ev[3].record()
        rec, _, n = nb.nbsi_detect(img, ctx=ctx)
        if ev is not None:
            ev[4].record()
        return n

    def corr_only(ev=None):
        if ev is not None:
            ev[0].record()
        nb.nbsi_correlate(spec_q, vis=vis, ctx=ctx)
        if ev is not None:
            ev[1].record()

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
    n_ev = 5 if args.stages == "all" else 2
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
    names = stage_names if args.stages == "all" else ["correlate"]
    stage_ms = {n: float(per[:, k].mean()) for k, n in enumerate(names)}
    if args.stages != "all":
        print(json.dumps({"correlate_ms": stage_ms["correlate"], "tops": ops / stage_ms["correlate"] / 1e9}))
        return

    # roofline of the correlator (one kernel per call: the events bracket exactly that launch)
    corr_bytes = C * (2 * n_in * T) + C * nprod * 8          # int8 spectra in + int32 vis out
    achieved = corr_bytes / (stage_ms["correlate"] * 1e-3) / 1e9
    corr_src = {"name": "correlate_i8_kernel", "files": ["paper_2606_04304_amd/csrc/correlate.hip"]}
    traffic = traffic_from_profile(corr_src, corr_bytes)
    roofline = {"kernel": "correlate_i8_kernel", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": corr_bytes,
                "mfma_frac": round(ops / (stage_ms["correlate"] * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4)}

    comp = {
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "correlator_tops": round(ops / stage_ms["correlate"] / 1e9, 2),
        "imaged_channels_per_s_imager": round(C / (stage_ms["image"] * 1e-3), 1),
        "imaged_channels_per_s_end_to_end": round(C / (ms_step * 1e-3), 1),
        "candidates": int(n_cand),
    }

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
