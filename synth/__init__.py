"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no step of the method: it only draws antenna layouts, complex int8
voltages with injected narrowband tones, and the configuration constants that both the
oracle and the HIP path receive as plain inputs.  It stands in for the instrument's
post-PFB voltage dump of the paper's Sec. 2.1 (one 30 s OVRO-LWA epoch), which is not
available here.

Workload shapes follow the five configurations of the build (tiny plain method,
instrument scale, uneven sub-bands, precision study, learned classifier):

* antennas: 16 or 352 dual-polarisation antennas, uniform in a disk (Sec. 1 gives the
  array as 352 antennas with a ~200 m core and baselines up to 2.4 km);
* voltages: complex int8, Gaussian sigma = 8 per component, clipped to +-127;
* tones: on-bin narrowband carriers from a point source at (l0, m0), with the
  geometric phase of a plane wave across the array.

Conventions (also listed as readings in the design notes):
* input i belongs to antenna a = i // 2, polarisation i % 2 (0 = X, 1 = Y);
* a voltage stream is [n_inputs][n_spec * n_fft][2] int8, (re, im) interleaved;
* fine channel c of an n_fft-point channelizer has baseband offset (c - n_fft/2)*f_s/n_fft
  and sky frequency nu0 + that offset (f_s = 23.9 kHz coarse channel, Sec. 2.1);
* a tone at baseband bin k0 (signed) multiplies antenna a by exp(+2 pi i nu (x_a l0 + y_a m0)/c),
  so that visibilities x_i conj(x_j) carry exp(+2 pi i (u l0 + v m0)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299_792_458.0      # m/s
F_COARSE = 23_900.0          # Hz, coarse (F-engine) channel width, "about 23.9 kHz" (Sec. 2.1)
NU0 = 70.0e6                 # Hz, representative sky frequency of the coarse channel
SIGMA = 8.0                  # voltage noise per component, LSB


@dataclass
class Tone:
    k0: int          # signed baseband bin in [-n_fft/2, n_fft/2)
    amp: float       # amplitude per component, LSB
    l0: float
    m0: float


@dataclass
class Config:
    name: str
    n_ant: int
    radius_m: float
    n_fft: int
    n_spec: int
    chan0: int
    n_chan: int
    n_pix: int
    method: str                 # "dft" or "grid"
    tones: list = field(default_factory=list)
    sigma: float = SIGMA
    seed_base: int = 1000
    gain: float = 0.0           # requantisation gain (float32 value), per input identical

    @property
    def n_in(self) -> int:
        return 2 * self.n_ant


def antenna_layout(n_ant: int, radius_m: float, seed: int) -> np.ndarray:
    """Positions uniform in a disk of the given radius, z = 0.  Returns [n_ant, 3] float64 metres."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u1 = rng.random(n_ant)
    u2 = rng.random(n_ant)
    r = radius_m * np.sqrt(u1)
    th = 2.0 * np.pi * u2
    xyz = np.zeros((n_ant, 3), dtype=np.float64)
    xyz[:, 0] = r * np.cos(th)
    xyz[:, 1] = r * np.sin(th)
    return xyz


def channel_freqs(n_fft: int, chan0: int, n_chan: int, nu0: float = NU0,
                  f_s: float = F_COARSE) -> np.ndarray:
    """Sky frequency of fine channels chan0 .. chan0+n_chan-1 (float64 Hz)."""
    c = np.arange(chan0, chan0 + n_chan, dtype=np.float64)
    return nu0 + (c - n_fft / 2) * (f_s / n_fft)


def tone_sky_freq(k0: int, n_fft: int, nu0: float = NU0, f_s: float = F_COARSE) -> float:
    return nu0 + k0 * (f_s / n_fft)


def hann_power_gain(n_fft: int) -> float:
    """Sum of squares of the periodic Hann window, 3N/8 (a config constant for gains)."""
    return 3.0 * n_fft / 8.0


def gain_loud_tone(n_fft: int, amp: float, sigma: float) -> np.float32:
    """Gain that maps a tone of amplitude `amp` plus 5 sigma of noise to 127 LSB."""
    return np.float32(127.0 / (amp * n_fft / 2 + 5.0 * sigma * math.sqrt(hann_power_gain(n_fft))))


def gain_noise(n_fft: int, sigma: float, target: float = 8.0) -> np.float32:
    """Gain that maps the per-component channel noise to `target` LSB rms."""
    return np.float32(target / (sigma * math.sqrt(hann_power_gain(n_fft))))


def approx_n_baselines_in_grid(ant_xyz: np.ndarray, nu: float, n_pix: int) -> int:
    """Rough count of baselines inside the gridding uv box, used only to size tone amplitudes."""
    u_max = (2 * n_pix / 2 - 4 - 1) * 0.25
    a, b = np.tril_indices(ant_xyz.shape[0], -1)
    u = (ant_xyz[a, 0] - ant_xyz[b, 0]) * nu / C_LIGHT
    v = (ant_xyz[a, 1] - ant_xyz[b, 1]) * nu / C_LIGHT
    return int(np.count_nonzero((np.abs(u) <= u_max) & (np.abs(v) <= u_max)))


def tone_amp_for_snr(snr: float, n_fft: int, n_spec: int, n_b: int, sigma: float) -> float:
    """Amplitude whose expected width-1 image SNR is `snr`: SNR = 2 sqrt(T N_b) A^2 N / (3 sigma^2)."""
    return math.sqrt(snr * 3.0 * sigma ** 2 / (2.0 * n_fft * math.sqrt(n_spec * n_b)))


def random_tones(n_tones: int, n_fft: int, chan0: int, n_chan: int, snr_lo: float, snr_hi: float,
                 ant_xyz: np.ndarray, n_spec: int, n_pix: int, seed: int, sigma: float = SIGMA,
                 edge: int = 17) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    tones = []
    used = set()
    while len(tones) < n_tones:
        c = int(rng.integers(chan0 + edge, chan0 + n_chan - edge))
        if any(abs(c - u) < 3 for u in used):
            continue
        while True:
            l0, m0 = rng.uniform(-0.9, 0.9, size=2)
            if l0 * l0 + m0 * m0 < 0.81:
                break
        snr = float(rng.uniform(snr_lo, snr_hi))
        k0 = c - n_fft // 2
        nb = approx_n_baselines_in_grid(ant_xyz, tone_sky_freq(k0, n_fft), n_pix)
        tones.append(Tone(k0=k0, amp=tone_amp_for_snr(snr, n_fft, n_spec, nb, sigma),
                          l0=float(l0), m0=float(m0)))
        used.add(c)
    return tones


def make_config(k: int) -> Config:
    """Configurations 1, 2 and 4 (the uneven-sub-band set is built by `subband_configs`)."""
    if k == 1:
        n_fft = 4096
        c_tone = n_fft // 2 + 256
        cfg = Config("tiny: 16 ant x 2 pol, 4096-pt, T=16, 64 ch, DFT 64^2", 16, 100.0, n_fft, 16,
                     c_tone - 32, 64, 64, "dft", seed_base=1000)
        cfg.tones = [Tone(k0=256, amp=4.0, l0=0.2, m0=-0.1)]
        cfg.gain = gain_loud_tone(n_fft, 4.0, SIGMA)
        return cfg
    if k == 2:
        n_fft = 65536
        cfg = Config("instrument: 352 ant x 2 pol, 65536-pt, T=32, 4096 ch, GRID 256^2", 352, 750.0,
                     n_fft, 32, n_fft // 2 - 2048, 4096, 256, "grid", seed_base=2000)
        xyz = antenna_layout(cfg.n_ant, cfg.radius_m, cfg.seed_base + 1)
        cfg.tones = random_tones(8, n_fft, cfg.chan0, cfg.n_chan, 3.0, 20.0, xyz, cfg.n_spec,
                                 cfg.n_pix, cfg.seed_base + 3)
        cfg.gain = gain_noise(n_fft, SIGMA)
        return cfg
    if k == 4:
        n_fft = 1 << 18
        cfg = Config("precision: 352 ant x 2 pol, 2^18-pt, T=8, 16384 ch, GRID 512^2", 352, 750.0,
                     n_fft, 8, n_fft // 2 - 8192, 16384, 512, "grid", seed_base=4000)
        xyz = antenna_layout(cfg.n_ant, cfg.radius_m, cfg.seed_base + 1)
        cfg.tones = random_tones(8, n_fft, cfg.chan0, cfg.n_chan, 3.0, 20.0, xyz, cfg.n_spec,
                                 cfg.n_pix, cfg.seed_base + 3)
        cfg.gain = gain_noise(n_fft, SIGMA)
        return cfg
    raise ValueError(f"no configuration {k}")


SUBBAND_NT = [(1 << 14, 128), (1 << 15, 64), (1 << 16, 32), (1 << 17, 16), (1 << 18, 8)]
SUBBAND_NPIX = [128, 256, 512]


def subband_configs(n_sub: int = 12, n_chan: int = 1024, n_ant: int = 352):
    """Uneven sub-bands: (N, T) and image size cycle; every sub-band holds 2^21 samples per input."""
    out = []
    for s in range(n_sub):
        n_fft, n_spec = SUBBAND_NT[s % len(SUBBAND_NT)]
        out.append(dict(n_fft=n_fft, n_spec=n_spec, chan0=n_fft // 2 - n_chan // 2, n_chan=n_chan,
                        n_pix=SUBBAND_NPIX[s % len(SUBBAND_NPIX)],
                        nu0=NU0 + (s - 6) * F_COARSE, gain=gain_noise(n_fft, SIGMA)))
    return out


def _tone_phasors(tones, ant_xyz, n_fft, nu0):
    """Per antenna complex gain of each tone (geometric phase), float64 [n_tones, n_ant]."""
    ph = []
    for t in tones:
        nu = tone_sky_freq(t.k0, n_fft, nu0)
        turns = nu * (ant_xyz[:, 0] * t.l0 + ant_xyz[:, 1] * t.m0) / C_LIGHT
        ph.append(np.exp(2j * np.pi * turns))
    return np.array(ph) if ph else np.zeros((0, ant_xyz.shape[0]), np.complex128)


def voltages(n_ant: int, n_fft: int, n_spec: int, tones, ant_xyz: np.ndarray, seed: int,
             sigma: float = SIGMA, device: str = "cpu", nu0: float = NU0, noise: bool = True,
             block_inputs: int = 32):
    """Complex int8 voltages [2*n_ant, n_spec*n_fft, 2] as a torch tensor on `device`.

    noise + tones are summed in float64, rounded half-to-even once and clipped to +-127.
    The noise comes from torch's generator for `device` seeded with `seed` (Philox on GPU,
    Mersenne Twister on CPU), drawn block by block over inputs.
    """
    import torch
    n_in = 2 * n_ant
    n_samp = n_spec * n_fft
    out = torch.empty((n_in, n_samp, 2), dtype=torch.int8, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    ph = _tone_phasors(tones, ant_xyz, n_fft, nu0)
    n = torch.arange(n_fft, device=device, dtype=torch.float64)
    carriers = []
    for t in tones:
        arg = (2.0 * math.pi / n_fft) * ((t.k0 % n_fft) * n % n_fft)
        carriers.append((t.amp * torch.cos(arg), t.amp * torch.sin(arg)))
    for i0 in range(0, n_in, block_inputs):
        i1 = min(n_in, i0 + block_inputs)
        if noise:
            x = torch.randn((i1 - i0, n_samp, 2), generator=gen, device=device, dtype=torch.float64)
            x.mul_(sigma)
        else:
            x = torch.zeros((i1 - i0, n_samp, 2), device=device, dtype=torch.float64)
        if tones:
            xv = x.view(i1 - i0, n_spec, n_fft, 2)
            ants = np.arange(i0, i1) // 2
            for ti, (cr, ci) in enumerate(carriers):
                g = ph[ti, ants]
                gr = torch.tensor(g.real, device=device, dtype=torch.float64)[:, None, None]
                gi = torch.tensor(g.imag, device=device, dtype=torch.float64)[:, None, None]
                xv[..., 0] += cr[None, None, :] * gr - ci[None, None, :] * gi
                xv[..., 1] += cr[None, None, :] * gi + ci[None, None, :] * gr
        torch.round(x, out=x)
        x.clamp_(-127.0, 127.0)
        out[i0:i1] = x.to(torch.int8)
        del x
    return out


def config_inputs(cfg: Config, device: str = "cpu", noise: bool = True):
    """Antenna positions, voltages, channel sky frequencies and per-input gains for a config."""
    xyz = antenna_layout(cfg.n_ant, cfg.radius_m, cfg.seed_base + 1)
    volt = voltages(cfg.n_ant, cfg.n_fft, cfg.n_spec, cfg.tones, xyz, cfg.seed_base + 2,
                    cfg.sigma, device=device, noise=noise)
    freq = channel_freqs(cfg.n_fft, cfg.chan0, cfg.n_chan)
    gain = np.full(cfg.n_in, cfg.gain, dtype=np.float32)
    return xyz, volt, freq, gain


def random_spectra(n_chan: int, n_in: int, n_spec: int, seed: int, sigma_q: float = 8.0,
                   device: str = "cpu", full_range: bool = False):
    """Random int8 correlator inputs [n_chan][n_in][2][n_spec] (Gaussian sigma_q, clipped +-127;
    or uniform over [-128, 127] when full_range)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    if full_range:
        return torch.randint(-128, 128, (n_chan, n_in, 2, n_spec), generator=gen,
                             device=device, dtype=torch.int16).to(torch.int8)
    x = torch.randn((n_chan, n_in, 2, n_spec), generator=gen, device=device) * sigma_q
    return torch.round(x).clamp_(-127, 127).to(torch.int8)


# ---------------------------------------------------------------------------------------------
# Learned-classifier inputs: initial weights and injected sky tones, RFI and broadband spikes
# ---------------------------------------------------------------------------------------------
NET_SHAPES = [(32, 33), (64, 32), (32, 64)]  # (out, in) channels of the three 3 x 3 convolutions


def net_init(seed: int) -> np.ndarray:
    """Initial classifier parameters (flat float32, the documented order): convolution and
    linear weights uniform in +-sqrt(6 / fan_in) (He), biases zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for co, ci in NET_SHAPES:
        lim = math.sqrt(6.0 / (ci * 9))
        parts.append(rng.uniform(-lim, lim, size=co * ci * 9))
        parts.append(np.zeros(co))
    parts.append(rng.uniform(-math.sqrt(6.0 / 32), math.sqrt(6.0 / 32), size=32))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


@dataclass
class Source:
    c: int        # fine channel
    l: float
    m: float
    amp: float    # image-plane peak (visibility amplitude on every baseline)


KIND_TONE, KIND_RFI, KIND_SPIKE, KIND_NOISE = 0, 1, 2, 3


def pixel_lm(x: float, y: float, n_pix: int):
    return (x - n_pix / 2) * 2.0 / n_pix, (y - n_pix / 2) * 2.0 / n_pix


def classifier_scene(rng: np.random.Generator, n_chan: int, n_pix: int, sigma_img: float,
                     n_tone: int, n_rfi: int, n_spike: int):
    """Random injections for one cube, as (kind, centre (c, x, y), [Source]) triples.

    * tone: one channel, a point source anywhere with l^2 + m^2 < 0.8^2, SNR 5-20;
    * RFI: near the horizon (0.88 < sqrt(l^2 + m^2) < 0.96), 3-6 point components within
      2.5 pixels of a centre, present in 1-8 consecutive channels and drifting by 0.5-1.5
      pixels per channel, SNR 6-30 per component;
    * broadband spike: one point source anywhere with l^2 + m^2 < 0.9^2 in 12-33 consecutive
      channels at a steady SNR 6-20.
    Injections keep 40 channels or 12 pixels from each other so stamps do not mix them."""
    taken = []

    def free(c0, c1, x, y):
        for (a0, a1, xx, yy) in taken:
            if c0 <= a1 + 40 and a0 <= c1 + 40 and abs(x - xx) < 12 and abs(y - yy) < 12:
                return False
        return 20 <= c0 and c1 < n_chan - 20

    out = []

    def place(kind, n_ch, r_lo, r_hi):
        for _ in range(200):
            c0 = int(rng.integers(20, n_chan - 20 - n_ch))
            r = math.sqrt(rng.uniform(r_lo * r_lo, r_hi * r_hi))
            th = rng.uniform(0, 2 * math.pi)
            x = n_pix / 2 + r * math.cos(th) * n_pix / 2
            y = n_pix / 2 + r * math.sin(th) * n_pix / 2
            if free(c0, c0 + n_ch - 1, x, y):
                taken.append((c0, c0 + n_ch - 1, x, y))
                return c0, x, y
        return None

    for _ in range(n_tone):
        p = place(KIND_TONE, 1, 0.0, 0.8)
        if p:
            c0, x, y = p
            l, m = pixel_lm(x, y, n_pix)
            out.append((KIND_TONE, (c0, x, y), [Source(c0, l, m, rng.uniform(5, 20) * sigma_img)]))
    for _ in range(n_rfi):
        n_ch = int(rng.integers(1, 9))
        p = place(KIND_RFI, n_ch, 0.88, 0.96)
        if p:
            c0, x, y = p
            comps = [(rng.uniform(-2.5, 2.5), rng.uniform(-2.5, 2.5), rng.uniform(6, 30))
                     for _ in range(int(rng.integers(3, 7)))]
            th = rng.uniform(0, 2 * math.pi)
            step = rng.uniform(0.5, 1.5)
            srcs = []
            for k in range(n_ch):
                for (dx, dy, snr) in comps:
                    l, m = pixel_lm(x + dx + k * step * math.cos(th), y + dy + k * step * math.sin(th), n_pix)
                    srcs.append(Source(c0 + k, l, m, snr * sigma_img))
            out.append((KIND_RFI, (c0, x, y), srcs))
    for _ in range(n_spike):
        n_ch = int(rng.integers(12, 34))
        p = place(KIND_SPIKE, n_ch, 0.0, 0.9)
        if p:
            c0, x, y = p
            l, m = pixel_lm(x, y, n_pix)
            amp = rng.uniform(6, 20) * sigma_img
            out.append((KIND_SPIKE, (c0, x, y), [Source(c0 + k, l, m, amp) for k in range(n_ch)]))
    return out


def add_sources(vis_f, ant_xyz: np.ndarray, freq: np.ndarray, sources, chunk: int = 64):
    """Add point sources to float32 visibilities vis_f [n_chan][n_in (n_in+1)/2][2] (torch, in
    place): the XX and YY products of every antenna pair a > b receive
    amp exp(+2 pi i nu ((x_a - x_b) l + (y_a - y_b) m) / c), the autocorrelations amp."""
    import torch
    dev = vis_f.device
    n_ant = ant_xyz.shape[0]
    a, b = np.tril_indices(n_ant)          # a >= b
    dx = torch.tensor(ant_xyz[a, 0] - ant_xyz[b, 0], dtype=torch.float64, device=dev)
    dy = torch.tensor(ant_xyz[a, 1] - ant_xyz[b, 1], dtype=torch.float64, device=dev)
    idx = []
    for p in (0, 1):
        i, j = 2 * a + p, 2 * b + p
        idx.append(torch.tensor(i * (i + 1) // 2 + j, dtype=torch.long, device=dev))
    # sources sharing a channel go to different passes, so no pass adds twice to one product
    # (the sums are then independent of scheduling)
    passes, seen = [], {}
    for src in sources:
        k = seen.get(src.c, 0)
        seen[src.c] = k + 1
        while len(passes) <= k:
            passes.append([])
        passes[k].append(src)
    flat = vis_f.view(-1, 2)
    for group in passes:
        for s0 in range(0, len(group), chunk):
            grp = group[s0:s0 + chunk]
            ch = torch.tensor([s.c for s in grp], dtype=torch.long, device=dev)
            nu = torch.tensor([freq[s.c] for s in grp], dtype=torch.float64, device=dev)
            l = torch.tensor([s.l for s in grp], dtype=torch.float64, device=dev)
            m = torch.tensor([s.m for s in grp], dtype=torch.float64, device=dev)
            amp = torch.tensor([s.amp for s in grp], dtype=torch.float64, device=dev)
            turns = (nu / C_LIGHT)[:, None] * (dx[None, :] * l[:, None] + dy[None, :] * m[:, None])
            turns = turns - torch.floor(turns)
            upd = torch.stack([amp[:, None] * torch.cos(2 * math.pi * turns),
                               amp[:, None] * torch.sin(2 * math.pi * turns)], dim=-1).float()
            for ix in idx:
                rows = (ch[:, None] * vis_f.shape[1] + ix[None, :]).reshape(-1)
                flat.index_copy_(0, rows, flat.index_select(0, rows) + upd.reshape(-1, 2))


def elliptical_blob(n_pix: int, x0: float, y0: float, amp: float, sigma_maj: float, sigma_min: float,
                    theta: float) -> np.ndarray:
    """[n_pix][n_pix] float64 image of an elliptical Gaussian blob: peak amp at (x0, y0) (x =
    column, y = row), standard deviations sigma_maj along the direction at angle theta from the
    +x axis (towards +y) and sigma_min across it."""
    y, x = np.mgrid[0:n_pix, 0:n_pix].astype(np.float64)
    u = (x - x0) * math.cos(theta) + (y - y0) * math.sin(theta)
    v = -(x - x0) * math.sin(theta) + (y - y0) * math.cos(theta)
    return amp * np.exp(-0.5 * (u / sigma_maj) ** 2 - 0.5 * (v / sigma_min) ** 2)


@dataclass
class Blob:
    c: int
    x: float
    y: float
    amp: float
    sigma_maj: float
    sigma_min: float
    theta: float
    extended: bool


def stage2_scene(rng: np.random.Generator, n_chan: int, n_pix: int, beam_sigma=(1.6, 1.2, 0.5),
                 n_point: int = 24, n_ext: int = 8, noisy=(), snr=(8.0, 40.0)):
    """A float32 image cube [n_chan][n_pix][n_pix] of unit white noise (sigma 1; the channels in
    noisy get sigma 3, or 0.3 for a negative entry -c - 1) with n_point beam-shaped blobs
    (beam_sigma = (sigma_maj, sigma_min, theta) in pixels and radians) and n_ext blobs 2.5-4
    times wider, at random sub-pixel positions at least 8 pixels inside the image, peaks
    snr[0]..snr[1] times the channel noise; blobs keep 12 pixels apart within a channel.
    Returns (cube, blobs)."""
    cube = rng.standard_normal((n_chan, n_pix, n_pix))
    sig = np.ones(n_chan)
    for c in noisy:
        if c >= 0:
            sig[c] = 3.0
        else:
            sig[-c - 1] = 0.3
    cube *= sig[:, None, None]
    blobs, taken = [], []
    for k in range(n_point + n_ext):
        ext = k >= n_point
        for _ in range(200):
            c = int(rng.integers(0, n_chan))
            x, y = rng.uniform(8, n_pix - 9), rng.uniform(8, n_pix - 9)
            if all(cc != c or math.hypot(x - xx, y - yy) >= 12 for (cc, xx, yy) in taken):
                break
        taken.append((c, x, y))
        f = rng.uniform(2.5, 4.0) if ext else 1.0
        th = rng.uniform(0, math.pi) if ext else beam_sigma[2]
        b = Blob(c, x, y, rng.uniform(*snr) * sig[c], beam_sigma[0] * f, beam_sigma[1] * f, th, ext)
        cube[c] += elliptical_blob(n_pix, b.x, b.y, b.amp, b.sigma_maj, b.sigma_min, b.theta)
        blobs.append(b)
    return cube.astype(np.float32), blobs
