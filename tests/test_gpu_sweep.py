"""GPU parity over seeded random shapes: the channelizer (every transform size from 256 to 2^18
points, bands anywhere in the spectrum, 1 to 16,384 channels), the correlator (1 to 420 inputs,
1 to 400 spectra: whole-channel and tiled kernels, repacked rows), the detector (12 to 6,000
channels, both noise models) and the gridded imager; then the correlator's Stokes-I epilogue
and its overlap with imaging, the tiled correlator up to 800 inputs and 1,100 spectra,
de-Doppler, the Stage I boxcar bank, the whole Stage I search (random FDR levels and noise
widths) and the Stage II fits, the calibrated and the FP32 correlators, and the batch runner over
random sub-band sets; each against the oracle (or the separate calls it must equal) with the fixed
cases' own checks and bars.  The shapes come from
fixed seeds, so the cases are the same on every run."""
import math
import random

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402
import test_gpu_batch as tb  # noqa: E402
import test_gpu_calibrate as tca  # noqa: E402
import test_gpu_drift as tdr  # noqa: E402
import test_gpu_parity as tp  # noqa: E402
import test_gpu_search as tse  # noqa: E402
import test_gpu_stage2 as ts2  # noqa: E402


def _shapes(seed):
    rng = random.Random(seed)
    chan, corr, det, img = [], [], [], []
    for _ in range(28):
        n = 1 << rng.randint(8, 18)
        c = min(rng.choice([1, 2, 3, rng.randint(1, 64), rng.randint(1, min(n, 16384)), min(n, 4096),
                            min(n, 16384)]), n, 16384)
        c0 = rng.randint(0, n - c)
        n_in = rng.randint(1, 3)
        t = rng.randint(1, 3) if n >= 65536 else rng.randint(1, 20)
        chan.append((n_in, n, t, c0, c))
    for _ in range(24):
        n_in = rng.choice([rng.randint(1, 40), rng.randint(40, 200), rng.randint(200, 420)])
        t = rng.choice([rng.randint(1, 32), rng.randint(33, 64), rng.randint(65, 400)])
        corr.append((rng.randint(1, 12) if n_in * t < 40000 else rng.randint(1, 3), n_in, t))
    for _ in range(16):
        n_chan = rng.choice([rng.randint(12, 200), rng.randint(200, 4096), rng.randint(4097, 6000)])
        det.append((n_chan, 8 * rng.randint(2, 8),
                    rng.choice([nb.NBSI_DETECT_PER_PIXEL, nb.NBSI_DETECT_PER_IMAGE])))
    for _ in range(6):
        n_pix = rng.choice([64, 128, 256])
        img.append((n_pix, rng.randint(12, 80), rng.uniform(0.8, 1.6) * n_pix))
    return chan, corr, det, img


CHAN, CORR, DET, IMG = _shapes(1)


@pytest.mark.parametrize("n_in,n_fft,n_spec,chan0,n_chan", CHAN)
def test_sweep_channelize(n_in, n_fft, n_spec, chan0, n_chan):
    tp.test_channelize_matches_oracle(n_in, n_fft, n_spec, chan0, n_chan)


@pytest.mark.parametrize("n_chan,n_in,n_spec", CORR)
def test_sweep_correlate(n_chan, n_in, n_spec):
    tp.test_correlate_bit_exact(n_chan, n_in, n_spec)


@pytest.mark.parametrize("n_chan,n_pix,mode", DET)
def test_sweep_detect(n_chan, n_pix, mode):
    tp.detect_parity(n_chan, n_pix, mode)


@pytest.mark.parametrize("n_pix,n_ant,radius", IMG)
def test_sweep_image_grid(n_pix, n_ant, radius):
    tp.test_image_grid_matches_dft_oracle(n_pix, n_ant, radius)


def _shapes2(seed):
    rng = random.Random(seed)
    stokes, overlap, tiled, drift, bank, fits = [], [], [], [], [], []
    for _ in range(10):
        n_pix = rng.choice([64, 128, 256])
        stokes.append((rng.randint(3, 90), rng.choice([rng.randint(1, 32), rng.randint(33, 64), rng.randint(65, 320)]),
                       rng.randint(1, 13), n_pix, rng.uniform(0.5, 1.5) * n_pix))
    for _ in range(6):
        overlap.append((rng.randint(3, 48), rng.choice([rng.randint(1, 32), rng.randint(33, 130)]),
                        rng.choice([64, 128, 256, 512]), rng.randint(1, 40)))
    for _ in range(8):
        tiled.append((rng.randint(1, 20), rng.randint(30, 800), rng.randint(65, 1100)))
    for _ in range(8):
        drift.append((rng.randint(1, 8), rng.randint(16, 500), 8 * rng.randint(1, 5), rng.randint(0, 16)))
    for _ in range(6):
        bank.append((rng.randint(60, 900), 8 * rng.randint(2, 6)))
    for _ in range(5):
        fits.append((rng.randint(1, 1000), rng.randint(8, 50), rng.choice([48, 64, 96, 128]), rng.randint(2, 5)))
    return stokes, overlap, tiled, drift, bank, fits


STOKES, OVERLAP, TILED, DRIFT, BANK, FITS = _shapes2(1)


@pytest.mark.parametrize("n_ant,n_spec,n_chan,n_pix,radius", STOKES)
def test_sweep_correlate_stokes(n_ant, n_spec, n_chan, n_pix, radius):
    tp.stokes_parity(n_ant, n_spec, n_chan, n_pix, radius)


@pytest.mark.parametrize("n_ant,n_spec,n_pix,n_chan", OVERLAP)
def test_sweep_correlate_image_overlapped(n_ant, n_spec, n_pix, n_chan):
    tp.test_correlate_image_overlapped_matches_sequential(n_ant, n_spec, n_pix, n_chan)


@pytest.mark.parametrize("n_chan,n_in,n_spec", TILED)
def test_sweep_correlate_tiled(n_chan, n_in, n_spec):
    tp.test_correlate_tiled_sampled_channels_bit_exact(n_chan, n_in, n_spec)


@pytest.mark.parametrize("n_sub,n_chan,n_pix,max_drift", DRIFT)
def test_sweep_dedoppler(n_sub, n_chan, n_pix, max_drift):
    tdr.test_dedoppler_matches_oracle(n_sub, n_chan, n_pix, max_drift)


@pytest.mark.parametrize("n_chan,n_pix", BANK)
def test_sweep_search_bank(n_chan, n_pix):
    tse.test_bank_matches_oracle(n_chan, n_pix)


@pytest.mark.parametrize("seed,n_chan,n_pix,half", FITS)
def test_sweep_stage2(seed, n_chan, n_pix, half):
    ts2.test_stage2_matches_oracle(seed, n_chan, n_pix, half)


def _batches(seed, n):
    rng = random.Random(seed)
    out = []
    for case in range(n):
        shapes = []
        for _ in range(rng.randint(1, 6)):
            n_fft = 1 << rng.randint(10, 18)
            n_chan = min(rng.choice([rng.randint(1, 100), rng.randint(100, 2000), rng.randint(2000, 16384)]), n_fft, 16384)
            chan0 = rng.randint(0, n_fft - n_chan)
            n_spec = max(1, min(rng.randint(1, 40), (1 << 19) // n_fft))
            shapes.append((n_fft, n_spec, chan0, n_chan, rng.choice([64, 128, 256])))
        out.append((rng.randint(4, 40), rng.random() < 0.5, rng.random() < 0.5, tuple(shapes), 1000 + case))
    return out


@pytest.mark.parametrize("n_ant,graph,overlap,shapes,seed", _batches(1, 6))
def test_sweep_batch(n_ant, graph, overlap, shapes, seed):
    """A random set of sub-bands through the batch runner (twice, outputs poisoned in between)
    gives the per-sub-band calls' spectra, visibilities and images bit for bit."""
    print(f"batch n_ant={n_ant} graph={graph} overlap={overlap} shapes={shapes}", flush=True)
    xyz, subs = tb._subbands(n_ant, list(shapes), seed=seed)
    ref = tb._per_subband(xyz, subs)
    b = nb.Batch(xyz, subs, graph=graph, overlap=overlap)
    for _ in range(2):
        tb._poison(b)
        b.run()
        torch.cuda.synchronize()
        tb._same(b, ref)
    b.close()


def _searches(seed, n):
    rng = random.Random(seed)
    return [(rng.randint(1, 10 ** 6), round(10 ** rng.uniform(math.log10(0.002), math.log10(0.6)), 4),
             rng.choice([1.0, 1.2, 1.4])) for _ in range(n)]


@pytest.mark.parametrize("seed,q,sigma", _searches(1, 6))
def test_sweep_search(seed, q, sigma):
    tse.search_parity(seed, q, sigma)


def _corr_shapes(seed, n, max_spec):
    rng = random.Random(seed)
    return [(rng.randint(1, 6), rng.choice([rng.randint(1, 64), rng.randint(64, 420)]), rng.randint(1, max_spec))
            for _ in range(n)]


@pytest.mark.parametrize("n_chan,n_in,n_spec", _corr_shapes(1, 6, 400))
def test_sweep_correlate_cal(n_chan, n_in, n_spec):
    tca.test_correlate_cal_matches_oracle(n_chan, n_in, n_spec)


# (int8 products summed over at most 200 spectra stay integers below 2^24: exact in float32)
@pytest.mark.parametrize("n_chan,n_in,n_spec", _corr_shapes(2, 6, 200))
def test_sweep_correlate_f32(n_chan, n_in, n_spec):
    tp.test_correlate_f32_matches_oracle(n_chan, n_in, n_spec)
