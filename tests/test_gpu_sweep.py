"""GPU parity over seeded random shapes: the channelizer (every transform size from 256 to 2^18
points, bands anywhere in the spectrum, 1 to 16,384 channels), the correlator (1 to 420 inputs,
1 to 400 spectra: whole-channel and tiled kernels, repacked rows), the detector (12 to 6,000
channels, both noise models) and the gridded imager, each against the oracle with the fixed
cases' own checks and bars.  The shapes come from a fixed seed, so the cases are the same on
every run."""
import random

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402
import test_gpu_parity as tp  # noqa: E402


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
