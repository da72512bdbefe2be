"""Calibration applied in the correlator's epilogue (nbsi_correlate_cal) against the oracle
(oracle.correlate then oracle.calibrate in float64), and calibrated imaging with uv-range cuts
against the direct-Fourier oracle."""
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


def _cal(n_chan, n_in, seed):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 2.0, (n_chan, n_in))
    ph = rng.uniform(-np.pi, np.pi, (n_chan, n_in))
    return np.stack([amp * np.cos(ph), amp * np.sin(ph)], -1).astype(np.float32)


@pytest.mark.parametrize("n_chan,n_in,n_spec", [
    (3, 48, 16),      # whole channel, K 32
    (2, 130, 64),     # whole channel, K 64, ragged panel
    (2, 100, 100),    # 128 x 128 tiles, spectra repacked to a 16-byte stride
    (1, 64, 256),     # tiles, aligned
    (2, 704, 32),     # the instrument's inputs
])
def test_correlate_cal_matches_oracle(n_chan, n_in, n_spec):
    print(f"correlate_cal n_chan={n_chan} n_in={n_in} n_spec={n_spec} "
          f"kernel {nb.nbsi_correlate_kernel(n_in, n_spec)}", flush=True)
    q = synth.random_spectra(n_chan, n_in, n_spec, seed=n_in + n_spec, full_range=True)
    cal = _cal(n_chan, n_in, 7 * n_in)
    got = nb.nbsi_correlate_cal(q.to(DEV), torch.from_numpy(cal).to(DEV)).cpu().numpy().astype(np.float64)
    ref = oracle.calibrate(oracle.correlate(q.numpy()), cal.astype(np.float64))
    scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
    err = np.abs(got - ref) / scale
    print(f"  max error / channel peak {err.max():.2e}", flush=True)
    assert err.max() < 1e-6  # a few float32 roundings of |w_i V_ij w_j| <= the channel peak
    # the plain correlator is unchanged and the identity correction gives its values as floats
    one = np.zeros_like(cal)
    one[..., 0] = 1.0
    v1 = nb.nbsi_correlate_cal(q.to(DEV), torch.from_numpy(one).to(DEV)).cpu().numpy()
    v0 = nb.nbsi_correlate(q.to(DEV)).cpu().numpy()
    np.testing.assert_array_equal(v1, v0.astype(np.float32))


@pytest.mark.parametrize("method", [nb.NBSI_IMAGE_DFT, nb.NBSI_IMAGE_GRID])
def test_calibrated_imaging_with_uv_range(method):
    n_ant, n_chan, n_pix = 24, 3, 64
    xyz = synth.antenna_layout(n_ant, 60.0, 31)
    freq = synth.channel_freqs(65536, 32768 - 1, n_chan)
    q = synth.random_spectra(n_chan, 2 * n_ant, 16, seed=9)
    cal = _cal(n_chan, 2 * n_ant, 10)
    vis = nb.nbsi_correlate_cal(q.to(DEV), torch.from_numpy(cal).to(DEV))
    ref_vis = oracle.calibrate(oracle.correlate(q.numpy()), cal.astype(np.float64))
    for uv_min, uv_max in ((0.0, np.inf), (3.0, 12.0)):
        plan = nb.nbsi_image_plan_create(xyz, freq, n_pix, method, uv_min=uv_min, uv_max=uv_max)
        nbase = plan.n_baselines()
        np.testing.assert_array_equal(
            nbase, oracle.count_baselines(xyz, freq, n_pix if method == nb.NBSI_IMAGE_GRID else 0, uv_min, uv_max))
        img = nb.nbsi_image(plan, vis).cpu().numpy()
        ref = oracle.image_dft(ref_vis, xyz, freq, n_pix, grid_n_pix=n_pix if method == nb.NBSI_IMAGE_GRID else 0,
                               uv_min=uv_min, uv_max=uv_max)
        err = np.abs(img - ref).max() / np.abs(ref).max()
        print(f"  method {method} uv [{uv_min}, {uv_max}]: |B| {nbase.tolist()}, max error {err:.2e}", flush=True)
        assert err < 1e-5
