"""The no-allocation detector entry point (nbsi_detect_noalloc) against nbsi_detect: the same
candidates and SNR cube, on two calls in a row (the second on a smaller cube, so the fixed
workspace holds the first call's leftovers), and its clear error when the candidates exceed the
fixed workspace."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402

DEV = torch.device("cuda", 0)


def _cube(n_chan, n_pix, seed, n_spikes):
    rng = np.random.default_rng(seed)
    cube = rng.standard_normal((n_chan, n_pix, n_pix)).astype(np.float32)
    cube += rng.uniform(-2, 2, size=(1, n_pix, n_pix)).astype(np.float32)
    for _ in range(n_spikes):
        c, y, x = rng.integers(0, n_chan), rng.integers(0, n_pix), rng.integers(0, n_pix)
        cube[c, y, x] += rng.uniform(6.0, 30.0)
    return torch.from_numpy(cube).to(DEV)


@pytest.mark.parametrize("mode", [nb.NBSI_DETECT_PER_PIXEL, nb.NBSI_DETECT_PER_IMAGE])
def test_noalloc_detect_matches_detect_twice(mode):
    # the per-image noise model sees the per-pixel offsets as noise (SNRs ~0.65 of the per-pixel
    # model's), so its low threshold is lower
    low = 2.5 if mode == nb.NBSI_DETECT_PER_PIXEL else 1.6
    for (n_chan, n_pix, seed, n_spikes, thresh) in [(700, 64, 1, 3000, low), (90, 32, 2, 40, 5.0)]:
        print(f"noalloc detect mode={mode} n_chan={n_chan} n_pix={n_pix}", flush=True)
        img = _cube(n_chan, n_pix, seed, n_spikes)
        rec_ref, snr_ref, n_ref = nb.nbsi_detect(img, mode=mode, thresh=thresh, want_snr=True)
        snr = torch.full_like(img, 7.0)
        rec, snr, n = nb.nbsi_detect_noalloc(img, mode=mode, thresh=thresh, snr=snr)
        torch.cuda.synchronize()
        assert n == n_ref > 0
        assert np.array_equal(rec, rec_ref)
        assert torch.equal(snr, snr_ref)
        # above 4,096 candidates the sort runs through the workspace's keys
        if n_chan == 700:
            assert n > 4096


def test_noalloc_detect_rejects_more_candidates_than_its_workspace():
    img = _cube(300, 64, 3, 0)
    with pytest.raises(nb.NbsiError) as ei:
        nb.nbsi_detect_noalloc(img, thresh=-1e30)
    assert ei.value.status == nb.NBSI_EOVERFLOW and "fixed workspace" in str(ei.value)
    # the next call still works
    small = _cube(64, 16, 4, 5)
    rec_ref, _, n_ref = nb.nbsi_detect(small)
    rec, _, n = nb.nbsi_detect_noalloc(small)
    assert n == n_ref and np.array_equal(rec, rec_ref)
