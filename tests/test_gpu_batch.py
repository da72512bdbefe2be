"""GPU parity of the batched path: uneven sub-bands (different FFT lengths, integration counts,
channel counts and image sizes) run as grouped persistent launches, optionally captured into a
hipGraph, must give exactly what the per-sub-band calls give (spectra, visibilities, images
bit-identical; the per-sub-band calls are themselves checked against the oracle in
test_gpu_parity.py), and their visibilities must equal the oracle's correlation of their own
spectra.  A graph is replayed several times with eager work between replays and every replay
is checked (outputs are overwritten with a sentinel first).
"""
import os

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

# n_fft, n_spec, chan0, n_chan, n_pix: every channelizer grouping (M = N <= 4096, P > 1 with
# M = 4096, M = 8192 and M = 16384), both correlator variants and three image sizes
SMALL = [
    (4096, 16, 2016, 64, 64),
    (16384, 4, 8000, 96, 128),
    (1024, 33, 0, 1024, 64),
    (65536, 2, 30000, 8192, 64),
    (1 << 18, 1, (1 << 17) - 100, 200, 128),
    (8192, 70, 4090, 20, 256),
]


def _subbands(n_ant, shapes, seed):
    xyz = synth.antenna_layout(n_ant, 150.0, seed)
    out = []
    for i, (n_fft, n_spec, chan0, n_chan, n_pix) in enumerate(shapes):
        nu0 = synth.NU0 + (i - len(shapes) // 2) * synth.F_COARSE
        tones = [synth.Tone(k0=chan0 + n_chan // 3 - n_fft // 2, amp=5.0, l0=0.15, m0=-0.1)]
        v = synth.voltages(n_ant, n_fft, n_spec, tones, xyz, seed + 10 + i, device="cuda", nu0=nu0)
        g = torch.full((2 * n_ant,), float(synth.gain_noise(n_fft, synth.SIGMA)), dtype=torch.float32, device=DEV)
        out.append(dict(volt=v, gain=g, n_fft=n_fft, n_spec=n_spec, chan0=chan0, n_chan=n_chan, n_pix=n_pix,
                        freq_hz=synth.channel_freqs(n_fft, chan0, n_chan, nu0)))
    return xyz, out


def _per_subband(xyz, subs, precision=nb.NBSI_PREC_FP32):
    ref = []
    for d in subs:
        q, _ = nb.nbsi_channelize(d["volt"], d["n_fft"], d["n_spec"], d["chan0"], d["n_chan"], d["gain"])
        vis = nb.nbsi_correlate(q)
        plan = nb.ImagePlan(xyz, d["freq_hz"], d["n_pix"], nb.NBSI_IMAGE_GRID)
        img = nb.nbsi_image(plan, vis, precision)
        torch.cuda.synchronize()
        plan.close()
        ref.append((q, vis, img))
    return ref


def _poison(batch):
    for d in batch.subbands:
        d["spec_q"].fill_(77)
        d["vis"].fill_(-12345)
        d["img"].fill_(float("nan"))


def _same(batch, ref, img_exact=True):
    for i, (d, (q, vis, img)) in enumerate(zip(batch.subbands, ref)):
        assert torch.equal(d["spec_q"], q), f"sub-band {i}: spectra differ"
        assert torch.equal(d["vis"], vis), f"sub-band {i}: visibilities differ"
        if img_exact:
            assert torch.equal(d["img"], img), f"sub-band {i}: images differ"
        else:
            a, b = d["img"].double(), img.double()
            err = (a - b).abs().max().item() / b.abs().max().item()
            assert err <= 1e-5, f"sub-band {i}: image differs by {err:.2e} of the peak"


@pytest.mark.parametrize("graph,overlap", [(True, False), (False, False), (True, True), (False, True)])
def test_batch_equals_per_subband(graph, overlap):
    """overlap: sub-band s + 1 is channelized while sub-band s is correlated and imaged on the
    batch's second stream (the graph flag is then not used)."""
    print(f"batch small graph={graph} overlap={overlap}", flush=True)
    xyz, subs = _subbands(12, SMALL, seed=31)
    ref = _per_subband(xyz, subs)
    b = nb.Batch(xyz, subs, graph=graph, overlap=overlap)
    for rep in range(3):
        _poison(b)
        b.run()
        torch.cuda.synchronize()
        _same(b, ref)
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device=DEV)
        assert torch.isfinite(x.sum()).item()
    b.close()


def test_batch_visibilities_match_oracle():
    print("batch vis vs oracle", flush=True)
    xyz, subs = _subbands(9, SMALL[:3], seed=47)
    b = nb.Batch(xyz, subs)
    b.run()
    torch.cuda.synchronize()
    for d in b.subbands:
        q = d["spec_q"].cpu().numpy()
        assert np.array_equal(d["vis"].cpu().numpy(), oracle.correlate(q))
    b.close()


def test_batch_images_match_oracle():
    print("batch images vs DFT oracle", flush=True)
    xyz, subs = _subbands(10, [(4096, 8, 1900, 6, 64), (16384, 2, 8100, 5, 128)], seed=53)
    b = nb.Batch(xyz, subs)
    b.run()
    torch.cuda.synchronize()
    for d in b.subbands:
        vis = d["vis"].cpu().numpy()
        ref = oracle.image_dft(vis, xyz, d["freq_hz"], d["n_pix"], grid_n_pix=d["n_pix"])
        got = d["img"].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= 1e-5, err
    b.close()


def test_batch_tall_grid_tile():
    """The 32-cell gridding tile: same spectra and visibilities, images within float32 rounding
    of the 16-cell per-sub-band path and within 1e-5 of the DFT oracle."""
    print("batch tall gridding tile", flush=True)
    xyz, subs = _subbands(12, SMALL, seed=83)
    ref = _per_subband(xyz, subs)
    b = nb.Batch(xyz, subs, grid_tall=True)
    assert b.describe().count('"grid_ge": 32') == len(SMALL)
    for rep in range(2):
        _poison(b)
        b.run()
        torch.cuda.synchronize()
        _same(b, ref, img_exact=False)
    d = b.subbands[1]
    sel = slice(0, 4)
    vis = d["vis"][sel].cpu().numpy()
    want = oracle.image_dft(vis, xyz, d["freq_hz"][sel], d["n_pix"], grid_n_pix=d["n_pix"])
    got = d["img"][sel].cpu().numpy().astype(np.float64)
    assert np.abs(got - want).max() / np.abs(want).max() <= 1e-5
    b.close()


@pytest.mark.parametrize("precision", [nb.NBSI_PREC_FP16, nb.NBSI_PREC_BF16])
def test_batch_reduced_precision_equals_per_subband(precision):
    print(f"batch precision={precision}", flush=True)
    xyz, subs = _subbands(12, SMALL[:4], seed=61)
    ref = _per_subband(xyz, subs, precision)
    b = nb.Batch(xyz, subs, precision=precision)
    for rep in range(2):
        _poison(b)
        b.run()
        torch.cuda.synchronize()
        _same(b, ref)
    b.close()


def json_subbands(desc):
    import json
    return json.loads(desc)["subbands"]


def test_batch_autotune_cache(tmp_path):
    print("batch autotune", flush=True)
    cache = str(tmp_path / "tune.txt")
    xyz, subs = _subbands(12, SMALL, seed=71)
    ref = _per_subband(xyz, subs)
    b = nb.Batch(xyz, subs, autotune=True, tune_cache=cache)
    desc = b.describe()
    assert '"subbands"' in desc and desc.count("corr_variant") == len(SMALL)
    lines = open(cache).read().split("\n")
    assert any(s.startswith("corr_n_in=24,n_spec=16 ") for s in lines)
    assert any(s.startswith("grid_n_ant=12,n_pix=256,n_chan=20 ") for s in lines)
    for rep in range(2):
        _poison(b)
        b.run()
        torch.cuda.synchronize()
        # a tuned gridding tile height changes the order of the per-cell sums: images agree to
        # float32 rounding, spectra and visibilities exactly
        _same(b, ref, img_exact=False)
    b.close()
    # a second plan takes every choice from the cache
    b2 = nb.Batch(xyz, subs, autotune=True, tune_cache=cache)
    assert b2.describe() == desc
    b2.close()
    # the overlapped form takes the same choices from the cache and gives the tuned outputs
    b3 = nb.Batch(xyz, subs, autotune=True, tune_cache=cache, overlap=True)
    assert json_subbands(b3.describe()) == json_subbands(desc)
    ref3 = [(d["spec_q"].clone(), d["vis"].clone(), d["img"].clone()) for d in b.subbands]
    _poison(b3)
    b3.run()
    torch.cuda.synchronize()
    _same(b3, ref3)
    b3.close()


def test_batch_rejects_bad_subbands():
    xyz, subs = _subbands(4, SMALL[:1], seed=3)
    bad = dict(subs[0], n_fft=3000)
    with pytest.raises(nb.NbsiError):
        nb.Batch(xyz, [subs[0], bad])
    bad = dict(subs[0], n_pix=96)
    with pytest.raises(nb.NbsiError):
        nb.Batch(xyz, [bad])


@pytest.mark.slow
def test_batch_uneven_subbands_full_size():
    """Twelve sub-bands of 352 antennas, FFT lengths 2^14..2^18, 8..128 spectra, 1024 channels
    each, images 128^2..512^2: batched graph replays equal the per-sub-band calls exactly."""
    print("batch full size (12 sub-bands, 352 antennas)", flush=True)
    n_ant = 352
    xyz = synth.antenna_layout(n_ant, 1500.0, 2024)
    subs = []
    for i, c in enumerate(synth.subband_configs(12, 1024, n_ant)):
        v = synth.voltages(n_ant, c["n_fft"], c["n_spec"], [], xyz, 500 + i, device="cuda", nu0=c["nu0"])
        g = torch.full((2 * n_ant,), float(c["gain"]), dtype=torch.float32, device=DEV)
        subs.append(dict(volt=v, gain=g, n_fft=c["n_fft"], n_spec=c["n_spec"], chan0=c["chan0"],
                         n_chan=c["n_chan"], n_pix=c["n_pix"],
                         freq_hz=synth.channel_freqs(c["n_fft"], c["chan0"], c["n_chan"], c["nu0"])))
    ref = _per_subband(xyz, subs)
    for overlap in (False, True):
        print(f"  overlap={overlap}", flush=True)
        b = nb.Batch(xyz, subs, graph=True, overlap=overlap)
        for rep in range(2):
            _poison(b)
            b.run()
            torch.cuda.synchronize()
            _same(b, ref)
        b.close()
