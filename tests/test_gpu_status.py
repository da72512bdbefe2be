"""nbsi_status: device flags for non-finite numbers and saturation, through the C ABI, and the
detector's handling of non-finite pixels (not searched; oracle-equal candidates elsewhere)."""
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


def _compare(rec, ref, snr_ref, tau, tol=1e-4):
    got = {(int(r["y"]), int(r["x"]), int(r["c"])): float(r["snr"]) for r in rec}
    exp = {(int(r["y"]), int(r["x"]), int(r["c"])): float(r["snr"]) for r in ref}
    n_chan = snr_ref.shape[0]
    for k in set(got) ^ set(exp):
        y, x, c = k
        s = snr_ref[c, y, x]
        near_tau = abs(s - tau) < tol * max(1, abs(s))
        near_nb = any(abs(s - snr_ref[cc, y, x]) < tol * max(1, abs(s)) for cc in (c - 1, c + 1) if 0 <= cc < n_chan)
        assert near_tau or near_nb, (k, s)
    for k in set(got) & set(exp):
        assert abs(got[k] - exp[k]) <= tol * max(1.0, abs(exp[k])), (k, got[k], exp[k])


@pytest.mark.parametrize("n_chan,n_pix,mode", [(200, 32, nb.NBSI_DETECT_PER_PIXEL), (150, 32, nb.NBSI_DETECT_PER_IMAGE),
                                               (5000, 8, nb.NBSI_DETECT_PER_PIXEL)])
def test_nan_cube_flagged_and_finite_pixels_match_oracle(n_chan, n_pix, mode):
    print(f"status detect n_chan={n_chan} n_pix={n_pix} mode={mode}", flush=True)
    ctx = nb.Context(0)
    assert nb.nbsi_status(ctx) == 0
    rng = np.random.default_rng(n_chan)
    cube = rng.standard_normal((n_chan, n_pix, n_pix)).astype(np.float32)
    cube += rng.uniform(-2, 2, size=(1, n_pix, n_pix)).astype(np.float32)
    for _ in range(40):
        cube[rng.integers(n_chan), rng.integers(n_pix), rng.integers(n_pix)] += rng.uniform(8, 30)
    h = n_pix // 2
    # non-finite values at in-horizon pixels (one whole spectrum NaN), and one below the horizon
    cube[3, h, h] = np.nan
    cube[n_chan - 1, h + 1, h - 2] = np.inf
    cube[n_chan // 2, h - 1, h + 1] = -np.inf
    cube[:, h - 2, h] = np.nan
    cube[0, 0, 0] = np.nan
    rec, snr, n = nb.nbsi_detect(torch.from_numpy(cube).to(DEV), mode=mode, thresh=5.0, want_snr=True, ctx=ctx)
    flags = nb.nbsi_status(ctx)
    assert flags == nb.NBSI_FLAG_CUBE_NONFINITE
    assert nb.nbsi_status(ctx) == 0  # cleared by the read
    ref, snr_ref, valid = oracle.detect.detect(cube, tau=5.0, mode="per_pixel" if mode == 0 else "per_image")
    for (y, x) in [(h, h), (h + 1, h - 2), (h - 1, h + 1), (h - 2, h)]:
        assert not valid[y, x]
        assert (snr.cpu().numpy()[:, y, x] == 0).all()
        assert not any((r["x"] == x and r["y"] == y) for r in rec)
    assert np.isfinite(snr.cpu().numpy()).all()
    _compare(rec, ref, snr_ref, 5.0)
    sg = snr.cpu().numpy().astype(np.float64)
    assert np.abs(sg[:, valid] - snr_ref[:, valid]).max() <= 1e-4 * max(1.0, np.abs(snr_ref).max())
    # a finite cube raises no flag; the fixed-workspace entry point flags the same way
    clean = np.nan_to_num(cube, nan=0.0, posinf=0.0, neginf=0.0)
    nb.nbsi_detect(torch.from_numpy(clean).to(DEV), mode=mode, ctx=ctx)
    assert nb.nbsi_status(ctx) == 0
    rec2, _, n2 = nb.nbsi_detect_noalloc(torch.from_numpy(cube).to(DEV), mode=mode, ctx=ctx)
    assert nb.nbsi_status(ctx) == nb.NBSI_FLAG_CUBE_NONFINITE
    assert n2 == n and np.array_equal(rec2, rec)
    ctx.close()


def test_channelizer_flags_non_finite_gain_and_saturation():
    ctx = nb.Context(0)
    n_in, n_fft, n_spec, chan0, n_chan = 4, 4096, 3, 1000, 64
    xyz = synth.antenna_layout(2, 50.0, 3)
    v = synth.voltages(2, n_fft, n_spec, [synth.Tone(k0=-1048 + 32, amp=1.0, l0=0.0, m0=0.0)], xyz, 4)[:n_in]
    v = v.contiguous().to(DEV)
    g0 = float(synth.gain_noise(n_fft, 8.0))
    gain = torch.full((n_in,), g0, device=DEV)
    q_ok, _ = nb.nbsi_channelize(v, n_fft, n_spec, chan0, n_chan, gain, want_q=True, ctx=ctx)
    assert nb.nbsi_status(ctx) == 0
    bad = gain.clone()
    bad[1] = float("nan")
    q_nan, f_nan = nb.nbsi_channelize(v, n_fft, n_spec, chan0, n_chan, bad, want_q=True, want_f=True, ctx=ctx)
    assert nb.nbsi_status(ctx) == nb.NBSI_FLAG_SPEC_NONFINITE
    qn, qo = q_nan.cpu().numpy(), q_ok.cpu().numpy()
    assert (qn[:, 1] == 0).all() and np.isnan(f_nan.cpu().numpy()[:, 1]).all()
    keep = [0, 2, 3]
    assert np.array_equal(qn[:, keep], qo[:, keep])
    # a gain 200 x too large saturates the loud tone's channel (and most noise) at +-127
    big = torch.full((n_in,), g0 * 200.0, device=DEV)
    q_big, _ = nb.nbsi_channelize(v, n_fft, n_spec, chan0, n_chan, big, want_q=True, ctx=ctx)
    assert nb.nbsi_status(ctx) == nb.NBSI_FLAG_SPEC_CLIPPED
    assert np.abs(q_big.cpu().numpy().astype(int)).max() == 127
    inf_gain = torch.full((n_in,), float("inf"), device=DEV)
    nb.nbsi_channelize(v, n_fft, n_spec, chan0, n_chan, inf_gain, want_q=True, ctx=ctx)
    assert nb.nbsi_status(ctx) & nb.NBSI_FLAG_SPEC_NONFINITE
    ctx.close()


@pytest.mark.parametrize("method", [nb.NBSI_IMAGE_GRID, nb.NBSI_IMAGE_DFT])
def test_imager_flags_non_finite_visibilities(method):
    ctx = nb.Context(0)
    n_ant = 24
    xyz = synth.antenna_layout(n_ant, 60.0, 9)
    freq = synth.channel_freqs(65536, 32768, 3)
    plan = nb.ImagePlan(xyz, freq, 64, method, ctx=ctx)
    n_in = 2 * n_ant
    rng = np.random.default_rng(2)
    vis = rng.standard_normal((3, n_in * (n_in + 1) // 2, 2)).astype(np.float32)
    vt = torch.from_numpy(vis).to(DEV)
    img = nb.nbsi_image(plan, vt)
    assert nb.nbsi_status(ctx) == 0 and torch.isfinite(img).all()
    pairs = plan.pairs() if method == nb.NBSI_IMAGE_GRID else np.array([[1, 0]])
    a, b = int(pairs[0, 0]), int(pairs[0, 1])
    t = (2 * a) * (2 * a + 1) // 2 + 2 * b      # XX of an imaged pair
    vis[1, t, 0] = np.nan
    img = nb.nbsi_image(plan, torch.from_numpy(vis).to(DEV))
    assert nb.nbsi_status(ctx) == nb.NBSI_FLAG_IMAGE_NONFINITE
    im = img.cpu().numpy()
    assert np.isfinite(im[[0, 2]]).all() and not np.isfinite(im[1]).all()
    ctx.close()


def test_calls_on_alternating_streams_of_one_context():
    """The default context follows torch's current stream; a call on a new stream waits for the
    context's earlier work, so calls sharing its scratch on different streams give the results of
    one stream."""
    ctx = nb.Context(0)
    n_ant = 48
    xyz = synth.antenna_layout(n_ant, 150.0, 5)
    freq = synth.channel_freqs(65536, 32768 - 150, 300)
    plan = nb.ImagePlan(xyz, freq, 128, nb.NBSI_IMAGE_GRID, ctx=ctx)
    n_in = 2 * n_ant
    rng = np.random.default_rng(8)
    vis = [torch.from_numpy(rng.integers(-900, 900, (300, n_in * (n_in + 1) // 2, 2)).astype(np.int32)).to(DEV)
           for _ in range(4)]
    ref = [nb.nbsi_image(plan, v).clone() for v in vis]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for k in range(8):
        with torch.cuda.stream(streams[k % 2]):
            outs.append(nb.nbsi_image(plan, vis[k % 4]))
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        assert torch.equal(o, ref[k % 4]), k
    ctx.close()
