"""Stage II on the GPU (nbsi_stage2, nbsi_beam) against the oracle (oracle/stage2.py): Gaussian
centroid fits, covariance errors, flags, and the synthesized beam of gridding and direct Fourier
plans."""
import math

import numpy as np
import pytest

import synth
import oracle
from oracle import stage2 as s2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402

DEV = torch.device("cuda", 0)
K = 2.0 * math.sqrt(2.0 * math.log(2.0))


def _cands(lst):
    a = np.zeros((len(lst), 5), np.int32)
    for i, (x, y, c) in enumerate(lst):
        a[i, :3] = (x, y, c)
    return torch.from_numpy(a).to(DEV)


def _assert_consistent(cut, f, x, y, sigma0, bmaj, bmin, ext):
    """A GPU record is a valid outcome of the fit of this cutout: its RSS is the model's at its
    parameters and no higher than at the starting point, its shape and errors follow from its
    parameters (errors where the normal matrix is well conditioned), and its flags from those."""
    cut = np.asarray(cut, np.float64)
    h = cut.shape[0] // 2
    p = np.array([f["amp"], f["x0"] - x, f["y0"] - y, f["a"], f["b"], f["c"], f["bkg"]])
    yy, xx = np.mgrid[-h:h + 1, -h:h + 1].astype(np.float64)
    rss = float(np.sum((s2.model(p, xx, yy) - cut) ** 2))
    rss0 = float(np.sum((s2.model(s2.initial(cut, sigma0), xx, yy) - cut) ** 2))
    assert abs(f["rss"] - rss) <= 1e-9 * rss + 1e-12 and rss <= rss0 * (1 + 1e-12)
    failed = bool(f["flags"] & nb.NBSI_S2_FIT_FAILED)
    pd = p[0] > 0 and p[3] > 0 and p[5] > 0 and p[3] * p[5] - p[4] ** 2 > 0
    if not failed:
        assert pd
        maj, mnr, _ = s2.shape(p[3], p[4], p[5])
        assert f["fwhm_maj"] == pytest.approx(maj, rel=1e-9) and f["fwhm_min"] == pytest.approx(mnr, rel=1e-9)
        assert bool(f["flags"] & nb.NBSI_S2_EXTENDED) == (maj > ext * bmaj or mnr > ext * bmin)
        J = s2.jacobian(p, xx, yy)
        H = J.T @ J
        if np.linalg.cond(H) < 1e10:
            err = np.sqrt(np.diag(np.linalg.inv(H)) * rss / (cut.size - 7))
            np.testing.assert_allclose(f["err"], err, rtol=1e-4)
    else:
        assert not pd or not np.all(np.isfinite(p)) or np.linalg.cond(s2.jacobian(p, xx, yy)) > 1e7


REJECT = nb.NBSI_S2_EXTENDED | nb.NBSI_S2_FIT_FAILED


def _shape_tol(p, tol):
    """First-order bound on how far (FWHM major, FWHM minor, position angle) move when the
    shape parameters a, b, c (p[3:6]) move within tol[3:6]: central differences of the oracle's
    shape function."""
    out = np.zeros(3)
    for k in range(3):
        h = 1e-6 * max(abs(p[3 + k]), 1e-9)
        up, dn = np.array(p[3:6], np.float64), np.array(p[3:6], np.float64)
        up[k] += h
        dn[k] -= h
        su, sd = np.array(s2.shape(*up)), np.array(s2.shape(*dn))
        dv = su - sd
        dv[2] = (dv[2] + math.pi / 2) % math.pi - math.pi / 2   # the angle is defined mod pi
        out += np.abs(dv / (2 * h)) * tol[3 + k]
    return out


def _compare(cube, cand_list, beam, half=4, ext=1.5, nk=1.5, noise_ok=(), reject_ok=()):
    """Runs both sides and checks them record by record; returns (GPU records, oracle results,
    number of fits that reached the same minimum).  noise_ok: candidates on noise alone, where
    the minimisers may stop at different stationary points; reject_ok: blobs much wider than the
    cutout, whose fits are degenerate (amplitude against background): there both sides must
    reject the candidate."""
    n_chan = cube.shape[0]
    bm = np.broadcast_to(np.asarray(beam, np.float64), (n_chan, 3)).copy()
    out = nb.nbsi_stage2(torch.from_numpy(cube).to(DEV), _cands(cand_list), torch.from_numpy(bm).to(DEV),
                         half=half, ext_factor=ext, noise_k=nk)
    torch.cuda.synchronize()
    g = nb.fits_host(out, len(cand_list))
    ref = s2.stage2(cube, [{"x": x, "y": y, "c": c} for (x, y, c) in cand_list], bm, ext, nk, half)
    # noise decisions: no channel within rounding of a bound (the GPU's sigma is float32)
    sig = s2.channel_noise(cube)
    med = float(s2.median_even_mean(sig, axis=0))
    for v in sig:
        for bound in (med / nk, med * nk):
            assert abs(v - bound) > 1e-5 * bound
    n_same = 0
    for i, (r, f) in enumerate(zip(ref, g)):
        of = r["fit"]
        if of is None:                              # outside: no fit on either side
            assert f["flags"] == r["flags"], (i, f["flags"], r["flags"])
            continue
        x, y, c = cand_list[i]
        cut = cube[c, y - half:y + half + 1, x - half:x + half + 1].astype(np.float64)
        yy, xx = np.mgrid[-half:half + 1, -half:half + 1].astype(np.float64)
        p_gpu = np.array([f["amp"], f["x0"], f["y0"], f["a"], f["b"], f["c"], f["bkg"]])
        well = of["ok"] and np.linalg.cond(s2.jacobian(of["p"], xx, yy)) < 1e4
        same_min = (of["ok"] and not f["flags"] & nb.NBSI_S2_FIT_FAILED
                    and abs(f["rss"] - of["rss"]) <= 1e-9 * of["rss"])
        if not (well and same_min):
            # an ill-conditioned fit (noise alone: many local minima and degenerate directions;
            # a blob much wider than the cutout: amplitude against background): the GPU's record
            # must be a valid outcome of the same fit, with the same noise and outside flags
            assert i in noise_ok or i in reject_ok, (i, well, same_min, f["rss"], of["rss"], f["flags"], r["flags"])
            sigma0 = bm[c, 0] / K if np.isfinite(bm[c, 0]) and bm[c, 0] > 0 else 1.0
            _assert_consistent(cut, f, x, y, sigma0, bm[c, 0], bm[c, 1], ext)
            assert (f["flags"] & ~REJECT) == (r["flags"] & ~REJECT)
            if i in reject_ok:   # the same decision, or both reject
                assert f["flags"] == r["flags"] or ((f["flags"] & REJECT) and (r["flags"] & REJECT)), \
                    (i, f["flags"], r["flags"])
            continue
        n_same += 1
        p_ref = np.array([of["p"][0], of["x0"], of["y0"], *of["p"][3:7]])
        assert f["flags"] == r["flags"], (i, f["flags"], r["flags"])
        tol = 1e-4 * of["err"] + 1e-9 * (1.0 + np.abs(p_ref))
        assert np.all(np.abs(p_gpu - p_ref) <= tol), (i, p_gpu - p_ref, tol)
        np.testing.assert_allclose(f["err"], of["err"], rtol=1e-5)
        # the axes and the angle are functions of (a, b, c): their bar is the parameters' bar
        # carried through those functions (an elongated blob magnifies it), with a floor
        stol = _shape_tol(p_ref, tol)
        assert abs(f["fwhm_maj"] - of["fwhm_maj"]) <= max(1e-6 * of["fwhm_maj"], 2 * stol[0]), (i, stol)
        assert abs(f["fwhm_min"] - of["fwhm_min"]) <= max(1e-6 * of["fwhm_min"], 2 * stol[1]), (i, stol)
        if of["fwhm_maj"] > 1.001 * of["fwhm_min"]:
            d = abs(f["pa"] - of["pa"])
            assert min(d, math.pi - d) < max(1e-5, 2 * stol[2]), (i, stol)
        assert f["chi2_red"] == pytest.approx(of["chi2_red"], rel=1e-5)
        # the extended decision is away from its bound
        bmaj, bmin = bm[c, 0], bm[c, 1]
        assert abs(of["fwhm_maj"] - ext * bmaj) > 1e-6 * bmaj and abs(of["fwhm_min"] - ext * bmin) > 1e-6 * bmin
    return g, ref, n_same


@pytest.mark.parametrize("seed,n_chan,n_pix,half", [(1, 16, 64, 4), (2, 40, 96, 5), (3, 9, 48, 2), (4, 24, 128, 3)])
def test_stage2_matches_oracle(seed, n_chan, n_pix, half):
    print(f"stage2 seed={seed} C={n_chan} N={n_pix} half={half}", flush=True)
    rng = np.random.default_rng(seed)
    bs = (1.6, 1.2, 0.5)
    cube, blobs = synth.stage2_scene(rng, n_chan, n_pix, beam_sigma=bs, n_point=12, n_ext=5, noisy=(2, -6))
    cl = [(int(round(b.x)), int(round(b.y)), b.c) for b in blobs]
    n_src = len(cl)
    # noise-only cutouts, edges, a channel outside the cube
    for _ in range(8):
        cl.append((int(rng.integers(half, n_pix - half)), int(rng.integers(half, n_pix - half)),
                   int(rng.integers(0, n_chan))))
    cl += [(half - 1, n_pix // 2, 0), (n_pix - half, 10, 1), (10, n_pix - 1, 2), (20, 20, n_chan), (20, 20, -1)]
    ext = {i for i, b in enumerate(blobs) if b.extended}
    g, ref, n_same = _compare(cube, cl, (K * bs[0], K * bs[1], bs[2]), half=half,
                              noise_ok=set(range(n_src, n_src + 8)), reject_ok=ext)
    assert n_same >= n_src - len(ext)          # every beam-shaped blob reaches the same minimum
    flags = g["flags"]
    for i, b in enumerate(blobs):
        if b.c in (2, 5):
            assert flags[i] & nb.NBSI_S2_NOISY
        if b.extended and half >= 4:
            assert flags[i] & (nb.NBSI_S2_EXTENDED | nb.NBSI_S2_FIT_FAILED)
    assert np.all(flags[-5:] & nb.NBSI_S2_OUTSIDE)
    assert flags[-2] == nb.NBSI_S2_OUTSIDE and flags[-1] == nb.NBSI_S2_OUTSIDE


def test_stage2_noise_free_blobs():
    """Noise-free blobs on a flat background: both sides reach the exact parameters."""
    n_pix, n_chan = 64, 4
    cube = np.full((n_chan, n_pix, n_pix), 0.1, np.float64)
    cube += np.random.default_rng(0).standard_normal(cube.shape) * 1e-3
    params = [(20.3, 30.6, 0, 8.0, 1.7, 1.1, 0.3), (40.0, 21.2, 1, 5.0, 1.5, 1.5, 0.0), (31.7, 44.4, 3, 9.0, 2.1, 1.0, 2.0)]
    for (x, y, c, a, sm, sn, th) in params:
        cube[c] += synth.elliptical_blob(n_pix, x, y, a, sm, sn, th)
    cube = cube.astype(np.float32)
    cl = [(int(round(x)), int(round(y)), c) for (x, y, c, *_ ) in params]
    g, ref, n_same = _compare(cube, cl, (4.0, 3.0, 0.0))
    assert n_same == 3
    for f, (x, y, c, a, sm, sn, th) in zip(g, params):
        assert abs(f["x0"] - x) < 1e-3 and abs(f["y0"] - y) < 1e-3
        assert f["fwhm_maj"] == pytest.approx(K * sm, rel=1e-3)


def test_stage2_full_frame_sample():
    """A 256-channel 256 x 256 cube (the instrument-scale image size) with 2048 candidates, the
    launch shape of the benchmark: every record's flags are valid and 64 sampled records match
    the oracle's fit on the same cutout."""
    n_chan, n_pix = 256, 256
    rng = np.random.default_rng(77)
    bs = (1.6, 1.2, 0.5)
    cube, blobs = synth.stage2_scene(rng, n_chan, n_pix, beam_sigma=bs, n_point=1536, n_ext=512, noisy=(5, 17, -100))
    cl = [(int(round(b.x)), int(round(b.y)), b.c) for b in blobs]
    beam = np.tile([K * bs[0], K * bs[1], bs[2]], (n_chan, 1))
    out = nb.nbsi_stage2(torch.from_numpy(cube).to(DEV), _cands(cl), torch.from_numpy(beam).to(DEV))
    torch.cuda.synchronize()
    g = nb.fits_host(out, len(cl))
    sig = s2.channel_noise(cube)
    med = float(s2.median_even_mean(sig, axis=0))
    noisy = (sig < med / 1.5) | (sig > 1.5 * med)
    assert sorted(np.flatnonzero(noisy)) == [5, 17, 99]
    np.testing.assert_array_equal((g["flags"] & nb.NBSI_S2_NOISY) != 0, noisy[[c for (_, _, c) in cl]])
    pick = rng.choice(len(cl), 64, replace=False)
    for i in pick:
        x, y, c = cl[i]
        of = s2.fit(cube[c, y - 4:y + 5, x - 4:x + 5].astype(np.float64), bs[0])
        f = g[i]
        if not blobs[i].extended:
            assert of["ok"] and not f["flags"] & nb.NBSI_S2_FIT_FAILED
        if of["ok"] and abs(f["rss"] - of["rss"]) <= 1e-9 * of["rss"]:
            assert abs(f["x0"] - (x + of["p"][1])) <= 1e-4 * of["err"][1] + 1e-8
            assert abs(f["y0"] - (y + of["p"][2])) <= 1e-4 * of["err"][2] + 1e-8
    kept = (g["flags"] == 0)
    ext = np.array([b.extended for b in blobs])
    assert kept[~ext].mean() > 0.9 and kept[ext].mean() < 0.1


def _psf_oracle(xyz, freq, n_pix, grid):
    n_in = 2 * xyz.shape[0]
    vis = np.zeros((len(freq), n_in * (n_in + 1) // 2, 2))
    vis[..., 0] = 1.0
    h = n_pix // 2
    pix = np.array([(x, y) for y in range(h - 2, h + 3) for x in range(h - 2, h + 3)])
    vals = oracle.image_dft_pixels(vis, xyz, freq, n_pix, pix, grid_n_pix=n_pix if grid else 0)
    out = []
    for c in range(len(freq)):
        psf = np.zeros((n_pix, n_pix))
        psf[pix[:, 1], pix[:, 0]] = vals[c]
        out.append(s2.beam(psf))
    return np.array(out)


@pytest.mark.parametrize("method,n_ant,radius,n_pix,n_chan", [(nb.NBSI_IMAGE_GRID, 96, 60.0, 256, 5),
                                                             (nb.NBSI_IMAGE_GRID, 48, 100.0, 128, 3),
                                                             (nb.NBSI_IMAGE_DFT, 16, 16.0, 64, 4)])
def test_beam_matches_oracle(method, n_ant, radius, n_pix, n_chan):
    print(f"beam method={method} A={n_ant} N={n_pix} C={n_chan}", flush=True)
    xyz = synth.antenna_layout(n_ant, radius, 9 + n_ant)
    xyz[:, 0] *= 1.6
    freq = synth.channel_freqs(65536, 32768 - 2, n_chan)
    freq = freq + np.arange(n_chan) * 2.0e6          # spread the channels so the beam changes
    plan = nb.ImagePlan(xyz, freq, n_pix, method)
    beam = nb.nbsi_beam(plan).cpu().numpy()
    ref = _psf_oracle(xyz, freq, n_pix, method == nb.NBSI_IMAGE_GRID)
    print(beam, ref, sep="\n", flush=True)
    np.testing.assert_allclose(beam[:, :2], ref[:, :2], rtol=1e-3)
    for c in range(n_chan):
        if ref[c, 0] > 1.01 * ref[c, 1]:
            d = abs(beam[c, 2] - ref[c, 2])
            assert min(d, math.pi - d) < 2e-3


def test_stage2_rejects_bad_arguments():
    cube = torch.zeros((8, 32, 32), dtype=torch.float32, device=DEV)
    beam = torch.ones((8, 3), dtype=torch.float64, device=DEV)
    c = _cands([(10, 10, 0)])
    for kw in (dict(half=1), dict(half=6), dict(ext_factor=0.0), dict(noise_k=0.5)):
        with pytest.raises(nb.NbsiError):
            nb.nbsi_stage2(cube, c, beam, **kw)
    with pytest.raises(nb.NbsiError):
        nb.nbsi_stage2(torch.zeros((2, 32, 32), dtype=torch.float32, device=DEV), c, beam[:2])
    out = nb.nbsi_stage2(cube, c[:0], beam)       # no candidates: nothing to do
    torch.cuda.synchronize()
    assert out.shape[0] == 1
