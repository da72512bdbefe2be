"""Full Stage I search on the GPU against the oracle (oracle/search.py): best-SNR and width cubes
of the boxcar bank, the Benjamini-Hochberg decision (taken in float64 on the GPU's own SNRs on
both sides), suppression and re-evaluation."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402
from oracle import search as osr  # noqa: E402
from oracle.detect import horizon_mask  # noqa: E402

DEV = torch.device("cuda", 0)


def _cube(n_chan, n_pix, seed, lines=(), sigma=1.0):
    rng = np.random.default_rng(seed)
    r = sigma * rng.standard_normal((n_chan, n_pix, n_pix))
    for (x, y, c0, w, snr) in lines:
        r[c0:c0 + w, y, x] += snr / math.sqrt(w)
    return r.astype(np.float32)


def _window_snr(r64, p, c, w, rho=()):
    s = c - w // 2
    return float(r64[s:s + w, p].sum() / osr.boxcar_sigma(w, rho))


def _check_bank(r, S, W, widths=osr.WIDTHS, tol=3e-5, rho=()):
    n_chan = r.shape[0]
    r64 = r.astype(np.float64).reshape(n_chan, -1)
    S_ref, W_ref = osr.boxcar_bank(r64, widths, rho)
    Sg = S.cpu().numpy().reshape(n_chan, -1).astype(np.float64)
    Wg = W.cpu().numpy().reshape(n_chan, -1).astype(np.int32)
    assert np.abs(Sg - S_ref).max() <= tol
    # the width must be the oracle's or one whose SNR ties the maximum within the tolerance
    bad = np.argwhere(Wg != W_ref)
    for c, p in bad[:2000]:
        assert Wg[c, p] in widths
        assert abs(_window_snr(r64, p, c, int(Wg[c, p]), rho) - S_ref[c, p]) <= tol
    return Sg, Wg


@pytest.mark.parametrize("n_chan,n_pix", [(777, 24), (256, 64), (40, 16)])
def test_bank_matches_oracle(n_chan, n_pix):
    print(f"search bank n_chan={n_chan} n_pix={n_pix}", flush=True)
    lines = [(5, 9, min(n_chan - 20, 300), 12, 12.0), (11, 13, n_chan // 3, 1, 9.0)]
    r = _cube(n_chan, n_pix, 100 + n_chan, lines)
    _, _, _, S, W = nb.nbsi_search(torch.from_numpy(r).to(DEV), fdr_q=0.01, want_cubes=True)
    torch.cuda.synchronize()
    _check_bank(r, S, W)


def _expected_records(r, Sg, Wg, sstar, n_pix, rho=()):
    """The oracle's suppression and re-evaluation on the GPU's S and W (float64), with the
    re-evaluated SNRs, to judge decisions near S*."""
    n_chan = r.shape[0]
    valid = horizon_mask(n_pix).ravel()
    acc = (Sg >= sstar) & valid[None, :]
    surv = osr.nms(Sg, Wg, acc)
    r64 = r.astype(np.float64).reshape(n_chan, -1)
    out = {}
    for c, p in zip(*np.nonzero(surv)):
        out[(int(p % n_pix), int(p // n_pix), int(c))] = osr.reevaluate(r64[:, p], int(c), int(Wg[c, p]), rho)
    return out


# (seed, q, noise sigma): the last four put the Benjamini-Hochberg threshold below 3 SNR (a
# lenient level, or noise wider than the unit-normal model as Hann-correlated channels give);
# at q = 0.6 it reaches voxels with S < 0
@pytest.mark.parametrize("seed,q,sigma", [(7, 0.01, 1.0), (8, 0.05, 1.0), (9, 0.2, 1.0), (10, 0.02, 1.4),
                                          (11, 0.05, 1.4), (12, 0.6, 1.0)])
def test_search_matches_oracle(seed, q, sigma):
    thr, got, lines = search_parity(seed, q, sigma)
    if sigma > 1.0 or q >= 0.2:
        assert thr < 3.0
    if q > 0.5:
        assert thr < 0.0
    # every injected line is found at its pixel near its centre
    for (x, y, c0, w, snr) in lines:
        hits = [k for k in got if k[0] == x and k[1] == y and abs(k[2] - (c0 + w // 2)) <= max(2, w // 2)]
        assert hits, (x, y, c0, w)


def search_parity(seed, q, sigma):
    """The whole search on a cube with four injected lines against the oracle: the bank, the
    Benjamini-Hochberg threshold, suppression and re-evaluation record by record, and the
    records' order; returns (S*, records by (x, y, c), the injected lines)."""
    n_chan, n_pix = 640, 32
    lines = [(9, 7, 300, 12, 14.0), (20, 12, 100, 1, 10.0), (14, 20, 500, 40, 16.0), (16, 16, 600, 3, 8.0)]
    print(f"search seed={seed} q={q} sigma={sigma}", flush=True)
    r = _cube(n_chan, n_pix, seed, lines, sigma)
    rec, thr, kprov, S, W = nb.nbsi_search(torch.from_numpy(r).to(DEV), fdr_q=q, want_cubes=True)
    torch.cuda.synchronize()
    print(f"  k* {kprov} S* {thr:.4f} records {len(rec)}", flush=True)
    Sg, Wg = _check_bank(r, S, W)
    valid = horizon_mask(n_pix).ravel()
    k_ref, s_ref = osr.bh_threshold(Sg[:, valid].ravel(), int(valid.sum()) * n_chan, q)
    assert kprov == k_ref and np.float32(thr) == np.float32(s_ref)
    exp = _expected_records(r, Sg, Wg, thr, n_pix)
    got = {(int(a["x"]), int(a["y"]), int(a["c"])): a for a in rec}
    for key, snr2 in exp.items():
        if abs(snr2 - thr) < 1e-4 * max(1.0, thr):
            continue  # a float32 re-evaluation may fall on either side of S*
        assert (key in got) == (snr2 >= thr), (key, snr2, thr)
    for key, a in got.items():
        assert key in exp
        c, p = key[2], key[1] * n_pix + key[0]
        assert a["width"] == Wg[c, p] and np.float32(a["snr"]) == np.float32(Sg[c, p])
    assert list(rec["y"] * 10 ** 6 + rec["x"] * 10 ** 4 + rec["c"]) == sorted(rec["y"] * 10 ** 6 + rec["x"] * 10 ** 4 + rec["c"])
    return thr, got, lines


def test_search_pure_noise_and_zero_cube():
    r = _cube(512, 32, 3)
    rec, thr, kprov, _, _ = nb.nbsi_search(torch.from_numpy(r).to(DEV), fdr_q=0.01)
    assert len(rec) == 0 and kprov == 0 and math.isinf(thr)
    z = torch.zeros((300, 16, 16), dtype=torch.float32, device=DEV)
    rec, thr, kprov, _, _ = nb.nbsi_search(z, fdr_q=0.05)
    assert len(rec) == 0 and kprov == 0


def test_search_custom_widths_and_errors():
    r = _cube(300, 16, 5, [(8, 8, 150, 5, 12.0)])
    rt = torch.from_numpy(r).to(DEV)
    rec, thr, kprov, S, W = nb.nbsi_search(rt, fdr_q=0.01, widths=[5, 1, 3, 5], want_cubes=True)
    torch.cuda.synchronize()
    _check_bank(r, S, W, widths=(1, 3, 5))
    assert any(a["x"] == 8 and a["y"] == 8 and a["width"] == 5 for a in rec)
    for bad in ([0], [129], list(range(1, 34))):
        with pytest.raises(nb.NbsiError):
            nb.nbsi_search(rt, widths=bad)
    with pytest.raises(nb.NbsiError):
        nb.nbsi_search(rt, fdr_q=0.0)
    # every searched voxel far above any threshold: BH accepts all m of them, and constant
    # flanks (MAD 0) discard every survivor, as in the oracle
    four = torch.full((64, 16, 16), 4.0, dtype=torch.float32, device=DEV)
    rec, thr, kprov, S4, _ = nb.nbsi_search(four, fdr_q=0.05, want_cubes=True)
    torch.cuda.synchronize()
    m = int(horizon_mask(16).sum()) * 64
    rec_ref, _, _, k_ref, s_ref = osr.search(np.full((64, 16, 16), 4.0), q=0.05)
    assert kprov == k_ref == m and len(rec) == len(rec_ref) == 0
    assert np.float32(thr) == np.float32(S4.cpu().numpy()[:, horizon_mask(16)].min())


# ---- noise correlated across channels (nbsi_search_corr) ----

def _hann_ma2():
    """MA(2) coefficients (unit variance) whose channel correlations are the images' (4/9, 1/36)."""
    from scipy.optimize import fsolve

    def eq(v):
        a0, a1, a2 = v
        S = a0 * a0 + a1 * a1 + a2 * a2
        return [a0 * a2 / S - nb.HANN_CROSS_RHO[1], (a0 * a1 + a1 * a2) / S - nb.HANN_CROSS_RHO[0], S - 1.0]

    return fsolve(eq, [0.8, 0.5, 0.05])


def _corr_cube(n_chan, n_pix, seed, lines=()):
    a = _hann_ma2()
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((n_chan + 2, n_pix, n_pix))
    r = a[0] * e[2:] + a[1] * e[1:-1] + a[2] * e[:-2]
    for (x, y, c0, w, snr) in lines:
        r[c0:c0 + w, y, x] += snr * osr.boxcar_sigma(w, nb.HANN_CROSS_RHO) / w
    return r.astype(np.float32)


@pytest.mark.parametrize("seed,q", [(21, 0.01), (22, 0.1)])
def test_search_corr_matches_oracle(seed, q):
    """Hann-correlated noise with lines: the bank under rho, BH, suppression and the rho-aware
    re-evaluation against the oracle; every line found."""
    n_chan, n_pix = 640, 32
    lines = [(9, 7, 300, 12, 14.0), (20, 12, 100, 1, 10.0), (14, 20, 500, 40, 16.0), (16, 16, 600, 3, 9.0)]
    print(f"search corr seed={seed} q={q}", flush=True)
    r = _corr_cube(n_chan, n_pix, seed, lines)
    rec, thr, kprov, S, W = nb.nbsi_search(torch.from_numpy(r).to(DEV), fdr_q=q, want_cubes=True,
                                           rho=nb.HANN_CROSS_RHO)
    torch.cuda.synchronize()
    print(f"  k* {kprov} S* {thr:.4f} records {len(rec)}", flush=True)
    Sg, Wg = _check_bank(r, S, W, rho=osr.HANN_CROSS_RHO)
    valid = horizon_mask(n_pix).ravel()
    k_ref, s_ref = osr.bh_threshold(Sg[:, valid].ravel(), int(valid.sum()) * n_chan, q)
    assert kprov == k_ref and np.float32(thr) == np.float32(s_ref)
    exp = _expected_records(r, Sg, Wg, thr, n_pix, rho=osr.HANN_CROSS_RHO)
    got = {(int(a["x"]), int(a["y"]), int(a["c"])): a for a in rec}
    for key, snr2 in exp.items():
        if abs(snr2 - thr) < 1e-4 * max(1.0, thr):
            continue  # a float32 re-evaluation may fall on either side of S*
        assert (key in got) == (snr2 >= thr), (key, snr2, thr)
    for key in got:
        assert key in exp
    for (x, y, c0, w, snr) in lines:
        hits = [k for k in got if k[0] == x and k[1] == y and abs(k[2] - (c0 + w // 2)) <= max(2, w // 2)]
        assert hits, (x, y, c0, w)


def test_search_corr_noise_only_and_errors():
    """Correlated noise alone: BH admits nothing under the matching rho and a great many voxels
    under the white-noise scale; invalid correlations are rejected."""
    r = torch.from_numpy(_corr_cube(512, 32, 23)).to(DEV)
    rec, thr, kprov, _, _ = nb.nbsi_search(r, fdr_q=0.01, rho=nb.HANN_CROSS_RHO)
    assert kprov == 0 and len(rec) == 0 and math.isinf(thr)
    _, _, k_white, _, _ = nb.nbsi_search(r, fdr_q=0.01)
    assert k_white > 100
    for bad in ([0.5] * 9, [1.0], [-1.0], [float("nan")], [-0.99]):
        with pytest.raises(nb.NbsiError):
            nb.nbsi_search(r, rho=bad)
