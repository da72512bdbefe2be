"""Pins of the oracle direct-Fourier imager (Sec. 2.2: all-sky imaging of each fine channel).

I(l, m) = (1/|B|) sum_{a>b} Re[V_I exp(-2 pi i (u l + v m))], V_I = (V_XX + V_YY)/2,
l = (x - N/2) 2/N, m = (y - N/2) 2/N.
"""
import numpy as np
import pytest

import synth

C = synth.C_LIGHT


def _vis_from_baseline_values(n_ant, values):
    """Fill XX and YY of every pair a > b with values[(a, b)] (float64 vis array [1][nprod][2])."""
    n_in = 2 * n_ant
    vis = np.zeros((1, n_in * (n_in + 1) // 2, 2))
    for (a, b), z in values.items():
        for p in (0, 1):
            i, j = 2 * a + p, 2 * b + p
            t = i * (i + 1) // 2 + j
            vis[0, t] = (z.real, z.imag)
    return vis


def test_single_baseline_fringe(orc):
    # Antenna 1 at x = 4 m, antenna 0 at the origin, nu = c: u = 4 wavelengths exactly, v = 0.
    xyz = np.array([[0.0, 0, 0], [4.0, 0, 0]])
    freq = np.array([C])
    n = 64
    img = orc.image_dft(_vis_from_baseline_values(2, {(1, 0): 1 + 0j}), xyz, freq, n)[0]
    # u l = (x - 32)/8: cos fringe with an 8 pixel period, constant along y
    np.testing.assert_allclose(img[:, 32], 1.0, atol=1e-12)
    np.testing.assert_allclose(img[:, 34], 0.0, atol=1e-12)
    np.testing.assert_allclose(img[:, 36], -1.0, atol=1e-12)
    np.testing.assert_allclose(img[:, 33], np.sqrt(0.5), atol=1e-12)
    img_i = orc.image_dft(_vis_from_baseline_values(2, {(1, 0): 1j}), xyz, freq, n)[0]
    # V = i gives sin: +1 a quarter period to the right of the centre
    np.testing.assert_allclose(img_i[:, 34], 1.0, atol=1e-12)
    np.testing.assert_allclose(img_i[:, 30], -1.0, atol=1e-12)


def test_stokes_i_averages_xx_and_yy(orc):
    xyz = np.array([[0.0, 0, 0], [4.0, 0, 0]])
    vis = np.zeros((1, 10, 2))
    vis[0, 3] = (3.0, 0)   # XX of (1, 0): t(2, 0)
    vis[0, 7] = (1.0, 0)   # YY of (1, 0): t(3, 1)
    vis[0, 4] = (100, 100)  # a cross-hand product: must be ignored
    img = orc.image_dft(vis, xyz, np.array([C]), 16)[0]
    np.testing.assert_allclose(img[8, 8], 2.0, atol=1e-12)


def _point_source_vis(xyz, nu, l0, m0):
    vals = {}
    for a in range(xyz.shape[0]):
        for b in range(a):
            u = (xyz[a, 0] - xyz[b, 0]) * nu / C
            v = (xyz[a, 1] - xyz[b, 1]) * nu / C
            vals[(a, b)] = np.exp(2j * np.pi * (u * l0 + v * m0))
    return _vis_from_baseline_values(xyz.shape[0], vals)


def test_point_source_is_shifted_beam(orc):
    n = 32
    xyz = synth.antenna_layout(12, 100.0, seed=5)
    nu = np.array([70e6])
    beam = orc.image_dft(_point_source_vis(xyz, 70e6, 0.0, 0.0), xyz, nu, n)[0]
    assert abs(beam[n // 2, n // 2] - 1.0) < 1e-12              # B(0, 0) = 1
    assert np.abs(beam).max() <= 1.0 + 1e-12
    # beam is point-symmetric: B(-l, -m) = B(l, m)
    np.testing.assert_allclose(beam[1:, 1:], beam[1:, 1:][::-1, ::-1], atol=1e-12)
    dx, dy = 5, -3
    l0, m0 = dx * 2.0 / n, dy * 2.0 / n
    img = orc.image_dft(_point_source_vis(xyz, 70e6, l0, m0), xyz, nu, n)[0]
    assert abs(img[n // 2 + dy, n // 2 + dx] - 1.0) < 1e-12
    # I(l, m) = B(l - l0, m - m0) on the overlap of the two pixel grids
    np.testing.assert_allclose(img[max(0, dy):n + min(0, dy), max(0, dx):n + min(0, dx)],
                               beam[max(0, -dy):n - max(0, dy), max(0, -dx):n - max(0, dx)],
                               atol=1e-11)


def test_zero_and_linearity(orc):
    n = 16
    xyz = synth.antenna_layout(6, 50.0, seed=2)
    freq = np.array([60e6, 80e6])
    rng = np.random.default_rng(0)
    nprod = 12 * 13 // 2
    v1 = rng.standard_normal((2, nprod, 2))
    v2 = rng.standard_normal((2, nprod, 2))
    assert np.abs(orc.image_dft(np.zeros_like(v1), xyz, freq, n)).max() == 0.0
    lhs = orc.image_dft(2.5 * v1 - 0.5 * v2, xyz, freq, n)
    rhs = 2.5 * orc.image_dft(v1, xyz, freq, n) - 0.5 * orc.image_dft(v2, xyz, freq, n)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_grid_uv_box_count_bruteforce(orc):
    xyz = synth.antenna_layout(352, 750.0, seed=2001)
    freq = np.array([69.9e6, 70.0e6, 70.1e6])
    for n_pix in (128, 256):
        U = (2 * n_pix / 2 - 8 / 2 - 1) * 0.25
        a, b = np.tril_indices(352, -1)
        for k, nu in enumerate(freq):
            u = (xyz[a, 0] - xyz[b, 0]) * nu / C
            v = (xyz[a, 1] - xyz[b, 1]) * nu / C
            expect = np.count_nonzero((np.abs(u) <= U) & (np.abs(v) <= U))
            assert orc.count_baselines(xyz, freq[k:k + 1], n_pix)[0] == expect
    # no cut: every pair a > b
    assert orc.count_baselines(xyz, freq[:1])[0] == 352 * 351 // 2


def test_uv_range_cut(orc):
    xyz = np.array([[0.0, 0, 0], [4.0, 0, 0], [0, 10.0, 0]])
    # nu = c: |uv| of (1,0) = 4, (2,0) = 10, (2,1) = sqrt(116)
    n_b = orc.count_baselines(xyz, np.array([C]), 0, 5.0, 10.5)
    assert n_b[0] == 1


@pytest.mark.parametrize("grid_n_pix,uv_min,uv_max", [(0, 0.0, np.inf), (32, 0.0, np.inf), (0, 2.0, 9.0)])
def test_pixel_list_equals_full_image(orc, grid_n_pix, uv_min, uv_max):
    # the direct Fourier image evaluated at a list of pixels is the full image at those pixels
    # (the same sum, written a second time for large images), for every baseline-set rule
    rng = np.random.default_rng(17)
    n_ant, n_chan, n = 12, 3, 32
    xyz = np.zeros((n_ant, 3))
    xyz[:, :2] = rng.uniform(-40.0, 40.0, (n_ant, 2))
    freq = 70e6 + 1e3 * np.arange(n_chan)
    n_in = 2 * n_ant
    vis = rng.standard_normal((n_chan, n_in * (n_in + 1) // 2, 2)) * 100.0
    full = orc.image_dft(vis, xyz, freq, n, grid_n_pix, uv_min, uv_max)
    pix = np.array([(0, 0), (31, 31), (16, 16), (3, 29), (29, 3), (7, 11), (16, 0), (0, 16)])
    got = orc.image_dft_pixels(vis, xyz, freq, n, pix, grid_n_pix, uv_min, uv_max)
    ref = full[:, pix[:, 1], pix[:, 0]]
    assert np.abs(ref).max() > 1.0
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(full).max())
