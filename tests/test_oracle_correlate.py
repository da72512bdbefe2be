"""Pins of the oracle correlator: the full cross-correlation of Sec. 2.1,
V_ij = sum_s q_i,s conj(q_j,s) for every pair i >= j, stored as a packed lower triangle."""
import numpy as np
import pytest

import synth


def test_bruteforce_python_ints(orc):
    rng = np.random.default_rng(11)
    n_chan, n_in, T = 2, 5, 7
    q = rng.integers(-128, 128, size=(n_chan, n_in, 2, T)).astype(np.int8)
    vis = orc.correlate(q)
    for c in range(n_chan):
        for i in range(n_in):
            for j in range(i + 1):
                acc = 0j
                for s in range(T):
                    a = complex(int(q[c, i, 0, s]), int(q[c, i, 1, s]))
                    b = complex(int(q[c, j, 0, s]), int(q[c, j, 1, s]))
                    acc += a * b.conjugate()
                t = i * (i + 1) // 2 + j
                assert vis[c, t, 0] == int(acc.real) and vis[c, t, 1] == int(acc.imag)


def test_matches_int64_matrix_product(orc):
    q = synth.random_spectra(3, 40, 33, seed=3).numpy()
    vis = orc.correlate(q)
    z = q[:, :, 0, :].astype(np.int64) + 1j * q[:, :, 1, :].astype(np.int64)
    # exact in complex128 for these magnitudes (< 2^53)
    full = np.einsum("cis,cjs->cij", z, np.conj(z))
    i, j = np.tril_indices(40)
    t = i * (i + 1) // 2 + j
    np.testing.assert_array_equal(vis[:, t, 0], full[:, i, j].real.astype(np.int64))
    np.testing.assert_array_equal(vis[:, t, 1], full[:, i, j].imag.astype(np.int64))


def test_autocorrelations_real_nonnegative(orc):
    q = synth.random_spectra(4, 17, 20, seed=9, full_range=True).numpy()
    vis = orc.correlate(q)
    t = np.arange(17) * (np.arange(17) + 1) // 2 + np.arange(17)
    assert (vis[:, t, 1] == 0).all()
    power = (q.astype(np.int64) ** 2).sum(axis=(2, 3))
    np.testing.assert_array_equal(vis[:, t, 0], power)


def test_constant_input(orc):
    T = 9
    vals = np.array([3 - 4j, -127 + 127j, 5j, -2])
    q = np.zeros((1, 4, 2, T), np.int8)
    q[0, :, 0, :] = vals.real[:, None]
    q[0, :, 1, :] = vals.imag[:, None]
    vis = orc.correlate(q)
    for i in range(4):
        for j in range(i + 1):
            e = T * vals[i] * np.conj(vals[j])
            t = i * (i + 1) // 2 + j
            assert vis[0, t, 0] == e.real and vis[0, t, 1] == e.imag


def test_int32_bound_at_65535_spectra(orc):
    # All -128: Re V = 2 * 128^2 * T = 2147450880 < 2^31 at T = 65535, overflows at 65536.
    q = np.full((1, 2, 2, 65535), -128, np.int8)
    vis = orc.correlate(q)
    assert vis[0, 0, 0] == 2 * 128 * 128 * 65535
    q2 = np.full((1, 1, 2, 65536), -128, np.int8)
    with pytest.raises(OverflowError):
        orc.correlate(q2)
