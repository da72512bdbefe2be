"""Pins of the calibration-apply oracle (oracle.calibrate) against closed forms (no GPU)."""
import numpy as np
import pytest

import oracle


def _rand(n_chan, n_in, seed):
    rng = np.random.default_rng(seed)
    nprod = n_in * (n_in + 1) // 2
    vis = rng.integers(-1000, 1000, size=(n_chan, nprod, 2)).astype(np.int32)
    cal = rng.standard_normal((n_chan, n_in, 2))
    return vis, cal


def test_identity_and_scaling():
    vis, cal = _rand(3, 7, 1)
    one = np.zeros_like(cal)
    one[..., 0] = 1.0
    np.testing.assert_array_equal(oracle.calibrate(vis, one), vis.astype(np.float64))
    # a real factor 2 on input 4 doubles its row and column; its auto four times
    two = one.copy()
    two[:, 4, 0] = 2.0
    out = oracle.calibrate(vis, two)
    for i in range(7):
        for j in range(i + 1):
            f = (2.0 if i == 4 else 1.0) * (2.0 if j == 4 else 1.0)
            t = oracle.tri_index(i, j)
            np.testing.assert_array_equal(out[:, t], f * vis[:, t])


def test_phase_only_two_inputs_by_hand():
    # V_10 = 3 + 4i, w_1 = exp(i pi/2) = i, w_0 = 1: V' = i (3 + 4i) = -4 + 3i
    vis = np.zeros((1, 3, 2), dtype=np.int32)
    vis[0, oracle.tri_index(1, 0)] = (3, 4)
    vis[0, oracle.tri_index(1, 1)] = (25, 0)
    cal = np.zeros((1, 2, 2))
    cal[0, 0] = (1.0, 0.0)
    cal[0, 1] = (0.0, 1.0)
    out = oracle.calibrate(vis, cal)
    assert tuple(out[0, oracle.tri_index(1, 0)]) == pytest.approx((-4.0, 3.0), abs=1e-15)
    # an auto stays real: |w|^2 V_ii
    assert tuple(out[0, oracle.tri_index(1, 1)]) == pytest.approx((25.0, 0.0), abs=1e-15)


def test_recovers_gain_corrupted_visibilities():
    # V_measured = g_i V_true conj(g_j); correcting with w = 1/g gives V_true back
    rng = np.random.default_rng(4)
    n_chan, n_in = 4, 9
    q = rng.standard_normal((n_chan, n_in, 30)) + 1j * rng.standard_normal((n_chan, n_in, 30))
    g = rng.uniform(0.5, 2.0, (n_chan, n_in)) * np.exp(1j * rng.uniform(-np.pi, np.pi, (n_chan, n_in)))
    i, j = np.tril_indices(n_in)
    order = np.argsort(oracle.tri_index(i, j))
    i, j = i[order], j[order]
    vtrue = np.einsum("cis,cjs->cij", q, np.conj(q))[:, i, j]
    vmeas = g[:, i] * vtrue * np.conj(g[:, j])
    w = 1.0 / g
    out = oracle.calibrate(np.stack([vmeas.real, vmeas.imag], -1), np.stack([w.real, w.imag], -1))
    np.testing.assert_allclose(out[..., 0] + 1j * out[..., 1], vtrue, rtol=1e-12, atol=1e-9)
