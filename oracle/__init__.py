"""Plain CPU oracle of the hot path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this package.
The product library never does.  The C part (oracle.c: FFT, DFT, channelizer, requantiser,
correlator, direct-Fourier imager) is built with gcc into liboracle.so next to this file;
the detector and classifier oracles are plain numpy (detect.py, net.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no fast-math) into liboracle.so."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int, ctypes.c_long, ctypes.c_double
        L.orc_fft_ri.argtypes = [P, i64]
        L.orc_dft.argtypes = [P, P, i64]
        L.orc_hann.argtypes = [i64, i64]
        L.orc_hann.restype = f64
        L.orc_channelize.argtypes = [P, i32, i32, i32, i32, i32, P]
        L.orc_requantize.argtypes = [P, i32, i32, i32, P, P]
        L.orc_correlate.argtypes = [P, i32, i32, i32, P]
        L.orc_count_baselines.argtypes = [i32, i32, P, P, i32, f64, f64, P]
        L.orc_image_dft.argtypes = [P, i32, i32, P, P, i32, i32, f64, f64, P]
        L.orc_image_dft_pixels.argtypes = [P, i32, i32, P, P, i32, i32, f64, f64, P, i32, P]
        L.orc_set_threads.argtypes = [i32]
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def fft(x: np.ndarray) -> np.ndarray:
    """Forward FFT (radix-2, FP64) of a complex vector."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    if lib().orc_fft_ri(_p(a), a.size) != 0:
        raise ValueError("length must be a power of two")
    return a


def dft(x: np.ndarray) -> np.ndarray:
    """O(N^2) DFT, the definition."""
    a = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(a)
    lib().orc_dft(_p(a), _p(out), a.size)
    return out


def hann(n_fft: int) -> np.ndarray:
    return np.array([lib().orc_hann(n, n_fft) for n in range(n_fft)])


def channelize(volt: np.ndarray, n_fft: int, n_spec: int, chan0: int, n_chan: int) -> np.ndarray:
    """volt [n_in][n_spec*n_fft][2] int8 -> complex128 [n_chan][n_in][n_spec]."""
    v = np.ascontiguousarray(volt, dtype=np.int8)
    n_in = v.shape[0]
    assert v.shape == (n_in, n_spec * n_fft, 2)
    out = np.empty((n_chan, n_in, n_spec, 2), dtype=np.float64)
    rc = lib().orc_channelize(_p(v), n_in, n_fft, n_spec, chan0, n_chan, _p(out))
    if rc != 0:
        raise ValueError(f"orc_channelize failed ({rc})")
    return out[..., 0] + 1j * out[..., 1]


def requantize(spec: np.ndarray, gain: np.ndarray) -> np.ndarray:
    """complex [n_chan][n_in][n_spec] -> int8 [n_chan][n_in][2][n_spec]."""
    n_chan, n_in, n_spec = spec.shape
    ri = np.ascontiguousarray(np.stack([spec.real, spec.imag], axis=-1), dtype=np.float64)
    g = np.ascontiguousarray(gain, dtype=np.float32)
    q = np.empty((n_chan, n_in, 2, n_spec), dtype=np.int8)
    lib().orc_requantize(_p(ri), n_chan, n_in, n_spec, _p(g), _p(q))
    return q


def correlate(q: np.ndarray) -> np.ndarray:
    """int8 [n_chan][n_in][2][n_spec] -> int32 [n_chan][n_in(n_in+1)/2][2]."""
    q = np.ascontiguousarray(q, dtype=np.int8)
    n_chan, n_in, two, n_spec = q.shape
    assert two == 2
    vis = np.empty((n_chan, n_in * (n_in + 1) // 2, 2), dtype=np.int32)
    rc = lib().orc_correlate(_p(q), n_chan, n_in, n_spec, _p(vis))
    if rc != 0:
        raise OverflowError("visibility does not fit in int32")
    return vis


def count_baselines(ant_xyz, freq, grid_n_pix: int = 0, uv_min: float = 0.0,
                    uv_max: float = np.inf) -> np.ndarray:
    xyz = np.ascontiguousarray(ant_xyz, dtype=np.float64)
    f = np.ascontiguousarray(freq, dtype=np.float64)
    n_b = np.empty(f.size, dtype=np.int64)
    lib().orc_count_baselines(f.size, xyz.shape[0], _p(xyz), _p(f), int(grid_n_pix),
                              float(uv_min), float(uv_max), _p(n_b))
    return n_b


def image_dft(vis: np.ndarray, ant_xyz, freq, n_pix: int, grid_n_pix: int = 0,
              uv_min: float = 0.0, uv_max: float = np.inf) -> np.ndarray:
    """vis [n_chan][nprod][2] (int32 or float) -> image [n_chan][n_pix][n_pix] float64.

    grid_n_pix > 0 restricts B to the gridded method's uv box for an image of that size."""
    v = np.ascontiguousarray(vis, dtype=np.float64)
    xyz = np.ascontiguousarray(ant_xyz, dtype=np.float64)
    f = np.ascontiguousarray(freq, dtype=np.float64)
    n_chan = v.shape[0]
    assert f.size == n_chan
    img = np.empty((n_chan, n_pix, n_pix), dtype=np.float64)
    rc = lib().orc_image_dft(_p(v), n_chan, xyz.shape[0], _p(xyz), _p(f), n_pix, int(grid_n_pix),
                             float(uv_min), float(uv_max), _p(img))
    if rc != 0:
        raise MemoryError("orc_image_dft failed")
    return img


def image_dft_pixels(vis: np.ndarray, ant_xyz, freq, n_pix: int, pix_xy, grid_n_pix: int = 0,
                     uv_min: float = 0.0, uv_max: float = np.inf) -> np.ndarray:
    """The direct Fourier image at the listed pixels only: pix_xy [n][2] (x, y) -> [n_chan][n]."""
    v = np.ascontiguousarray(vis, dtype=np.float64)
    xyz = np.ascontiguousarray(ant_xyz, dtype=np.float64)
    f = np.ascontiguousarray(freq, dtype=np.float64)
    pix = np.ascontiguousarray(pix_xy, dtype=np.int32)
    out = np.empty((v.shape[0], pix.shape[0]), dtype=np.float64)
    rc = lib().orc_image_dft_pixels(_p(v), v.shape[0], xyz.shape[0], _p(xyz), _p(f), n_pix,
                                    int(grid_n_pix), float(uv_min), float(uv_max), _p(pix),
                                    pix.shape[0], _p(out))
    if rc != 0:
        raise MemoryError("orc_image_dft_pixels failed")
    return out


def calibrate(vis: np.ndarray, cal: np.ndarray) -> np.ndarray:
    """Apply calibration solutions (Sec. 2.2) to visibilities: vis [n_chan][nprod][2] (packed
    lower triangle, input i >= j), cal [n_chan][n_in][2] complex correction factors w (the inverse
    of the measured gains, bandpass included):  V'_ij = w_i V_ij conj(w_j), in float64."""
    v = np.asarray(vis, dtype=np.float64)
    w = np.asarray(cal, dtype=np.float64)
    wc = w[..., 0] + 1j * w[..., 1]                       # [n_chan][n_in]
    n_in = wc.shape[1]
    i, j = np.tril_indices(n_in)                          # row-major over i, then j <= i
    order = np.argsort(tri_index(i, j))
    i, j = i[order], j[order]
    vc = v[..., 0] + 1j * v[..., 1]
    out = wc[:, i] * vc * np.conj(wc[:, j])
    return np.stack([out.real, out.imag], axis=-1)


def tri_index(i, j):
    """Packed lower-triangle index t(i, j) = i(i+1)/2 + j, i >= j."""
    return i * (i + 1) // 2 + j


from . import detect  # noqa: E402  (numpy detector oracle)
from . import net  # noqa: E402  (numpy classifier oracle)
from . import search  # noqa: E402  (numpy full Stage I search oracle)
from . import drift  # noqa: E402  (numpy drift-rate search oracle)
from . import stage2  # noqa: E402  (numpy/SciPy Stage II cuts and Gaussian centroid fits)
