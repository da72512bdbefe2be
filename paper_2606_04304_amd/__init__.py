"""Python binding of libnbsi (include/nbsi.h): argument marshalling only.

Every function has the name of the C entry point it wraps and enqueues that entry point on
torch's current HIP stream.  Tensors must be on the context's device, contiguous and of the
documented dtype; outputs are allocated with torch when not supplied.  All computation runs
in the HIP kernels of libnbsi.so; if the library is missing this module raises on first use.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbsi.so")

NBSI_OK = 0
NBSI_EINVAL = -1
NBSI_EOVERFLOW = -2
NBSI_ENOMEM = -3
NBSI_EHIP = -4
NBSI_ETRUNC = -5
NBSI_EUNSUPPORTED = -6
NBSI_MAX_SPEC = 65535
NBSI_IMAGE_DFT = 0
NBSI_IMAGE_GRID = 1
NBSI_VIS_I32 = 0
NBSI_VIS_F32 = 1
NBSI_PREC_FP32 = 0
NBSI_PREC_FP16 = 1
NBSI_PREC_BF16 = 2
NBSI_DETECT_PER_PIXEL = 0
NBSI_DETECT_PER_IMAGE = 1

EXPORTS = [
    "nbsi_version", "nbsi_strerror", "nbsi_create", "nbsi_destroy", "nbsi_set_stream",
    "nbsi_last_error", "nbsi_synchronize", "nbsi_check_channelize", "nbsi_check_correlate",
    "nbsi_check_image", "nbsi_check_detect", "nbsi_channelize", "nbsi_correlate",
    "nbsi_correlate_f32", "nbsi_image_plan_create", "nbsi_image_plan_destroy",
    "nbsi_image_plan_nbase", "nbsi_image", "nbsi_detect", "nbsi_batch_plan", "nbsi_batch_run",
    "nbsi_batch_describe", "nbsi_batch_destroy", "nbsi_stamps", "nbsi_net_create", "nbsi_net_destroy",
    "nbsi_net_set_params", "nbsi_net_get_params", "nbsi_net_forward", "nbsi_net_grad", "nbsi_net_adam",
    "nbsi_net_train_step", "nbsi_correlate_kernel", "nbsi_image_plan_pairs", "nbsi_correlate_stokes",
    "nbsi_image_stokes", "nbsi_correlate_image", "nbsi_search", "nbsi_search_corr", "nbsi_correlate_cal", "nbsi_dedoppler", "nbsi_beam", "nbsi_stage2",
    "nbsi_detect_noalloc", "nbsi_status",
]
NBSI_FLAG_SPEC_NONFINITE = 0x1
NBSI_FLAG_SPEC_CLIPPED = 0x2
NBSI_FLAG_IMAGE_NONFINITE = 0x4
NBSI_FLAG_CUBE_NONFINITE = 0x8
NBSI_DETECT_NOALLOC_MAX_CANDS = 65536
NBSI_DETECT_NOALLOC_BYTES = 2097408
NBSI_DEDOPPLER_MAX_SUB = 8
NBSI_DEDOPPLER_MAX_DRIFT = 16
NBSI_S2_FIT_FAILED, NBSI_S2_EXTENDED, NBSI_S2_NOISY, NBSI_S2_OUTSIDE = 1, 2, 4, 8
NBSI_S2_MAX_HALF = 5
NBSI_S2_MAX_CANDS = 1 << 22
NBSI_BEAM_HALF = 2
NBSI_SEARCH_MAX_WIDTHS = 32
NBSI_SEARCH_MAX_WIDTH = 128
NBSI_SEARCH_MAX_LAG = 8
# Channel correlations of the noise of this library's images (periodic Hann window: the windowed
# spectra's neighbouring channels correlate at -2/3 and 1/6 at lags 1 and 2, so the
# cross-correlations of independent inputs, and the images made of them, at 4/9 and 1/36):
# nbsi_search(..., rho=HANN_CROSS_RHO) on an SNR cube of those images.
HANN_CROSS_RHO = (4.0 / 9.0, 1.0 / 36.0)
NBSI_STAMP_CHANNELS = 33
NBSI_STAMP_PIXELS = 9
NBSI_NET_NPARAM = 46529
NBSI_NET_MAX_BATCH = 8192
NBSI_BATCH_GRAPH = 1
NBSI_BATCH_AUTOTUNE = 2
NBSI_BATCH_GRID_TALL = 4
NBSI_BATCH_OVERLAP = 8

CAND_DTYPE = np.dtype([("x", np.int32), ("y", np.int32), ("c", np.int32), ("width", np.int32),
                       ("snr", np.float32)])
# nbsi_fit (160 bytes)
FIT_DTYPE = np.dtype([("amp", np.float64), ("x0", np.float64), ("y0", np.float64), ("a", np.float64),
                      ("b", np.float64), ("c", np.float64), ("bkg", np.float64), ("err", np.float64, (7,)),
                      ("fwhm_maj", np.float64), ("fwhm_min", np.float64), ("pa", np.float64),
                      ("rss", np.float64), ("chi2_red", np.float64), ("flags", np.int32), ("n_iter", np.int32)])
assert FIT_DTYPE.itemsize == 160


class NbsiError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        msg = lib().nbsi_strerror(status).decode()
        super().__init__(f"{msg} ({status}){': ' + detail if detail else ''}")


_lib = None


def lib():
    """Load libnbsi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.nbsi_version.restype = I
        L.nbsi_strerror.argtypes = [I]
        L.nbsi_strerror.restype = ctypes.c_char_p
        L.nbsi_create.argtypes = [ctypes.POINTER(P), I, P]
        L.nbsi_destroy.argtypes = [P]
        L.nbsi_set_stream.argtypes = [P, P]
        L.nbsi_last_error.argtypes = [P]
        L.nbsi_last_error.restype = ctypes.c_char_p
        L.nbsi_synchronize.argtypes = [P]
        L.nbsi_status.argtypes = [P, ctypes.POINTER(ctypes.c_uint32)]
        L.nbsi_check_channelize.argtypes = [I, I, I, I, I]
        L.nbsi_check_correlate.argtypes = [I, I, I]
        L.nbsi_check_image.argtypes = [I, I, I, I, I, D, D]
        L.nbsi_check_detect.argtypes = [I, I, I, I]
        L.nbsi_channelize.argtypes = [P, P, I, I, I, I, I, P, P, P]
        L.nbsi_correlate.argtypes = [P, P, I, I, I, P]
        L.nbsi_correlate_f32.argtypes = [P, P, I, I, I, P]
        L.nbsi_correlate_cal.argtypes = [P, P, I, I, I, P, P]
        L.nbsi_dedoppler.argtypes = [P, P, I, I, I, I, P, P]
        L.nbsi_beam.argtypes = [P, P, P]
        L.nbsi_stage2.argtypes = [P, P, I, I, P, I, P, I, D, D, P]
        L.nbsi_image_plan_create.argtypes = [P, P, I, P, I, I, I, D, D, ctypes.POINTER(P)]
        L.nbsi_image_plan_destroy.argtypes = [P]
        L.nbsi_image_plan_nbase.argtypes = [P, P]
        L.nbsi_image.argtypes = [P, P, P, I, I, P]
        L.nbsi_image_plan_pairs.argtypes = [P, ctypes.POINTER(I), P]
        L.nbsi_correlate_stokes.argtypes = [P, P, I, I, I, P, P, P]
        L.nbsi_image_stokes.argtypes = [P, P, P, I, P]
        L.nbsi_correlate_image.argtypes = [P, P, I, I, I, P, I, I, P, P, P]
        L.nbsi_search.argtypes = [P, P, I, I, P, I, D, P, P, P, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_float),
                                  ctypes.POINTER(ctypes.c_int64)]
        L.nbsi_search_corr.argtypes = [P, P, I, I, P, I, P, I, D, P, P, P, I, ctypes.POINTER(I),
                                       ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int64)]
        L.nbsi_detect.argtypes = [P, P, I, I, I, ctypes.c_float, P, P, I, P]
        L.nbsi_detect_noalloc.argtypes = [P, P, I, I, I, ctypes.c_float, P, P, I, P]
        L.nbsi_batch_plan.argtypes = [P, P, I, P, I, I, I, ctypes.c_char_p, ctypes.POINTER(P)]
        L.nbsi_batch_run.argtypes = [P]
        L.nbsi_batch_describe.argtypes = [P, ctypes.c_char_p, I]
        L.nbsi_batch_destroy.argtypes = [P]
        L.nbsi_correlate_kernel.argtypes = [I, I]
        L.nbsi_correlate_kernel.restype = ctypes.c_char_p
        F = ctypes.c_float
        L.nbsi_stamps.argtypes = [P, P, I, I, P, I, P]
        L.nbsi_net_create.argtypes = [P, P, I, ctypes.POINTER(P)]
        L.nbsi_net_destroy.argtypes = [P]
        L.nbsi_net_set_params.argtypes = [P, P]
        L.nbsi_net_get_params.argtypes = [P, P]
        L.nbsi_net_forward.argtypes = [P, P, I, P, I, P]
        L.nbsi_net_grad.argtypes = [P, P, I, P, P, I, P, P]
        L.nbsi_net_adam.argtypes = [P, P, F, F, F, F]
        L.nbsi_net_train_step.argtypes = [P, P, I, P, P, I, F, P]
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _check(status: int, ctx=None):
    if status != NBSI_OK:
        detail = lib().nbsi_last_error(ctx._h).decode() if ctx is not None and ctx._h else ""
        raise NbsiError(status, detail)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, dtype, name, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name}: expected a contiguous {dtype} tensor")
    if t.device != device:
        raise ValueError(f"{name}: tensor on {t.device}, context on {device}")


class Context:
    """nbsi_create / nbsi_destroy around one HIP device; calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _check(lib().nbsi_create(ctypes.byref(h), int(device), None))
        self._h = h

    def _sync_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device).cuda_stream
        lib().nbsi_set_stream(self._h, ctypes.c_void_p(s))

    def close(self):
        if getattr(self, "_h", None):
            lib().nbsi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def nbsi_status(ctx: "Context | None" = None) -> int:
    """Wait for the context's work and return (and clear) its NBSI_FLAG_* bits."""
    ctx = ctx or nbsi_create(0)
    ctx._sync_stream()
    f = ctypes.c_uint32(0)
    _check(lib().nbsi_status(ctx._h, ctypes.byref(f)), ctx)
    return int(f.value)


def nbsi_create(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def nbsi_channelize(volt, n_fft: int, n_spec: int, chan0: int, n_chan: int, gain,
                    want_q: bool = True, want_f: bool = False, spec_q=None, spec_f=None,
                    ctx: Context | None = None):
    """volt [n_in][n_spec*n_fft][2] int8, gain [n_in] float32 -> (spec_q, spec_f), each
    [n_chan][n_in][2][n_spec] (int8 / float32) or None."""
    torch = _torch()
    ctx = ctx or nbsi_create(volt.device.index or 0)
    _need(volt, torch.int8, "volt", ctx.device)
    _need(gain, torch.float32, "gain", ctx.device)
    n_in = volt.shape[0]
    if want_q and spec_q is None:
        spec_q = torch.empty((n_chan, n_in, 2, n_spec), dtype=torch.int8, device=ctx.device)
    if want_f and spec_f is None:
        spec_f = torch.empty((n_chan, n_in, 2, n_spec), dtype=torch.float32, device=ctx.device)
    ctx._sync_stream()
    _check(lib().nbsi_channelize(ctx._h, _ptr(volt), n_in, n_fft, n_spec, chan0, n_chan, _ptr(gain),
                                 _ptr(spec_q) if want_q else None, _ptr(spec_f) if want_f else None),
           ctx)
    return (spec_q if want_q else None), (spec_f if want_f else None)


def nbsi_correlate(spec_q, vis=None, ctx: Context | None = None):
    """spec_q [n_chan][n_in][2][n_spec] int8 -> vis [n_chan][n_in(n_in+1)/2][2] int32."""
    torch = _torch()
    ctx = ctx or nbsi_create(spec_q.device.index or 0)
    _need(spec_q, torch.int8, "spec_q", ctx.device)
    n_chan, n_in, two, n_spec = spec_q.shape
    if vis is None:
        vis = torch.empty((n_chan, n_in * (n_in + 1) // 2, 2), dtype=torch.int32, device=ctx.device)
    ctx._sync_stream()
    _check(lib().nbsi_correlate(ctx._h, _ptr(spec_q), n_chan, n_in, n_spec, _ptr(vis)), ctx)
    return vis


def nbsi_correlate_cal(spec_q, cal, vis=None, ctx: Context | None = None):
    """spec_q int8 + cal [n_chan][n_in][2] float32 correction factors -> calibrated visibilities
    w_i V_ij conj(w_j) [n_chan][n_in(n_in+1)/2][2] float32."""
    torch = _torch()
    ctx = ctx or nbsi_create(spec_q.device.index or 0)
    _need(spec_q, torch.int8, "spec_q", ctx.device)
    _need(cal, torch.float32, "cal", ctx.device)
    n_chan, n_in, two, n_spec = spec_q.shape
    if tuple(cal.shape) != (n_chan, n_in, 2):
        raise ValueError(f"cal shape {tuple(cal.shape)} does not match spec_q")
    if vis is None:
        vis = torch.empty((n_chan, n_in * (n_in + 1) // 2, 2), dtype=torch.float32, device=ctx.device)
    _need(vis, torch.float32, "vis", ctx.device)
    if tuple(vis.shape) != (n_chan, n_in * (n_in + 1) // 2, 2):
        raise ValueError(f"vis shape {tuple(vis.shape)} does not match spec_q")
    ctx._sync_stream()
    _check(lib().nbsi_correlate_cal(ctx._h, _ptr(spec_q), n_chan, n_in, n_spec, _ptr(cal), _ptr(vis)), ctx)
    return vis


def nbsi_correlate_kernel(n_in: int, n_spec: int) -> str:
    """Name of the kernel nbsi_correlate runs for this shape."""
    return lib().nbsi_correlate_kernel(int(n_in), int(n_spec)).decode()


def nbsi_correlate_f32(spec_f, vis=None, ctx: Context | None = None):
    torch = _torch()
    ctx = ctx or nbsi_create(spec_f.device.index or 0)
    _need(spec_f, torch.float32, "spec_f", ctx.device)
    n_chan, n_in, two, n_spec = spec_f.shape
    if vis is None:
        vis = torch.empty((n_chan, n_in * (n_in + 1) // 2, 2), dtype=torch.float32, device=ctx.device)
    ctx._sync_stream()
    _check(lib().nbsi_correlate_f32(ctx._h, _ptr(spec_f), n_chan, n_in, n_spec, _ptr(vis)), ctx)
    return vis


class ImagePlan:
    """nbsi_image_plan_create / destroy."""

    def __init__(self, ant_xyz, freq_hz, n_pix: int, method: int = NBSI_IMAGE_GRID,
                 uv_min: float = 0.0, uv_max: float = float("inf"), ctx: Context | None = None):
        self.ctx = ctx or nbsi_create(0)
        self.ant_xyz = np.ascontiguousarray(ant_xyz, dtype=np.float64)
        self.freq = np.ascontiguousarray(freq_hz, dtype=np.float64)
        self.n_ant = self.ant_xyz.shape[0]
        self.n_chan = self.freq.size
        self.n_pix = int(n_pix)
        self.method = int(method)
        h = ctypes.c_void_p()
        self.ctx._sync_stream()
        _check(lib().nbsi_image_plan_create(
            self.ctx._h, self.ant_xyz.ctypes.data_as(ctypes.c_void_p), self.n_ant,
            self.freq.ctypes.data_as(ctypes.c_void_p), self.n_chan, self.n_pix, self.method,
            float(uv_min), float(uv_max), ctypes.byref(h)), self.ctx)
        self._h = h

    def n_baselines(self) -> np.ndarray:
        out = np.empty(self.n_chan, dtype=np.int64)
        _check(lib().nbsi_image_plan_nbase(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def n_pairs(self) -> int:
        """Number of candidate pairs (the length of a channel's Stokes-I row)."""
        n = ctypes.c_int()
        _check(lib().nbsi_image_plan_pairs(self._h, ctypes.byref(n), None))
        return n.value

    def pairs(self) -> np.ndarray:
        """Candidate pairs [n_pairs][2] int32 (a, b), a > b, in Stokes-I row order."""
        out = np.empty((max(1, self.n_pairs()), 2), dtype=np.int32)
        n = ctypes.c_int()
        _check(lib().nbsi_image_plan_pairs(self._h, ctypes.byref(n), out.ctypes.data_as(ctypes.c_void_p)))
        return out[:n.value]

    def close(self):
        if getattr(self, "_h", None):
            lib().nbsi_image_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nbsi_image_plan_create(ant_xyz, freq_hz, n_pix, method=NBSI_IMAGE_GRID, uv_min=0.0,
                           uv_max=float("inf"), ctx=None) -> ImagePlan:
    return ImagePlan(ant_xyz, freq_hz, n_pix, method, uv_min, uv_max, ctx)


def nbsi_image(plan: ImagePlan, vis, precision: int = NBSI_PREC_FP32, img=None):
    """vis int32 or float32 [n_chan][nprod][2] -> img [n_chan][n_pix][n_pix] float32."""
    torch = _torch()
    ctx = plan.ctx
    if vis.dtype == torch.int32:
        vt = NBSI_VIS_I32
    elif vis.dtype == torch.float32:
        vt = NBSI_VIS_F32
    else:
        raise TypeError("vis must be int32 or float32")
    _need(vis, vis.dtype, "vis", ctx.device)
    n_in = 2 * plan.n_ant
    if tuple(vis.shape) != (plan.n_chan, n_in * (n_in + 1) // 2, 2):
        raise ValueError(f"vis shape {tuple(vis.shape)} does not match the plan")
    if img is None:
        img = torch.empty((plan.n_chan, plan.n_pix, plan.n_pix), dtype=torch.float32, device=ctx.device)
    ctx._sync_stream()
    _check(lib().nbsi_image(ctx._h, plan._h, _ptr(vis), vt, int(precision), _ptr(img)), ctx)
    return img


def nbsi_correlate_stokes(spec_q, plan: ImagePlan, vis=None, stokes_i=None, ctx: Context | None = None):
    """spec_q int8 -> (vis as nbsi_correlate, stokes_i [n_chan][plan.n_pairs()][2] float32).  ctx:
    the context to run on (default: the plan's), e.g. one with its own scratch for another stream."""
    torch = _torch()
    ctx = ctx or plan.ctx
    _need(spec_q, torch.int8, "spec_q", ctx.device)
    n_chan, n_in, two, n_spec = spec_q.shape
    if vis is None:
        vis = torch.empty((n_chan, n_in * (n_in + 1) // 2, 2), dtype=torch.int32, device=ctx.device)
    _need(vis, torch.int32, "vis", ctx.device)
    if tuple(vis.shape) != (n_chan, n_in * (n_in + 1) // 2, 2):
        raise ValueError(f"vis shape {tuple(vis.shape)} does not match spec_q")
    if stokes_i is None:
        stokes_i = torch.empty((n_chan, max(1, plan.n_pairs()), 2), dtype=torch.float32, device=ctx.device)
    _need(stokes_i, torch.float32, "stokes_i", ctx.device)
    if stokes_i.dim() != 3 or stokes_i.shape[0] != n_chan or stokes_i.shape[1] != max(1, plan.n_pairs()) \
            or stokes_i.shape[2] != 2:
        raise ValueError(f"stokes_i shape {tuple(stokes_i.shape)} does not match the plan")
    ctx._sync_stream()
    _check(lib().nbsi_correlate_stokes(ctx._h, _ptr(spec_q), n_chan, n_in, n_spec, plan._h, _ptr(vis),
                                       _ptr(stokes_i)), ctx)
    return vis, stokes_i


def nbsi_image_stokes(plan: ImagePlan, stokes_i, precision: int = NBSI_PREC_FP32, img=None,
                      ctx: Context | None = None):
    """stokes_i [n_chan][n_pairs][2] float32 (from nbsi_correlate_stokes) -> img, as nbsi_image
    (ctx: the context to run on, default the plan's)."""
    torch = _torch()
    ctx = ctx or plan.ctx
    _need(stokes_i, torch.float32, "stokes_i", ctx.device)
    if stokes_i.dim() != 3 or stokes_i.shape[0] != plan.n_chan or stokes_i.shape[1] != max(1, plan.n_pairs()) \
            or stokes_i.shape[2] != 2:
        raise ValueError(f"stokes_i shape {tuple(stokes_i.shape)} does not match the plan")
    if img is None:
        img = torch.empty((plan.n_chan, plan.n_pix, plan.n_pix), dtype=torch.float32, device=ctx.device)
    ctx._sync_stream()
    _check(lib().nbsi_image_stokes(ctx._h, plan._h, _ptr(stokes_i), int(precision), _ptr(img)), ctx)
    return img


def nbsi_correlate_image(spec_q, plan: ImagePlan, precision: int = NBSI_PREC_FP32, n_stages: int = 0,
                         vis=None, stokes_i=None, img=None, ctx: Context | None = None):
    """nbsi_correlate_stokes then nbsi_image_stokes, overlapped over n_stages channel ranges
    (0: the library's default) -> (vis, stokes_i, img), bit for bit those of the two calls."""
    torch = _torch()
    ctx = ctx or plan.ctx
    _need(spec_q, torch.int8, "spec_q", ctx.device)
    n_chan, n_in, two, n_spec = spec_q.shape
    nprod = n_in * (n_in + 1) // 2
    if vis is None:
        vis = torch.empty((n_chan, nprod, 2), dtype=torch.int32, device=ctx.device)
    if stokes_i is None:
        stokes_i = torch.empty((n_chan, max(1, plan.n_pairs()), 2), dtype=torch.float32, device=ctx.device)
    if img is None:
        img = torch.empty((plan.n_chan, plan.n_pix, plan.n_pix), dtype=torch.float32, device=ctx.device)
    _need(vis, torch.int32, "vis", ctx.device)
    _need(stokes_i, torch.float32, "stokes_i", ctx.device)
    _need(img, torch.float32, "img", ctx.device)
    if tuple(vis.shape) != (n_chan, nprod, 2):
        raise ValueError(f"vis shape {tuple(vis.shape)} does not match spec_q")
    if tuple(stokes_i.shape) != (n_chan, max(1, plan.n_pairs()), 2):
        raise ValueError(f"stokes_i shape {tuple(stokes_i.shape)} does not match the plan")
    if tuple(img.shape) != (plan.n_chan, plan.n_pix, plan.n_pix):
        raise ValueError(f"img shape {tuple(img.shape)} does not match the plan")
    ctx._sync_stream()
    _check(lib().nbsi_correlate_image(ctx._h, _ptr(spec_q), n_chan, n_in, n_spec, plan._h, int(precision),
                                      int(n_stages), _ptr(vis), _ptr(stokes_i), _ptr(img)), ctx)
    return vis, stokes_i, img


def nbsi_search(snr, fdr_q: float = 0.01, widths=None, max_out: int = 1 << 20, want_cubes: bool = False,
                ctx: Context | None = None, rho=None):
    """Full Stage I search of a standardised residual cube snr [n_chan][n_pix][n_pix] float32:
    (candidate records sorted by (y, x, c), BH threshold S* (inf if none), provisional count k*,
    best-SNR cube or None, best-width cube (uint8) or None).  rho: the noise's channel
    correlations at lags 1, 2, ... (None or empty: white; HANN_CROSS_RHO for this library's
    images), through nbsi_search_corr.  Blocks until done."""
    torch = _torch()
    ctx = ctx or nbsi_create(snr.device.index or 0)
    _need(snr, torch.float32, "snr", ctx.device)
    n_chan, n_pix, _ = snr.shape
    S = torch.empty_like(snr) if want_cubes else None
    W = torch.empty(snr.shape, dtype=torch.uint8, device=ctx.device) if want_cubes else None
    out = torch.empty((max(1, max_out), 5), dtype=torch.int32, device=ctx.device)
    wl = None
    n_w = 0
    if widths is not None:
        wl = np.ascontiguousarray(widths, dtype=np.int32)
        n_w = int(wl.size)
    n_out = ctypes.c_int()
    thr = ctypes.c_float()
    kprov = ctypes.c_int64()
    ctx._sync_stream()
    rl = np.ascontiguousarray(rho if rho is not None else (), dtype=np.float64)
    st = lib().nbsi_search_corr(ctx._h, _ptr(snr), n_chan, n_pix,
                                wl.ctypes.data_as(ctypes.c_void_p) if wl is not None else None, n_w,
                                rl.ctypes.data_as(ctypes.c_void_p) if rl.size else None, int(rl.size), float(fdr_q),
                                _ptr(S), _ptr(W), _ptr(out), max_out, ctypes.byref(n_out), ctypes.byref(thr),
                                ctypes.byref(kprov))
    if st not in (0, NBSI_ETRUNC):
        _check(st, ctx)
    n = min(n_out.value, max_out)
    rec = out[:n].cpu().numpy().copy().view(CAND_DTYPE).reshape(-1)
    return rec, float(thr.value), int(kprov.value), S, W


def nbsi_dedoppler(snr_sub, max_drift: int, best=None, drift=None, ctx: Context | None = None):
    """snr_sub [n_sub][n_chan][n_pix][n_pix] float32 -> (best de-Dopplered SNR [n_chan][n_pix][n_pix]
    float32, its total drift in channels int8)."""
    torch = _torch()
    ctx = ctx or nbsi_create(snr_sub.device.index or 0)
    _need(snr_sub, torch.float32, "snr_sub", ctx.device)
    n_sub, n_chan, n_pix, _ = snr_sub.shape
    if best is None:
        best = torch.empty((n_chan, n_pix, n_pix), dtype=torch.float32, device=ctx.device)
    if drift is None:
        drift = torch.empty((n_chan, n_pix, n_pix), dtype=torch.int8, device=ctx.device)
    _need(best, torch.float32, "best", ctx.device)
    _need(drift, torch.int8, "drift", ctx.device)
    if tuple(best.shape) != (n_chan, n_pix, n_pix) or tuple(drift.shape) != (n_chan, n_pix, n_pix):
        raise ValueError("best / drift shape does not match snr_sub")
    ctx._sync_stream()
    _check(lib().nbsi_dedoppler(ctx._h, _ptr(snr_sub), n_sub, n_chan, n_pix, int(max_drift), _ptr(best),
                                _ptr(drift)), ctx)
    return best, drift


def nbsi_beam(plan: "ImagePlan", beam=None):
    """Synthesized beam per channel of a plan: float64 device tensor [n_chan][3] (FWHM major,
    minor in pixels, position angle in radians)."""
    torch = _torch()
    ctx = plan.ctx
    if beam is None:
        beam = torch.empty((plan.n_chan, 3), dtype=torch.float64, device=ctx.device)
    _need(beam, torch.float64, "beam", ctx.device)
    if tuple(beam.shape) != (plan.n_chan, 3):
        raise ValueError("beam must be [n_chan][3]")
    ctx._sync_stream()
    _check(lib().nbsi_beam(ctx._h, plan._h, _ptr(beam)), ctx)
    return beam


def nbsi_stage2(img, cands, beam, half: int = 4, ext_factor: float = 1.5, noise_k: float = 1.5, out=None,
                ctx: Context | None = None):
    """Stage II fits and flags: img [n_chan][n_pix][n_pix] float32, cands int32 device tensor
    [n][5] (nbsi_cand records), beam float64 [n_chan][3] -> uint8 device tensor [n][160] of
    nbsi_fit records (view on the host with FIT_DTYPE)."""
    torch = _torch()
    ctx = ctx or nbsi_create(img.device.index or 0)
    _need(img, torch.float32, "img", ctx.device)
    _need(cands, torch.int32, "cands", ctx.device)
    _need(beam, torch.float64, "beam", ctx.device)
    n_chan, n_pix, _ = img.shape
    if cands.dim() != 2 or cands.shape[1] != 5:
        raise ValueError("cands must be [n][5] int32 (nbsi_cand records)")
    if tuple(beam.shape) != (n_chan, 3):
        raise ValueError("beam must be [n_chan][3]")
    n = cands.shape[0]
    if out is None:
        out = torch.empty((max(1, n), FIT_DTYPE.itemsize), dtype=torch.uint8, device=ctx.device)
    _need(out, torch.uint8, "out", ctx.device)
    if out.numel() < n * FIT_DTYPE.itemsize:
        raise ValueError("out too small")
    ctx._sync_stream()
    _check(lib().nbsi_stage2(ctx._h, _ptr(img), n_chan, n_pix, _ptr(cands), n, _ptr(beam), int(half),
                             float(ext_factor), float(noise_k), _ptr(out)), ctx)
    return out


def fits_host(out, n: int) -> np.ndarray:
    """nbsi_fit records of a device buffer as a numpy structured array."""
    return out.reshape(-1)[:n * FIT_DTYPE.itemsize].cpu().numpy().copy().view(FIT_DTYPE).reshape(-1)


def _detect_call(fn, img, mode, thresh, want_snr, max_out, ctx, snr=None, out=None):
    torch = _torch()
    ctx = ctx or nbsi_create(img.device.index or 0)
    _need(img, torch.float32, "img", ctx.device)
    n_chan, n_pix, _ = img.shape
    if want_snr and snr is None:
        snr = torch.empty_like(img)
    if out is None:
        out = torch.empty((max(1, max_out), 5), dtype=torch.int32, device=ctx.device)
    n_out = ctypes.c_int(0)
    ctx._sync_stream()
    st = fn(ctx._h, _ptr(img), n_chan, n_pix, int(mode), float(thresh), _ptr(snr), _ptr(out), int(max_out),
            ctypes.byref(n_out))
    if st not in (NBSI_OK, NBSI_ETRUNC):
        _check(st, ctx)
    n = min(n_out.value, max_out)
    rec = out[:n].cpu().numpy().view(CAND_DTYPE).reshape(-1)
    return rec, snr, n_out.value


def nbsi_detect(img, mode: int = NBSI_DETECT_PER_PIXEL, thresh: float = 5.0, want_snr: bool = False,
                max_out: int = 1 << 20, ctx: Context | None = None):
    """img [n_chan][n_pix][n_pix] float32 -> (candidates as a numpy structured array sorted by
    (y, x, c), snr cube or None).  Blocks until the candidate count is known."""
    return _detect_call(lib().nbsi_detect, img, mode, thresh, want_snr, max_out, ctx)


def nbsi_detect_noalloc(img, mode: int = NBSI_DETECT_PER_PIXEL, thresh: float = 5.0, snr=None, out=None,
                        max_out: int = 1 << 16, ctx: Context | None = None):
    """nbsi_detect with the library's fixed per-GPU workspace: the C call allocates nothing.
    snr (optional [n_chan][n_pix][n_pix] float32) and out ([max_out][5] int32) are the caller's
    tensors (out is allocated here when not given).  Returns (candidates, snr, true count)."""
    return _detect_call(lib().nbsi_detect_noalloc, img, mode, thresh, False, max_out, ctx, snr=snr, out=out)


class NbsiSubband(ctypes.Structure):
    """nbsi_subband: one sub-band of a batch (device pointers, host frequency list)."""
    _fields_ = [("volt", ctypes.c_void_p), ("gain", ctypes.c_void_p), ("n_fft", ctypes.c_int),
                ("n_spec", ctypes.c_int), ("chan0", ctypes.c_int), ("n_chan", ctypes.c_int),
                ("freq_hz_host", ctypes.c_void_p), ("n_pix", ctypes.c_int), ("spec_q", ctypes.c_void_p),
                ("vis", ctypes.c_void_p), ("img", ctypes.c_void_p)]


class Batch:
    """nbsi_batch_plan / run / describe / destroy.

    subbands: list of dicts with volt [n_in][n_spec*n_fft][2] int8 and gain [n_in] float32 device
    tensors, n_fft, n_spec, chan0, n_chan, freq_hz (host array of n_chan) and n_pix.  The output
    tensors spec_q, vis and img are allocated here (or taken from the dict) and kept on the
    object; every run() rewrites them."""

    def __init__(self, ant_xyz, subbands, precision: int = NBSI_PREC_FP32, graph: bool = True,
                 autotune: bool = False, tune_cache: str | None = None, ctx: Context | None = None,
                 grid_tall: bool = False, overlap: bool = False):
        torch = _torch()
        self.ctx = ctx or nbsi_create(0)
        dev = self.ctx.device
        self.ant_xyz = np.ascontiguousarray(ant_xyz, dtype=np.float64)
        n_ant = self.ant_xyz.shape[0]
        n_in = 2 * n_ant
        self.subbands = []
        arr = (NbsiSubband * len(subbands))()
        for i, sbd in enumerate(subbands):
            d = dict(sbd)
            _need(d["volt"], torch.int8, "volt", dev)
            _need(d["gain"], torch.float32, "gain", dev)
            if d["volt"].shape[0] != n_in or d["gain"].numel() != n_in:
                raise ValueError(f"sub-band {i}: volt/gain do not have 2 n_ant = {n_in} inputs")
            C, T, n_pix = int(d["n_chan"]), int(d["n_spec"]), int(d["n_pix"])
            d["freq_hz"] = np.ascontiguousarray(d["freq_hz"], dtype=np.float64)
            if d["freq_hz"].size != C:
                raise ValueError(f"sub-band {i}: freq_hz needs n_chan entries")
            if d.get("spec_q") is None:
                d["spec_q"] = torch.empty((C, n_in, 2, T), dtype=torch.int8, device=dev)
            if d.get("vis") is None:
                d["vis"] = torch.empty((C, n_in * (n_in + 1) // 2, 2), dtype=torch.int32, device=dev)
            if d.get("img") is None:
                d["img"] = torch.empty((C, n_pix, n_pix), dtype=torch.float32, device=dev)
            _need(d["spec_q"], torch.int8, "spec_q", dev)
            _need(d["vis"], torch.int32, "vis", dev)
            _need(d["img"], torch.float32, "img", dev)
            arr[i] = NbsiSubband(d["volt"].data_ptr(), d["gain"].data_ptr(), int(d["n_fft"]), T,
                                 int(d["chan0"]), C, d["freq_hz"].ctypes.data, n_pix,
                                 d["spec_q"].data_ptr(), d["vis"].data_ptr(), d["img"].data_ptr())
            self.subbands.append(d)
        flags = ((NBSI_BATCH_GRAPH if graph else 0) | (NBSI_BATCH_AUTOTUNE if autotune else 0)
                 | (NBSI_BATCH_GRID_TALL if grid_tall else 0) | (NBSI_BATCH_OVERLAP if overlap else 0))
        h = ctypes.c_void_p()
        self.ctx._sync_stream()
        _check(lib().nbsi_batch_plan(self.ctx._h, self.ant_xyz.ctypes.data_as(ctypes.c_void_p), n_ant, arr,
                                     len(subbands), int(precision), flags,
                                     tune_cache.encode() if tune_cache else None, ctypes.byref(h)), self.ctx)
        self._h = h

    def run(self):
        self.ctx._sync_stream()
        _check(lib().nbsi_batch_run(self._h), self.ctx)

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().nbsi_batch_describe(self._h, buf, len(buf)))
        return buf.value.decode()

    def close(self):
        if getattr(self, "_h", None):
            lib().nbsi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nbsi_batch_plan(ant_xyz, subbands, precision=NBSI_PREC_FP32, graph=True, autotune=False, tune_cache=None,
                    ctx=None) -> Batch:
    return Batch(ant_xyz, subbands, precision, graph, autotune, tune_cache, ctx)


def nbsi_batch_run(batch: Batch) -> None:
    batch.run()


def nbsi_batch_describe(batch: Batch) -> str:
    return batch.describe()


def nbsi_batch_destroy(batch: Batch) -> None:
    batch.close()


def nbsi_stamps(cube, cands, stamps=None, ctx: Context | None = None):
    """cube [n_chan][n_pix][n_pix] float32, cands: int32 device tensor [n][5] (nbsi_cand records,
    as nbsi_detect returns them) -> stamps [n][33][9][9] float16."""
    torch = _torch()
    ctx = ctx or nbsi_create(cube.device.index or 0)
    _need(cube, torch.float32, "cube", ctx.device)
    _need(cands, torch.int32, "cands", ctx.device)
    if cands.dim() != 2 or cands.shape[1] != 5:
        raise ValueError("cands must be [n][5] int32 records (x, y, c, width, snr bits)")
    n = cands.shape[0]
    if stamps is None:
        stamps = torch.empty((n, NBSI_STAMP_CHANNELS, NBSI_STAMP_PIXELS, NBSI_STAMP_PIXELS), dtype=torch.float16,
                             device=ctx.device)
    _need(stamps, torch.float16, "stamps", ctx.device)
    ctx._sync_stream()
    _check(lib().nbsi_stamps(ctx._h, _ptr(cube), cube.shape[0], cube.shape[1], _ptr(cands), n, _ptr(stamps)), ctx)
    return stamps


class Net:
    """nbsi_net_*: the candidate classifier with its FP32 master parameters and Adam state."""

    def __init__(self, params, max_batch: int = 1024, ctx: Context | None = None):
        self.ctx = ctx or nbsi_create(0)
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != NBSI_NET_NPARAM:
            raise ValueError(f"params must have {NBSI_NET_NPARAM} entries")
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        self.ctx._sync_stream()
        _check(lib().nbsi_net_create(self.ctx._h, p.ctypes.data_as(ctypes.c_void_p), self.max_batch,
                                     ctypes.byref(h)), self.ctx)
        self._h = h

    def _stamps(self, stamps, index, n):
        torch = _torch()
        _need(stamps, torch.float16, "stamps", self.ctx.device)
        if index is not None:
            _need(index, torch.int32, "index", self.ctx.device)
            n = index.numel() if n is None else n
        else:
            n = stamps.shape[0] if n is None else n
        return n

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.ctx._sync_stream()
        _check(lib().nbsi_net_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)), self.ctx)

    def get_params(self) -> np.ndarray:
        out = np.empty(NBSI_NET_NPARAM, dtype=np.float32)
        self.ctx._sync_stream()
        _check(lib().nbsi_net_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)), self.ctx)
        return out

    def forward(self, stamps, index=None, n=None, logits=None):
        torch = _torch()
        n = self._stamps(stamps, index, n)
        if logits is None:
            logits = torch.empty(n, dtype=torch.float32, device=self.ctx.device)
        self.ctx._sync_stream()
        _check(lib().nbsi_net_forward(self._h, _ptr(stamps), stamps.shape[0], _ptr(index), n, _ptr(logits)),
               self.ctx)
        return logits

    def grad(self, stamps, labels, index=None, n=None, grad=None):
        """(loss tensor [1], gradient tensor [NBSI_NET_NPARAM]) of a batch."""
        torch = _torch()
        n = self._stamps(stamps, index, n)
        _need(labels, torch.float32, "labels", self.ctx.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.ctx.device)
        if grad is None:
            grad = torch.empty(NBSI_NET_NPARAM, dtype=torch.float32, device=self.ctx.device)
        self.ctx._sync_stream()
        _check(lib().nbsi_net_grad(self._h, _ptr(stamps), stamps.shape[0], _ptr(index), _ptr(labels), n, _ptr(loss),
                                   _ptr(grad)), self.ctx)
        return loss, grad

    def adam(self, grad=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.ctx._sync_stream()
        _check(lib().nbsi_net_adam(self._h, _ptr(grad), float(lr), float(beta1), float(beta2), float(eps)),
               self.ctx)

    def train_step(self, stamps, labels, index=None, n=None, lr=1e-3, loss=None):
        torch = _torch()
        n = self._stamps(stamps, index, n)
        _need(labels, torch.float32, "labels", self.ctx.device)
        self.ctx._sync_stream()
        _check(lib().nbsi_net_train_step(self._h, _ptr(stamps), stamps.shape[0], _ptr(index), _ptr(labels), n,
                                         float(lr), _ptr(loss)), self.ctx)
        return loss

    def close(self):
        if getattr(self, "_h", None):
            lib().nbsi_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nbsi_net_create(params, max_batch=1024, ctx=None) -> Net:
    return Net(params, max_batch, ctx)
