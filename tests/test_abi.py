"""The C-ABI library loads, exports every symbol include/nbsi.h declares, and validates
arguments on the host (no GPU needed for any of this)."""
import ctypes
import os
import re

import pytest

import paper_2606_04304_amd as nb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "nbsi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbsi_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = nb.lib()
    names = _header_symbols()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(nb.EXPORTS)


def test_version_and_strerror():
    L = nb.lib()
    assert L.nbsi_version() == 1
    assert L.nbsi_strerror(nb.NBSI_ETRUNC) == b"output truncated"
    assert L.nbsi_strerror(12345) == b"unknown status"


@pytest.mark.parametrize("args,code", [
    ((32, 4096, 16, 2016, 64), nb.NBSI_OK),
    ((704, 65536, 32, 30720, 4096), nb.NBSI_OK),
    ((704, 1 << 18, 8, 122880, 16384), nb.NBSI_OK),
    ((32, 4095, 16, 0, 64), nb.NBSI_EINVAL),          # not a power of two
    ((32, 128, 16, 0, 64), nb.NBSI_EINVAL),           # too short
    ((32, 1 << 19, 16, 0, 64), nb.NBSI_EINVAL),       # too long
    ((32, 4096, 65536, 0, 64), nb.NBSI_EOVERFLOW),    # int32 bound of the correlator
    ((32, 4096, 0, 0, 64), nb.NBSI_EINVAL),
    ((32, 4096, 16, 4090, 64), nb.NBSI_EINVAL),       # window past the last channel
    ((32, 4096, 16, -1, 64), nb.NBSI_EINVAL),
    ((32, 1 << 16, 16, 0, 32768), nb.NBSI_EINVAL),    # band wider than one sub-transform
    ((0, 4096, 16, 0, 64), nb.NBSI_EINVAL),
])
def test_check_channelize(args, code):
    assert nb.lib().nbsi_check_channelize(*args) == code


def test_check_correlate():
    L = nb.lib()
    assert L.nbsi_check_correlate(4096, 704, 32) == nb.NBSI_OK
    assert L.nbsi_check_correlate(1, 1, 65535) == nb.NBSI_OK
    assert L.nbsi_check_correlate(1, 1, 65536) == nb.NBSI_EOVERFLOW
    assert L.nbsi_check_correlate(0, 4, 4) == nb.NBSI_EINVAL
    assert L.nbsi_check_correlate(4, 0, 4) == nb.NBSI_EINVAL


def test_check_image():
    L = nb.lib()
    inf = float("inf")
    assert L.nbsi_check_image(64, 16, 64, nb.NBSI_IMAGE_DFT, nb.NBSI_PREC_FP32, 0.0, inf) == 0
    assert L.nbsi_check_image(4096, 352, 256, nb.NBSI_IMAGE_GRID, nb.NBSI_PREC_BF16, 0.0, inf) == 0
    assert L.nbsi_check_image(4, 16, 96, nb.NBSI_IMAGE_GRID, 0, 0.0, inf) == nb.NBSI_EINVAL  # not 2^k
    assert L.nbsi_check_image(4, 16, 32, nb.NBSI_IMAGE_GRID, 0, 0.0, inf) == nb.NBSI_EINVAL  # < 64
    assert L.nbsi_check_image(4, 16, 36, nb.NBSI_IMAGE_DFT, 0, 0.0, inf) == nb.NBSI_EINVAL   # not 8k
    assert L.nbsi_check_image(4, 1, 64, 0, 0, 0.0, inf) == nb.NBSI_EINVAL
    assert L.nbsi_check_image(4, 16, 64, 7, 0, 0.0, inf) == nb.NBSI_EINVAL
    assert L.nbsi_check_image(4, 16, 64, 0, 9, 0.0, inf) == nb.NBSI_EINVAL
    assert L.nbsi_check_image(4, 16, 64, 0, 0, 5.0, 1.0) == nb.NBSI_EINVAL
    assert L.nbsi_check_image(4, 16, 64, 0, 0, float("nan"), inf) == nb.NBSI_EINVAL


def test_check_detect():
    L = nb.lib()
    assert L.nbsi_check_detect(4096, 256, nb.NBSI_DETECT_PER_PIXEL, 100) == 0
    assert L.nbsi_check_detect(2, 256, 0, 100) == nb.NBSI_EINVAL
    assert L.nbsi_check_detect(64, 250, 0, 100) == nb.NBSI_EINVAL
    assert L.nbsi_check_detect(64, 256, 5, 100) == nb.NBSI_EINVAL
    assert L.nbsi_check_detect(64, 256, 0, -1) == nb.NBSI_EINVAL


def test_null_context_is_rejected():
    L = nb.lib()
    assert L.nbsi_channelize(None, None, 1, 4096, 1, 0, 1, None, None, None) == nb.NBSI_EINVAL
    assert L.nbsi_correlate(None, None, 1, 1, 1, None) == nb.NBSI_EINVAL
    assert L.nbsi_correlate_f32(None, None, 1, 1, 1, None) == nb.NBSI_EINVAL
    assert L.nbsi_image(None, None, None, 0, 0, None) == nb.NBSI_EINVAL
    n = ctypes.c_int(0)
    assert L.nbsi_detect(None, None, 8, 8, 0, 5.0, None, None, 0, ctypes.byref(n)) == nb.NBSI_EINVAL
    assert L.nbsi_destroy(None) == nb.NBSI_EINVAL
    assert L.nbsi_synchronize(None) == nb.NBSI_EINVAL
    assert L.nbsi_correlate_stokes(None, None, 1, 2, 1, None, None, None) == nb.NBSI_EINVAL
    assert L.nbsi_image_stokes(None, None, None, 0, None) == nb.NBSI_EINVAL
    assert L.nbsi_correlate_image(None, None, 1, 2, 1, None, 0, 0, None, None, None) == nb.NBSI_EINVAL
    assert L.nbsi_status(None, None) == nb.NBSI_EINVAL
    assert L.nbsi_detect_noalloc(None, None, 8, 8, 0, 5.0, None, None, 0, ctypes.byref(n)) == nb.NBSI_EINVAL


def test_binding_constants_match_the_header():
    """Every integer #define of include/nbsi.h that the binding also names has the same value."""
    text = open(os.path.join(ROOT, "include", "nbsi.h")).read()
    defs = {}
    for name, val in re.findall(r"^#define\s+(NBSI_\w+)\s+(\(1 << \d+\)|\(-?\d+\)|-?\d+)", text, re.M):
        defs[name] = eval(val, {"__builtins__": {}})
    shared = [n for n in defs if hasattr(nb, n)]
    assert len(shared) >= 20, shared
    for n in shared:
        assert getattr(nb, n) == defs[n], (n, getattr(nb, n), defs[n])
    assert defs["NBSI_BATCH_OVERLAP"] == 8 and defs["NBSI_DEFAULT_STAGES"] >= 1


def test_create_without_gfx950_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = nb.lib().nbsi_create(ctypes.byref(h), 0, None)
    assert rc in (nb.NBSI_EHIP, nb.NBSI_EUNSUPPORTED) and not h.value
