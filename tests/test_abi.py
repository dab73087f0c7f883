"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/prony.h, and validates arguments before
launching anything (through a validation-only handle, device -1)."""
import ctypes
import os
import re

import pytest

from paper_2012_11430_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "prony.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(prony_[A-Za-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = _lib.load()
    declared = _declared_symbols()
    assert "prony_build_S" in declared and "prony_coeffs" in declared
    for name in declared:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"
    assert set(_lib.SIGNATURES) == set(declared)


@pytest.fixture()
def vhandle():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.prony_create(ctypes.byref(h), -1) == _lib.PRONY_OK
    yield lib, h
    assert lib.prony_destroy(h) == _lib.PRONY_OK


P = ctypes.c_void_p(0x1000)   # never dereferenced: validation-only handles launch nothing
NULL = ctypes.c_void_p(0)


def _err(lib, h):
    return lib.prony_last_error(h).decode()


def test_validation_only_handle_reaches_enodev_for_valid_arguments(vhandle):
    lib, h = vhandle
    assert lib.prony_samples(h, 2, 15, 5, P, P, NULL, P) == _lib.PRONY_ENODEV
    assert lib.prony_build_T(h, 2, 15, 1, P, P, 256) == _lib.PRONY_ENODEV
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 5, 1, P, P, 5, 1, _lib.PRONY_FP32, 0, P) == _lib.PRONY_ENODEV
    assert lib.prony_coeffs(h, 2, 15, 5, P, P, P, P, NULL) == _lib.PRONY_ENODEV
    assert lib.prony_synchronize(h) == _lib.PRONY_ENODEV


@pytest.mark.parametrize("d,n", [(0, 5), (4, 5), (2, 0), (-1, 3)])
def test_bad_dimensions_rejected(vhandle, d, n):
    lib, h = vhandle
    assert lib.prony_samples(h, d, n, 2, P, P, NULL, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S(h, d, n, 2, P, P, 2, 1, P, P, 2, 1, 0, 0, P) == _lib.PRONY_EINVAL


def test_build_S_argument_checks(vhandle):
    lib, h = vhandle
    # m > N
    assert lib.prony_build_S(h, 1, 3, 5, P, P, 5, 1, P, P, 5, 1, 0, 0, P) == _lib.PRONY_EINVAL
    # m > 32 is a valid request the MFMA kernels do not cover
    assert lib.prony_build_S(h, 2, 15, 33, P, P, 33, 1, P, P, 33, 1, 0, 0, P) == _lib.PRONY_ENOTSUP
    assert "m > 32" in _err(lib, h)
    # null pointers, strides, precision, flags
    assert lib.prony_build_S(h, 2, 15, 5, NULL, P, 5, 1, P, P, 5, 1, 0, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 0, 1, P, P, 5, 1, 0, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 5, 1, P, P, 5, -1, 0, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 5, 1, P, P, 5, 1, 7, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 5, 1, P, P, 5, 1, 0, 2, P) == _lib.PRONY_EINVAL
    # S_0 flag accepted
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 5, 1, P, P, 5, 1, 0, _lib.PRONY_WITH_S0, P) == _lib.PRONY_ENODEV
    # the split-bfloat16 precision is a valid request for the S-build only
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 5, 1, P, P, 5, 1, _lib.PRONY_BF16X3, 0, P) == _lib.PRONY_ENODEV
    assert lib.prony_build_S(h, 2, 15, 5, P, P, 5, 1, P, P, 5, 1, 3, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_adjoint(h, 2, 15, 5, P, 5, 1, P, P, 5, 1, P, _lib.PRONY_BF16X3, P) == _lib.PRONY_EINVAL
    assert lib.prony_toeplitz_mm(h, 2, 15, 0, P, 4, P, 4, _lib.PRONY_BF16X3, P, 4) == _lib.PRONY_EINVAL
    arr = (_lib.InstanceDesc * 1)(_desc(2, 15, 5))
    out = ctypes.c_void_p()
    assert lib.prony_batch_create(h, 1, arr, _lib.PRONY_BF16X3, ctypes.byref(out)) == _lib.PRONY_EINVAL
    # tuning entries: single-instance entries for every precision, batch entries for FP32/FP64
    assert lib.prony_tune_set(h, 2, 15, 5, _lib.PRONY_BF16X3, 0, 512) == _lib.PRONY_OK
    assert lib.prony_tune_set(h, 2, 15, 5, _lib.PRONY_BF16X3, _lib.PRONY_TUNE_BATCHED, 2) == _lib.PRONY_EINVAL
    assert lib.prony_tune_set(h, 2, 15, 5, _lib.PRONY_BF16X3, 0, 0) == _lib.PRONY_OK


def test_tune_entries_and_cache_loader(vhandle, tmp_path):
    lib, h = vhandle
    got = ctypes.c_int(-1)
    assert lib.prony_tune_set(h, 3, 19, 30, _lib.PRONY_FP32, 0, 768) == _lib.PRONY_OK
    assert lib.prony_tune_get(h, 3, 19, 30, _lib.PRONY_FP32, 0, ctypes.byref(got)) == _lib.PRONY_OK
    assert got.value == 768
    assert lib.prony_tune_get(h, 3, 19, 30, _lib.PRONY_FP32, _lib.PRONY_TUNE_BATCHED, ctypes.byref(got)) == 0
    assert got.value == 0
    assert lib.prony_tune_get(h, 3, 19, 30, _lib.PRONY_FP32, 4, ctypes.byref(got)) == _lib.PRONY_EINVAL
    assert lib.prony_tune_set(h, 3, 19, 30, _lib.PRONY_FP32, 0, 0) == _lib.PRONY_OK
    assert lib.prony_autotune(h, None) == _lib.PRONY_EINVAL
    assert lib.prony_autotune(h, str(tmp_path / "missing.json").encode()) == _lib.PRONY_EINVAL
    cache = tmp_path / "tune.json"
    cache.write_text('{"devices": {}, "version": 1}')
    assert lib.prony_autotune(h, str(cache).encode()) == _lib.PRONY_ENODEV   # needs the device's name


def test_build_T_and_coeffs_argument_checks(vhandle):
    lib, h = vhandle
    assert lib.prony_build_T(h, 2, 15, 3, P, P, 256) == _lib.PRONY_EINVAL      # which > d
    assert lib.prony_build_T(h, 2, 15, 0, P, P, 255) == _lib.PRONY_EINVAL      # ld < N
    assert lib.prony_build_T(h, 2, 15, 0, NULL, P, 256) == _lib.PRONY_EINVAL
    assert lib.prony_coeffs(h, 2, 15, 65, P, P, P, P, NULL) == _lib.PRONY_ENOTSUP
    assert lib.prony_coeffs(h, 1, 3, 5, P, P, P, P, NULL) == _lib.PRONY_EINVAL  # m > N
    assert lib.prony_coeffs(h, 2, 15, 5, P, NULL, P, P, NULL) == _lib.PRONY_EINVAL
    assert lib.prony_samples(h, 2, 15, 0, P, P, NULL, P) == _lib.PRONY_EINVAL
    assert lib.prony_reserve(h, 2, 15, 65) == _lib.PRONY_EINVAL


def test_huge_grid_is_not_supported(vhandle):
    lib, h = vhandle
    assert lib.prony_samples(h, 3, 2000, 2, P, P, NULL, P) == _lib.PRONY_ENOTSUP


def test_null_handle_and_error_text():
    lib = _lib.load()
    assert lib.prony_build_S(NULL, 2, 15, 5, P, P, 5, 1, P, P, 5, 1, 0, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_last_error(NULL) == b"invalid handle"
    assert lib.prony_create(None, 0) == _lib.PRONY_EINVAL


def _desc(d, n, m, ptr=P):
    return _lib.InstanceDesc(d, n, m, ptr.value, ptr.value, ptr.value, ptr.value, ptr.value)


def test_batch_validation(vhandle):
    lib, h = vhandle
    arr = (_lib.InstanceDesc * 3)(_desc(2, 15, 5), _desc(1, 100, 32), _desc(3, 3, 8))
    out = ctypes.c_void_p()
    assert lib.prony_batch_create(h, 3, arr, _lib.PRONY_FP32, ctypes.byref(out)) == _lib.PRONY_ENODEV
    bad = (_lib.InstanceDesc * 3)(_desc(2, 15, 5), _desc(2, 15, 5), _desc(1, 3, 5))
    assert lib.prony_batch_create(h, 3, bad, _lib.PRONY_FP32, ctypes.byref(out)) == _lib.PRONY_EINVAL
    assert "instance 2" in _err(lib, h)
    big = (_lib.InstanceDesc * 1)(_desc(2, 15, 40))
    assert lib.prony_batch_create(h, 1, big, _lib.PRONY_FP64, ctypes.byref(out)) == _lib.PRONY_ENOTSUP
    nul = (_lib.InstanceDesc * 1)(_desc(2, 15, 5, NULL))
    assert lib.prony_batch_create(h, 1, nul, _lib.PRONY_FP64, ctypes.byref(out)) == _lib.PRONY_EINVAL
    assert lib.prony_batch_create(h, 0, arr, _lib.PRONY_FP64, ctypes.byref(out)) == _lib.PRONY_EINVAL
    assert lib.prony_batch_create(h, 3, arr, 9, ctypes.byref(out)) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_batched(h, NULL) == _lib.PRONY_EINVAL
    assert lib.prony_batch_set_schedule(NULL, _lib.PRONY_SCHEDULE_QUEUE) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_adjoint_batched(h, NULL, P, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_adjoint_batched(NULL, NULL, P, P) == _lib.PRONY_EINVAL
    assert lib.prony_graph_launch(h, NULL) == _lib.PRONY_EINVAL
    assert lib.prony_graph_destroy(NULL) == _lib.PRONY_EINVAL


def test_adjoint_validation(vhandle):
    lib, h = vhandle
    assert lib.prony_build_S_adjoint(h, 2, 47, 16, P, 16, 1, P, P, 16, 1, P, _lib.PRONY_FP32, P) == _lib.PRONY_ENODEV
    assert lib.prony_build_S_adjoint(h, 2, 47, 33, P, 33, 1, P, P, 33, 1, P, 0, P) == _lib.PRONY_ENOTSUP
    assert lib.prony_build_S_adjoint(h, 1, 3, 5, P, 5, 1, P, P, 5, 1, P, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_adjoint(h, 2, 47, 16, P, 16, 1, P, P, 16, 1, NULL, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_adjoint(h, 2, 47, 16, P, 0, 1, P, P, 16, 1, P, 0, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_adjoint(h, 2, 47, 16, P, 16, 1, P, P, 16, 1, P, 5, P) == _lib.PRONY_EINVAL


def test_toeplitz_mm_validation(vhandle):
    lib, h = vhandle
    assert lib.prony_toeplitz_mm(h, 2, 15, 0, P, 10, P, 10, _lib.PRONY_FP64, P, 10) == _lib.PRONY_ENODEV
    assert lib.prony_toeplitz_mm(h, 2, 15, 2, P, 10, P, 10, _lib.PRONY_FP64, P, 10) == _lib.PRONY_EINVAL
    assert lib.prony_toeplitz_mm(h, 2, 15, 0, P, 65, P, 65, _lib.PRONY_FP64, P, 65) == _lib.PRONY_EINVAL
    assert lib.prony_toeplitz_mm(h, 2, 15, 0, P, 10, P, 9, _lib.PRONY_FP64, P, 10) == _lib.PRONY_EINVAL
    assert lib.prony_toeplitz_mm(h, 2, 15, 0, NULL, 10, P, 10, _lib.PRONY_FP64, P, 10) == _lib.PRONY_EINVAL
    assert lib.prony_toeplitz_mm(h, 2, 15, 1, P, 10, P, 10, 7, P, 10) == _lib.PRONY_EINVAL
    assert lib.prony_toeplitz_mm(h, 4, 15, 0, P, 10, P, 10, _lib.PRONY_FP64, P, 10) == _lib.PRONY_EINVAL
