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


def _plan(lib, h, d, n, m, prec, flags=0):
    frag, wgs, chunk = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ws = ctypes.c_size_t()
    st = lib.prony_build_S_plan(h, d, n, m, prec, flags, ctypes.byref(frag), ctypes.byref(wgs), ctypes.byref(chunk),
                                ctypes.byref(ws))
    return st, frag.value, wgs.value, chunk.value, ws.value


def test_plan_query_on_a_validation_only_handle(vhandle):
    # the planner runs on the host: validation-only handles plan for 256 CUs, 160 KiB LDS
    lib, h = vhandle
    st, frag, wgs, chunk, ws = _plan(lib, h, 2, 63, 20, _lib.PRONY_FP32)
    assert st == _lib.PRONY_OK
    assert frag == 2 and chunk % 16 == 0 and ws > 0
    rows = 64 * frag
    NR = 65 ** 2                            # row-extended rows (n+2)^d
    row_tiles = -(-NR // rows)
    assert wgs % row_tiles == 0 and (wgs // row_tiles) * chunk >= 64 ** 2
    # more workgroups for a larger target; the split-bfloat16 plan has 32-wide chunks
    assert lib.prony_tune_set(h, 2, 63, 20, _lib.PRONY_FP32, 0, 8 * 256) == _lib.PRONY_OK
    assert _plan(lib, h, 2, 63, 20, _lib.PRONY_FP32)[2] > wgs
    assert _plan(lib, h, 2, 63, 20, _lib.PRONY_BF16X3)[3] % 32 == 0
    # argument checks as for prony_build_S
    assert _plan(lib, h, 2, 63, 40, _lib.PRONY_FP32)[0] == _lib.PRONY_ENOTSUP
    assert _plan(lib, h, 4, 63, 20, _lib.PRONY_FP32)[0] == _lib.PRONY_EINVAL
    assert _plan(lib, h, 2, 63, 20, 7)[0] == _lib.PRONY_EINVAL
    assert _plan(lib, h, 2, 63, 20, _lib.PRONY_FP32, 8)[0] == _lib.PRONY_EINVAL
    assert lib.prony_build_S_plan(h, 2, 63, 20, _lib.PRONY_FP32, 0, None, None, None, None) == _lib.PRONY_OK


def test_tile_entries_exact_and_bucket(vhandle):
    lib, h = vhandle
    frag, tgt = ctypes.c_int(-1), ctypes.c_int(-1)
    # 4 fragments per wave where the instantiation supports it (FP32, 3 column blocks)
    assert lib.prony_tune_set_tile(h, 2, 63, 20, _lib.PRONY_FP32, 0, 4, 512) == _lib.PRONY_OK
    assert _plan(lib, h, 2, 63, 20, _lib.PRONY_FP32)[1] == 4
    assert lib.prony_tune_get_tile(h, 2, 63, 20, _lib.PRONY_FP32, 0, ctypes.byref(frag), ctypes.byref(tgt)) == 0
    assert (frag.value, tgt.value) == (4, 512)
    # FP64 supports 4 fragments only up to 2 accumulator blocks per fragment: the
    # pair form with one column block (m <= 8); m = 9..16 takes the three-product
    # form (3 blocks) and m = 20 the pair form with 3 blocks, which fall back to 2
    assert lib.prony_tune_set_tile(h, 2, 63, 20, _lib.PRONY_FP64, 0, 4, 0) == _lib.PRONY_OK
    assert _plan(lib, h, 2, 63, 20, _lib.PRONY_FP64)[1] == 2
    assert lib.prony_tune_set_tile(h, 2, 63, 16, _lib.PRONY_FP64, 0, 4, 0) == _lib.PRONY_OK
    assert _plan(lib, h, 2, 63, 16, _lib.PRONY_FP64)[1] == 2
    assert lib.prony_tune_set_tile(h, 2, 63, 8, _lib.PRONY_FP64, 0, 4, 0) == _lib.PRONY_OK
    assert _plan(lib, h, 2, 63, 8, _lib.PRONY_FP64)[1] == 4
    # a bucket entry (same d, floor(log2 N), ceil(m/8)) applies to other shapes of the bucket ...
    assert lib.prony_tune_set_tile(h, 3, 19, 30, _lib.PRONY_FP32, _lib.PRONY_TUNE_BUCKET, 1, 0) == _lib.PRONY_OK
    assert _plan(lib, h, 3, 18, 29, _lib.PRONY_FP32)[1] == 1          # N = 6859: same bucket as 8000
    assert _plan(lib, h, 3, 20, 29, _lib.PRONY_FP32)[1] == 2          # N = 9261: another bucket
    assert _plan(lib, h, 3, 18, 24, _lib.PRONY_FP32)[1] == 2          # 3 column blocks: another bucket
    # ... and the exact entry wins field by field
    assert lib.prony_tune_set_tile(h, 3, 18, 29, _lib.PRONY_FP32, 0, 2, 0) == _lib.PRONY_OK
    assert _plan(lib, h, 3, 18, 29, _lib.PRONY_FP32)[1] == 2
    assert lib.prony_tune_get_tile(h, 3, 18, 29, _lib.PRONY_FP32, _lib.PRONY_TUNE_BUCKET, ctypes.byref(frag),
                                   ctypes.byref(tgt)) == 0
    assert (frag.value, tgt.value) == (1, 0)
    # validation: fragments 3, 4 for batch members, unknown flags
    assert lib.prony_tune_set_tile(h, 2, 63, 20, _lib.PRONY_FP32, 0, 3, 0) == _lib.PRONY_EINVAL
    assert lib.prony_tune_set_tile(h, 2, 63, 20, _lib.PRONY_FP32, _lib.PRONY_TUNE_BATCHED, 4, 0) == _lib.PRONY_EINVAL
    assert lib.prony_tune_set_tile(h, 2, 63, 20, _lib.PRONY_FP32, 4, 1, 0) == _lib.PRONY_EINVAL
    # prony_tune_set keeps the entry's fragments; removing both fields removes the entry
    assert lib.prony_tune_set(h, 2, 63, 20, _lib.PRONY_FP32, 0, 1024) == _lib.PRONY_OK
    assert lib.prony_tune_get_tile(h, 2, 63, 20, _lib.PRONY_FP32, 0, ctypes.byref(frag), ctypes.byref(tgt)) == 0
    assert (frag.value, tgt.value) == (4, 1024)
    assert lib.prony_tune_set_tile(h, 2, 63, 20, _lib.PRONY_FP32, 0, 0, 0) == _lib.PRONY_OK
    assert lib.prony_tune_get_tile(h, 2, 63, 20, _lib.PRONY_FP32, 0, ctypes.byref(frag), ctypes.byref(tgt)) == 0
    assert (frag.value, tgt.value) == (0, 0)


def _cache(tmp_path, text, name="c.json"):
    p = tmp_path / name
    p.write_text(text)
    return str(p).encode()


def test_cache_loader_reads_exact_and_bucket_entries(vhandle, tmp_path):
    lib, h = vhandle
    frag, tgt = ctypes.c_int(), ctypes.c_int()
    doc = {"version": 2, "devices": {
        "other:1": {"2,63,20,fp32,single": 999},
        "gfx950:256": {"2,63,20,fp32,single": {"target": 512, "fragments": 4},
                       "1,40,5,fp64,single": 256,
                       "bucket:3,19,30,fp32,batch": {"fragments": 1, "target": 2},
                       "2,47,16,bf16x3,single": {"target": 768}}}}
    import json
    path = _cache(tmp_path, json.dumps(doc))
    assert lib.prony_autotune_device(h, path, b"gfx950:256") == _lib.PRONY_OK
    lib.prony_tune_get_tile(h, 2, 63, 20, _lib.PRONY_FP32, 0, ctypes.byref(frag), ctypes.byref(tgt))
    assert (frag.value, tgt.value) == (4, 512)
    lib.prony_tune_get_tile(h, 1, 40, 5, _lib.PRONY_FP64, 0, ctypes.byref(frag), ctypes.byref(tgt))
    assert (frag.value, tgt.value) == (0, 256)
    lib.prony_tune_get_tile(h, 3, 19, 30, _lib.PRONY_FP32, _lib.PRONY_TUNE_BATCHED | _lib.PRONY_TUNE_BUCKET,
                            ctypes.byref(frag), ctypes.byref(tgt))
    assert (frag.value, tgt.value) == (1, 2)
    # the device key is matched as a JSON key of "devices", escapes decoded; a key of
    # the same text elsewhere (here, inside another device's object) is not taken
    esc = ('{"devices": {"other:1": {"gfx950:257": {}}, "gfx\\u0039" "50:257": 3}}')
    assert lib.prony_autotune_device(h, _cache(tmp_path, esc, "e.json"), b"gfx950:257") == _lib.PRONY_EINVAL
    esc = '{"version": 1, "devices": {"other:1": {"gfx950:257": 5}, "gfx\\u003950:257": {"2,15,5,fp64,single": 77}}}'
    assert lib.prony_autotune_device(h, _cache(tmp_path, esc, "e2.json"), b"gfx950:257") == _lib.PRONY_OK
    lib.prony_tune_get_tile(h, 2, 15, 5, _lib.PRONY_FP64, 0, ctypes.byref(frag), ctypes.byref(tgt))
    assert tgt.value == 77
    # a device without entries registers nothing; a validation handle needs the explicit key
    assert lib.prony_autotune_device(h, path, b"none:0") == _lib.PRONY_OK
    assert lib.prony_autotune(h, path) == _lib.PRONY_ENODEV


@pytest.mark.parametrize("text", [
    "", "{", "[]", "{\"devices\": [1]}", "{\"version\": 3, \"devices\": {}}",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp32,single\": -1}}}",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp32,single\": 1.5}}}",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp99,single\": 1}}}",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp32,single,x\": 1}}}",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp32,single\": {\"fragments\": 3}}}}",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp32,single\": 1}}} trailing",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp32,single\": \"1\"}}}",
    "{\"devices\": {\"d:1\": {\"2,15,5,fp32,single\": 1,}}}",
    "{\"a\": \"\\ud800\"}", "{\"a\": \"\\x\"}", "{\"a\": \"unterminated}",
    "[" * 100 + "]" * 100,
])
def test_cache_loader_rejects_malformed_documents(vhandle, tmp_path, text):
    lib, h = vhandle
    assert lib.prony_autotune_device(h, _cache(tmp_path, text), b"d:1") == _lib.PRONY_EINVAL
    assert _err(lib, h).startswith("prony_")


def test_cache_loader_survives_mutated_documents(vhandle, tmp_path):
    # random truncations, byte flips and insertions of a valid cache: every load
    # returns OK or EINVAL (no crash, no hang); the sanitizer build runs this too
    import json
    import random
    lib, h = vhandle
    base = json.dumps({"version": 2, "devices": {"d:1": {"2,15,5,fp32,single": {"target": 5, "fragments": 2},
                                                         "bucket:3,4,9,fp64,batch": 3, "1,9,2,bf16x3,single": 7}}})
    rng = random.Random(1234)
    alphabet = '{}[]",:\\u0123456789.eE-+ abcdtrufnl'
    path = tmp_path / "m.json"
    for _ in range(1500):
        s = list(base)
        for _ in range(rng.randint(1, 4)):
            op = rng.randint(0, 2)
            i = rng.randrange(len(s) + 1)
            if op == 0 and s:
                del s[min(i, len(s) - 1)]
            elif op == 1:
                s.insert(i, rng.choice(alphabet))
            elif s:
                s[min(i, len(s) - 1)] = rng.choice(alphabet)
        if rng.random() < 0.2:
            s = s[:rng.randrange(len(s) + 1)]
        path.write_text("".join(s))
        assert lib.prony_autotune_device(h, str(path).encode(), b"d:1") in (_lib.PRONY_OK, _lib.PRONY_EINVAL)


def test_planner_over_a_sweep_of_shapes(vhandle):
    # every precision, flag and fragment count over ragged shapes: the host planner's
    # index arithmetic (run under the host sanitizers by the sanitizer build as well)
    lib, h = vhandle
    for d, n in [(1, 1), (1, 63), (1, 4000), (2, 1), (2, 15), (2, 63), (2, 200), (3, 1), (3, 7), (3, 19), (3, 40)]:
        N = (n + 1) ** d
        for m in sorted({1, 2, 7, 16, 17, 32} & set(range(1, min(N, 32) + 1))):
            for prec in (_lib.PRONY_FP64, _lib.PRONY_FP32, _lib.PRONY_BF16X3):
                for frag in (0, 1, 2, 4):
                    assert lib.prony_tune_set_tile(h, d, n, m, prec, 0, frag, 0) == _lib.PRONY_OK
                    for flags in (0, _lib.PRONY_WITH_S0):
                        st, f, wgs, chunk, ws = _plan(lib, h, d, n, m, prec, flags)
                        if st == _lib.PRONY_ENOTSUP:     # a window that does not fit LDS
                            assert "LDS" in _err(lib, h) or "32-bit" in _err(lib, h), (d, n, m)
                            continue
                        assert st == _lib.PRONY_OK, (d, n, m, prec, frag, flags, _err(lib, h))
                        assert f in (1, 2, 4) and wgs >= 1 and chunk >= 16 and ws > 0
                        rows = 64 * f
                        assert wgs % -(-((n + 2) ** d) // rows) == 0
                assert lib.prony_tune_set_tile(h, d, n, m, prec, 0, 0, 0) == _lib.PRONY_OK


def test_prepared_factor_validation(vhandle):
    lib, h = vhandle
    out = ctypes.c_void_p(0x1234)
    # valid arguments reach ENODEV (the plan needs no device) and leave the output cleared
    assert lib.prony_factors_create(h, 2, 15, 5, P, 5, 1, P, P, 5, 1, _lib.PRONY_FP32, 0,
                                    ctypes.byref(out)) == _lib.PRONY_ENODEV
    assert not out.value
    assert lib.prony_factors_create(h, 2, 15, 5, P, 5, 1, P, P, 5, 1, _lib.PRONY_FP32, 0, None) == _lib.PRONY_EINVAL
    assert lib.prony_factors_create(h, 2, 15, 5, NULL, 5, 1, P, P, 5, 1, _lib.PRONY_FP32, 0,
                                    ctypes.byref(out)) == _lib.PRONY_EINVAL
    assert lib.prony_factors_create(h, 2, 15, 40, P, 40, 1, P, P, 40, 1, _lib.PRONY_FP32, 0,
                                    ctypes.byref(out)) == _lib.PRONY_ENOTSUP
    assert lib.prony_factors_create(h, 2, 15, 5, P, 5, 1, P, P, 5, 1, 7, 0, ctypes.byref(out)) == _lib.PRONY_EINVAL
    assert lib.prony_factors_create(h, 2, 15, 5, P, 5, 1, P, P, 5, 1, _lib.PRONY_FP32, 8,
                                    ctypes.byref(out)) == _lib.PRONY_EINVAL
    assert "flag" in _err(lib, h)
    assert lib.prony_build_S_factors(h, NULL, P, P) == _lib.PRONY_EINVAL
    assert lib.prony_build_S_factors(NULL, P, P, P) == _lib.PRONY_EINVAL
    assert lib.prony_factors_destroy(NULL) == _lib.PRONY_EINVAL
    assert lib.prony_factors_info(NULL, None, None, None, None, None) == _lib.PRONY_EINVAL
