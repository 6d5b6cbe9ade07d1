"""The C-ABI library loads and exports what include/qt.h declares.

These run without a GPU: argument checks that fail before any HIP call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "qt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qt_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("qt_build", "qt_multiply", "qt_to_blocks", "qt_free", "qt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1501_07800_amd as qt
    lib = ctypes.CDLL(qt.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(qt.EXPORTS) == set(_declared())


def test_version_and_error_string():
    import paper_1501_07800_amd as qt
    assert "gfx950" in qt.version()
    assert isinstance(qt.lib.qt_last_error(), bytes)


def test_null_handles_rejected():
    import paper_1501_07800_amd as qt
    out = ctypes.c_void_p()
    assert qt.lib.qt_multiply(None, None, 0, None, ctypes.byref(out)) == qt.QT_ERR_ARG
    assert out.value is None
    assert qt.lib.qt_info(None, None, None, None, None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_nblocks(None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_stats(None, None, 0, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_build(0, 0, 32, 32, 0, None, None, None, 0, None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_probe_mfma(0, None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_to_blocks_noalloc(None, None, None, None, 0, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_probe_batched(0, 32, 64000, None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_tune_leaf_cached(None, None, 0, None, 1, b"c", None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_plan_tune_cached(None, None, 1, b"c", None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_tune_cache(None) == qt.QT_OK
    assert qt.lib.qt_multiply_tau(None, None, 0.0, 0, None, ctypes.byref(out)) == qt.QT_ERR_ARG
    assert qt.lib.qt_multiply_tau(None, None, -1.0, 0, None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_norms(None, None, None, 0, None) == qt.QT_ERR_ARG
    qt.lib.qt_free(None)


@pytest.mark.parametrize("args,status", [
    ((64, 64, 7, 7, 0), 2),        # block size not in {16, 32, 64}
    ((64, 64, 32, 96, 0), 2),      # leaf / b = 3, not a power of two
    ((64, 64, 16, 256, 0), 2),     # leaf / b = 16 > 8
    ((100, 64, 32, 32, 0), 2),     # dimension not a multiple of b
    ((-32, 64, 32, 32, 0), 1),     # negative size
    ((64, 64, 32, 32, -1), 1),     # negative block count
    ((64, 64, 32, 32, 3), 1),      # NULL block list
])
def test_build_argument_checks(args, status):
    import paper_1501_07800_amd as qt
    out = ctypes.c_void_p()
    rc = qt.lib.qt_build(*args, None, None, None, 0, None, ctypes.byref(out))
    assert rc == status, qt.lib.qt_last_error()
    assert out.value is None
    assert qt.lib.qt_last_error()


def test_plan_and_tuner_argument_checks():
    import paper_1501_07800_amd as qt
    out = ctypes.c_void_p()
    assert qt.lib.qt_plan_create(0, None, None, 0, None, ctypes.byref(out)) == qt.QT_ERR_ARG
    assert out.value is None
    assert qt.lib.qt_plan_create(1, None, None, 0, None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_plan_execute(None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_plan_replay(None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_plan_tune(None, None, 1, None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_plan_set_schedule(None, 0) == qt.QT_ERR_ARG
    assert qt.lib.qt_plan_result(None, 0, ctypes.byref(out)) == qt.QT_ERR_ARG
    assert qt.lib.qt_plan_info(None, None, None, None) == qt.QT_ERR_ARG
    qt.lib.qt_plan_destroy(None)
    best = ctypes.c_int32()
    assert qt.lib.qt_tune_leaf(None, None, 0, None, 1, ctypes.byref(best), None, None, 0, None) == qt.QT_ERR_ARG


def test_set_allocator_argument_checks():
    """qt_set_allocator needs both callbacks or neither (no GPU needed)."""
    import paper_1501_07800_amd as qt
    a = qt.ALLOC_FN(lambda n, s, c: None)
    f = qt.FREE_FN(lambda p, s, c: None)
    assert qt.lib.qt_set_allocator(ctypes.cast(a, ctypes.c_void_p), None, None) == qt.QT_ERR_ARG
    assert qt.lib.qt_set_allocator(None, ctypes.cast(f, ctypes.c_void_p), None) == qt.QT_ERR_ARG
    prev = qt._installed
    assert qt.lib.qt_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p), None) == 0
    assert qt.lib.qt_set_allocator(None, None, None) == 0
    if prev is not None:          # put back what the binding installed
        qt.set_allocator(prev[2], prev[3])
