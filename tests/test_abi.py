"""The C ABI library loads and exports what include/*.h declares; host-side
argument checks return SPAMM_EINVAL before any device work (no GPU needed)."""
import ctypes
import os

import pytest

import paper_1011_3534_amd as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(sp.LIB_PATH):
        pytest.skip("libspamm.so not built (run paper_1011_3534_amd.build)")
    return sp.lib()


def test_every_declared_symbol_is_exported():
    L = _lib_or_skip()
    names = sp.declared_symbols()
    assert {"spamm_build", "spamm_multiply", "spamm_sp2"} <= set(names)
    for name in names:
        assert hasattr(L, name), f"{name} declared in include/ but not exported"


def test_build_rejects_bad_arguments():
    L = _lib_or_skip()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert L.spamm_build(None, 16, 16, 1, 64, None, ctypes.byref(h)) == 1          # null input
    assert L.spamm_build(fake, 0, 16, 1, 64, None, ctypes.byref(h)) == 1           # n < 1
    assert L.spamm_build(fake, 16, 8, 1, 64, None, ctypes.byref(h)) == 1           # lda < n
    assert L.spamm_build(fake, 16, 16, 1, 48, None, ctypes.byref(h)) == 1          # bad leaf
    assert L.spamm_build(fake, 16, 16, 1, 16, None, ctypes.byref(h)) == 1          # leaf 16 not built
    assert L.spamm_build(fake, 16, 16, 9, 64, None, ctypes.byref(h)) == 1          # bad dtype
    assert L.spamm_build(fake, 16, 16, 1, 64, None, None) == 1                     # null out
    assert h.value is None
    assert b"leaf" in L.spamm_last_error() or b"null" in L.spamm_last_error()


def test_view_build_rejects_bad_layouts():
    # a view reads the caller's array in place: no padding, 16-byte rows,
    # 32-bit buffer offsets (checked before any device work)
    L = _lib_or_skip()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert L.spamm_build_view(fake, 100, 128, 1, 64, None, ctypes.byref(h)) == 1          # n % leaf != 0
    assert b"multiple of the leaf" in L.spamm_last_error()
    assert L.spamm_build_view(ctypes.c_void_p(0x1004), 128, 128, 1, 64, None, ctypes.byref(h)) == 1  # base
    assert L.spamm_build_view(fake, 128, 130, 1, 64, None, ctypes.byref(h)) == 1          # row pitch 520 B
    assert b"16-byte" in L.spamm_last_error()
    assert L.spamm_build_view(fake, 128, 1 << 23, 1, 64, None, ctypes.byref(h)) == 1      # 64 rows = 2 GiB
    assert b"2^31" in L.spamm_last_error()
    assert L.spamm_build_view(None, 128, 128, 1, 64, None, ctypes.byref(h)) == 1
    assert L.spamm_build_view(fake, 128, 128, 1, 48, None, ctypes.byref(h)) == 1
    assert h.value is None
    PA = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    N = (ctypes.c_int64 * 2)(128, 96)
    LD = (ctypes.c_int64 * 2)(128, 96)
    PO = (ctypes.c_void_p * 2)(None, None)
    assert L.spamm_build_view_batched(2, PA, N, LD, 1, 64, None, PO) == 1                 # 96 % 64
    assert PO[0] is None and PO[1] is None


def test_multiply_rejects_null_operands():
    L = _lib_or_skip()
    h = ctypes.c_void_p()
    assert L.spamm_multiply(None, None, 1e-6, 1, None, ctypes.byref(h), None) == 1
    assert L.spamm_multiply(None, None, 1e-6, 1, None, None, None) == 1
    assert h.value is None


def test_helpers_reject_null():
    L = _lib_or_skip()
    assert L.spamm_to_dense(None, None, 1, None) == 1
    assert L.spamm_norms(None, 0, None, 0, None) == 1
    cnt = ctypes.c_int64()
    assert L.spamm_task_list(None, None, 0, ctypes.byref(cnt), None) == 1
    assert L.spamm_info(None, None, None, None, None) == 1
    L.spamm_free(None)                                                           # no-op


def test_allocator_callbacks_outlive_reinstall():
    # handles keep the allocator they were made with: the ctypes thunks must
    # stay alive when the allocator is installed again or switched back
    _lib_or_skip()
    sp.use_torch_allocator(True)
    a, d = sp._alloc_cb, sp._dealloc_cb
    sp.use_torch_allocator(True)
    assert sp._alloc_cb is a and sp._dealloc_cb is d
    sp.use_torch_allocator(False)
    assert sp._alloc_cb is a and sp._dealloc_cb is d


def test_set_allocator_requires_both_functions():
    L = _lib_or_skip()
    alloc = sp._ALLOC_FN(lambda n, s, c: None)
    assert L.spamm_set_allocator(alloc, sp._DEALLOC_FN(), None) == 1
    assert L.spamm_set_allocator(sp._ALLOC_FN(), sp._DEALLOC_FN(), None) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sp, "_lib", None)
    monkeypatch.setattr(sp, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        sp.lib()


def test_autotune_rejects_bad_arguments():
    L = _lib_or_skip()
    n = (ctypes.c_int64 * 1)(64)
    tau = (ctypes.c_double * 1)(1e-6)
    ptrs = (ctypes.c_void_p * 1)(0x1000)
    best = sp.Tune()
    bad_leaf = (ctypes.c_int32 * 1)(48)
    good = (ctypes.c_int32 * 1)(64)
    assert L.spamm_autotune_batched(0, ptrs, n, 1, tau, 1, good, 1, 1e-6, 1, None, None, ctypes.byref(best), None) == 1
    assert L.spamm_autotune_batched(1, ptrs, n, 1, tau, 1, bad_leaf, 1, 1e-6, 1, None, None, ctypes.byref(best), None) == 1
    assert L.spamm_autotune_batched(1, ptrs, n, 1, tau, 1, good, 4, 1e-6, 1, None, None, ctypes.byref(best), None) == 1
    assert L.spamm_autotune_batched(1, ptrs, n, 1, tau, 1, good, 1, 0.0, 1, None, None, ctypes.byref(best), None) == 1
    assert L.spamm_autotune_batched(1, ptrs, n, 1, tau, 1, good, 1, 1e-6, 0, None, None, ctypes.byref(best), None) == 1
    assert L.spamm_autotune_batched(1, ptrs, n, 1, tau, 1, good, 1, 1e-6, 1, None, None, None, None) == 1


def test_batched_and_sp2_reject_bad_arguments():
    L = _lib_or_skip()
    PP = ctypes.c_void_p * 1
    tau = (ctypes.c_double * 1)(1e-6)
    assert L.spamm_multiply_batched(0, PP(), PP(), tau, 1, None, None, PP(), None) == 1
    assert L.spamm_multiply_batched(129, PP(), PP(), tau, 1, None, None, PP(), None) == 1
    assert L.spamm_multiply_batched(1, None, None, tau, 1, None, None, PP(), None) == 1
    h = ctypes.c_void_p()
    assert L.spamm_sp2(None, 1, 1e-6, 10, 1e-6, 1, None, ctypes.byref(h), None) == 1
