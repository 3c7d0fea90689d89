"""The C ABI library loads and exports every entry point include/haze.h
declares; host-side error paths that need no GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "haze.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hz_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze
    if not os.path.exists(haze.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return haze


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("hz_splat_index_field", "hz_trace_views", "hz_submit", "hz_poll"):
        assert required in names


def test_library_exports_every_declared_symbol(haze):
    L = C.CDLL(haze.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(haze.EXPORTS) == _declared()


def test_context_create_without_gpu_fails_cleanly(haze):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = haze.lib()
    h = C.c_void_p()
    assert L.hz_ctx_create(0, 0, C.byref(h)) == haze.E_DEVICE
    assert h.value is None
    assert "device" in haze.last_error()
    with pytest.raises(haze.HazeError):
        haze.Context(0)


def test_null_arguments_are_rejected(haze):
    L = haze.lib()
    assert L.hz_ctx_create(0, 0, None) == haze.E_INVALID
    assert L.hz_splat_index_field(None, None, None, None, None, None) == haze.E_INVALID
    assert "NULL" in haze.last_error()
    assert L.hz_trace_views(None, None, None, 0, None, None, 0, None, None) == haze.E_INVALID
    assert L.hz_field_release(None, None) == haze.E_INVALID
    assert L.hz_ctx_memory(None, None, None) == haze.E_INVALID
    L.hz_ctx_destroy(None)   # ignored
