"""CPU-side checks of the C ABI: the library builds for gfx950, loads, and
exports every entry point that include/embedjoin.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "embedjoin.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ej_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    import paper_1702_00093_amd as ej
    if not os.path.exists(ej.LIB_PATH):
        from paper_1702_00093_amd import build
        build.build()
    return ej.LIB_PATH


def test_header_declares_the_stage_entry_points():
    d = _declared()
    for name in ["ej_embed", "ej_lsh_bucket", "ej_candidates", "ej_verify", "ej_join"]:
        assert name in d


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    import paper_1702_00093_amd as ej
    assert sorted(ej.EXPORTS) == _declared()


def test_version_and_null_handling(libpath):
    import paper_1702_00093_amd as ej
    L = ej.lib()
    assert L.ej_version() >= 10000
    # calls with a null context fail cleanly without touching a device
    assert L.ej_join(None, None, None, 0, 0, 1, 1, 1, 0, None) == ej.EJ_EINVAL
    assert L.ej_last_error(None) == b"null context"
    assert L.ej_workspace_bytes(None) == 0
    L.ej_destroy(None)
    L.ej_result_free(None)


def test_gfx950_code_object_present(libpath):
    data = open(libpath, "rb").read()
    assert b"gfx950" in data


def test_tune_calls_reject_null_context(libpath):
    import ctypes as C
    import paper_1702_00093_amd as ej
    L = ej.lib()
    v = C.c_uint32()
    assert L.ej_tune_set(None, b"radix_bits", 8) == ej.EJ_EINVAL
    assert L.ej_tune_get(None, b"radix_bits", C.byref(v)) == ej.EJ_EINVAL
