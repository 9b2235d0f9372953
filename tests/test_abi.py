"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/elm.h declares, and rejects calls without a handle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elm.h")
LIB = os.path.join(ROOT, "paper_2011_02436_amd", "libelm.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(elm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2011_02436_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_path_calls():
    names = declared_functions()
    for n in ("elm_hidden", "elm_rank_factor", "elm_pinv_solve", "elm_predict"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    lib.elm_status_string.restype = ctypes.c_char_p
    lib.elm_status_string.argtypes = [ctypes.c_int]
    seen = set()
    for st in range(8):
        s = lib.elm_status_string(st).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 8
    assert lib.elm_status_string(99).decode() == "unknown status"


def test_null_handle_rejected(lib):
    vp = ctypes.c_void_p
    assert lib.elm_hidden(vp(), 10, 2, 3, vp(1), 2, vp(1), 3, vp(1), 0, vp(1), 3, vp(), 0, 2) == 1
    f = vp()
    r = ctypes.c_int64()
    assert lib.elm_rank_factor(vp(), 10, 3, vp(1), 3, 0, 0, ctypes.c_double(0.0), ctypes.byref(f),
                               ctypes.byref(r)) == 1
    assert lib.elm_pinv_solve(vp(), vp(), 2, vp(1), 2, vp(1), 3, ctypes.c_double(1e-10), 0, vp(1), 2,
                              vp()) == 1
    assert lib.elm_predict(vp(), 10, 2, 3, 2, vp(1), 2, vp(1), 3, vp(1), 0, vp(1), 2, vp(1), 2, vp()) == 1
    assert lib.elm_create(None, vp()) == 1
    assert lib.elm_destroy(vp()) == 0
    assert lib.elm_factor_destroy(vp()) == 0


def test_binding_module_fails_loudly_without_library(tmp_path, monkeypatch):
    # the binding refuses to import when libelm.so is absent (no CPU fallback)
    import importlib.util
    src = os.path.join(ROOT, "paper_2011_02436_amd", "elm.py")
    dst = tmp_path / "elm_copy.py"
    dst.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("elm_copy", str(dst))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)
