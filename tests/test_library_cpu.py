"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every function
declared in include/wqfd.h, and the binding refuses to run without it."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wqfd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("wq_build_rules", "wq_rules_info_get", "wq_assemble_rows", "cut_assemble", "wq_assemble_adjoint",
              "wq_rules_free", "wq_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2211_06427_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libwqfd.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_last_error_is_callable_without_gpu():
    from paper_2211_06427_amd import _lib
    lib = _lib.load()
    assert isinstance(lib.wq_last_error(), bytes)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2211_06427_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "missing.so"))


def test_invalid_arguments_rejected_before_device_work():
    """Argument validation happens on the host; these calls never touch a GPU."""
    from paper_2211_06427_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    mesh = _lib.WqMesh((ctypes.c_int32 * 3)(4, 4, 4), 0, (ctypes.c_double * 3)(0, 0, 0), (ctypes.c_double * 3)(1, 1, 1))
    ls = _lib.WqLevelset()
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), None, None, ctypes.byref(h)) == -1
    assert b"degree" in lib.wq_last_error()
    mesh.degree = 7
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), None, None, ctypes.byref(h)) == -5
    mesh.degree = 2
    mesh.nel[1] = 0
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), None, None, ctypes.byref(h)) == -1
    mesh.nel[1] = 4
    ls.kind = 9
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), None, None, ctypes.byref(h)) == -1
    ls.kind = 0
    opts = _lib.WqOptions(9, 0)
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), ctypes.byref(opts), None, ctypes.byref(h)) == -1
    opts = _lib.WqOptions(3, 0x10)                      # unknown option bit
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), ctypes.byref(opts), None, ctypes.byref(h)) == -1
    opts = _lib.WqOptions(4, _lib.WQ_OPT_MOMENT_FIT)     # the fitted rule needs depth <= 3
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), ctypes.byref(opts), None, ctypes.byref(h)) == -5
    mesh.degree = 5
    opts = _lib.WqOptions(3, _lib.WQ_OPT_TENSOR)         # the coefficient tensor: degrees 1..4
    assert lib.wq_build_rules(ctypes.byref(mesh), ctypes.byref(ls), ctypes.byref(opts), None, ctypes.byref(h)) == -5
    assert b"degrees 1..4" in lib.wq_last_error()
    mesh.degree = 2
    assert lib.wq_assemble(None, 0, 3, None, None, None, None) == -1
    assert lib.wq_assemble_tensor(None, 0, None, None, None) == -1
    assert lib.wq_assemble_rows(None, 0, 3, None, None, None, None) == -1
    assert lib.cut_assemble(None, 0, 3, None, None, None, None) == -1
    assert lib.wq_assemble_adjoint(None, 0, 3, None, None, None, None) == -1
    assert lib.wq_rules_info_get(None, None) == -1
