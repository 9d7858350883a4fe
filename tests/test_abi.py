"""The C-ABI library loads on the CPU and exports every declared symbol."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fea.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fea_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1805_03949_amd as fea
    lib = ctypes.CDLL(fea.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n
    assert set(fea.EXPORTS) == set(names)


def test_version_and_error_string_without_gpu():
    import paper_1805_03949_amd as fea
    assert fea.version().startswith("fea-gfx950")
    assert fea._lib.fea_last_error() == b""
