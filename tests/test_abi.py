"""The C ABI library (CPU-only checks): it loads and exports every function
include/iwpp.h declares; the Python binding validates arguments before any
GPU call."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "iwpp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(iwpp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_declared_symbols():
    from paper_1209_3314_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1209_3314_amd import build

        build.build()
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert names == sorted(_lib.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.iwpp_version() >= 1


def test_binding_rejects_bad_tensors_before_the_library():
    torch = pytest.importorskip("torch")
    import paper_1209_3314_amd as iw

    cpu = torch.zeros((4, 4), dtype=torch.uint8)
    with pytest.raises(ValueError):
        iw.morph_recon(cpu, cpu)
    with pytest.raises(TypeError):
        iw.edt(torch.zeros((4, 4), dtype=torch.float32))
    with pytest.raises(TypeError):
        iw.edt([[0, 1]])
