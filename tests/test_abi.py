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


# C struct name in include/iwpp.h -> ctypes mirror in the binding
_MIRRORS = {"iwpp_options": "Options", "iwpp_stats": "Stats", "iwpp_kernel_time": "KernelTime",
            "iwpp_job": "Job", "iwpp_server_options": "ServerOptions", "iwpp_server_stats": "ServerStats",
            "iwpp_queue_options": "QueueOptions"}


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding passes through the ABI has the header's size
    and field offsets (a C program built with gcc against include/iwpp.h
    prints them)."""
    import shutil
    import subprocess

    from paper_1209_3314_amd import _lib

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "iwpp.h"', 'int main(void) {']
    for cname, pyname in _MIRRORS.items():
        st = getattr(_lib, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, pyname in _MIRRORS.items():
        st = getattr(_lib, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(st), cname
        for f, _ in st._fields_:
            assert got[(cname, f)] == getattr(st, f).offset, (cname, f)
