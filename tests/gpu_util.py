"""Helpers for the GPU tests: skip cleanly without a GPU, fail loudly without
the library, and print the case name before each GPU step."""
import sys

import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1209_3314_amd as iw
    from paper_1209_3314_amd import _lib

    _lib.load()  # raises if libiwpp.so is missing: there is no fallback
    return torch, iw


def announce(*parts):
    print("[gpu case]", *parts, file=sys.stderr, flush=True)
