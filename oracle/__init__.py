"""Plain, slow CPU oracle for the IWPP operations of arXiv 1209.3314.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1209_3314_amd``), and the GPU library never calls
it.

Two layers:

* ``liboracle.so`` (``iwpp_oracle.c``, plain C, single-threaded): the
  sequential algorithms of the paper -- Fast Hybrid reconstruction
  (Algorithm 2), the round reading of the propagation EDT (Algorithms 3/6) in
  frontier and dense form, Algorithm 3 literally, and two exact EDTs.
* numpy (this file): the definition of reconstruction by dilation -- the
  elementary geodesic dilation of Sec. 2.1 iterated until nothing changes.

Parity status (each pin lives in ``tests/test_oracle_*.py``):

* ``mr_fh``        pinned: equals ``mr_iterate`` (the definition) and the
  threshold-decomposition closed form; invariants and special cases.
* ``mr_iterate``   pinned: threshold decomposition, special cases.
* ``edt_rounds``   pinned: equals ``edt_dense``; exact on one-row images, on a
  single feature (with round count = Chebyshev/Manhattan radius); never below
  the exact EDT; the Fig. 3 error case (170 where exact is 169) reproduced.
  Agreement with the paper's own (lost) outputs is parity unpinned.
* ``edt_dense``    pinned as above (it is the other half of the self-check).
* ``edt_alg3``     reported only (differences from the round reading).
* ``edt_exact_bf`` / ``edt_exact_sep`` pinned against each other and scipy's
  exact EDT.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i64 = ctypes.c_int64
    lib.oracle_mr_fh.argtypes = [u8p, u8p, u8p, i64, i64, ctypes.c_int, i64p]
    lib.oracle_mr_erode.argtypes = [u8p, u8p, u8p, i64, i64, ctypes.c_int, i64p]
    for name in ("oracle_edt_rounds", "oracle_edt_dense", "oracle_edt_alg3"):
        getattr(lib, name).argtypes = [u8p, i32p, i32p, i64, i64, ctypes.c_int, i64p]
    lib.oracle_edt_exact_bf.argtypes = [u8p, i32p, i32p, i64, i64]
    lib.oracle_edt_exact_sep.argtypes = [u8p, i64p, i64, i64]
    for name in ("oracle_mr_fh", "oracle_edt_rounds", "oracle_edt_dense", "oracle_edt_alg3",
                 "oracle_edt_exact_bf", "oracle_edt_exact_sep"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _u8(img) -> np.ndarray:
    a = np.ascontiguousarray(img, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError("expected a 2-D image")
    return a


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


# --------------------------------------------------------------------------
# Morphological reconstruction by dilation (Sec. 2.1)

def mr_fh(marker, mask, conn: int = 8, return_stats: bool = False):
    """Sequential Fast Hybrid reconstruction rho_I(J) (Algorithm 2).

    The marker is clamped to the mask first (J <- J ^ I).  With
    ``return_stats`` also returns a dict: ``initial`` (pixels queued by the
    anti-raster scan), ``pops`` (Q_ref, queue pops of the propagation phase),
    ``pushes`` and ``depth`` (longest chain of queue generations).
    """
    lib = _load()
    J, I = _u8(marker), _u8(mask)
    if J.shape != I.shape:
        raise ValueError("marker and mask must have the same shape")
    h, w = J.shape
    out = np.empty_like(J)
    st = np.zeros(4, dtype=np.int64)
    _check(lib.oracle_mr_fh(_ptr(J, ctypes.c_uint8), _ptr(I, ctypes.c_uint8), _ptr(out, ctypes.c_uint8),
                            h, w, conn, _ptr(st, ctypes.c_int64)), "oracle_mr_fh")
    if return_stats:
        return out, {"initial": int(st[0]), "pops": int(st[1]), "pushes": int(st[2]), "depth": int(st[3])}
    return out


def mr_erode(marker, mask, conn: int = 8, return_stats: bool = False):
    """Reconstruction by erosion rho*_I(J): the limit of
    J(p) <- max(min{J(q) : q in N_G(p) U {p}}, I(p)) from a marker above the
    mask (a marker below the mask is raised to it first).  Stats as mr_fh."""
    lib = _load()
    J, I = _u8(marker), _u8(mask)
    if J.shape != I.shape:
        raise ValueError("marker and mask must have the same shape")
    h, w = J.shape
    out = np.empty_like(J)
    st = np.zeros(4, dtype=np.int64)
    _check(lib.oracle_mr_erode(_ptr(J, ctypes.c_uint8), _ptr(I, ctypes.c_uint8), _ptr(out, ctypes.c_uint8),
                               h, w, conn, _ptr(st, ctypes.c_int64)), "oracle_mr_erode")
    if return_stats:
        return out, {"initial": int(st[0]), "pops": int(st[1]), "pushes": int(st[2]), "depth": int(st[3])}
    return out


def geodesic_erosion(J: np.ndarray, I: np.ndarray, conn: int = 8) -> np.ndarray:
    """One elementary geodesic erosion: J'(p) = max(min{J(q) : q in N_G(p) U {p}}, I(p));
    pixels outside the image are not neighbours."""
    J = np.asarray(J)
    h, w = J.shape
    P = np.full((h + 2, w + 2), 256, dtype=np.int16)  # 256 padding never wins a min of bytes
    P[1:-1, 1:-1] = J
    m = P[1:-1, 1:-1].copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if (dy, dx) == (0, 0) or (conn == 4 and dy != 0 and dx != 0):
                continue
            m = np.minimum(m, P[1 + dy:h + 1 + dy, 1 + dx:w + 1 + dx])
    return np.maximum(m, np.asarray(I)).astype(np.uint8)


def mr_erode_iterate(marker, mask, conn: int = 8) -> np.ndarray:
    """rho*_I(J) by its definition: geodesic erosions from max(J, I) until
    nothing changes (slow; small images)."""
    I = _u8(mask)
    J = np.maximum(_u8(marker), I)
    while True:
        K = geodesic_erosion(J, I, conn)
        if np.array_equal(K, J):
            return J
        J = K


def geodesic_dilation(J: np.ndarray, I: np.ndarray, conn: int = 8) -> np.ndarray:
    """One elementary geodesic dilation of Sec. 2.1:
    J'(p) = max{J(q) : q in N_G(p) U {p}} ^ I(p); pixels outside the image are
    not neighbours."""
    J = np.asarray(J)
    h, w = J.shape
    P = np.zeros((h + 2, w + 2), dtype=np.int16)  # 0 padding never wins a max of values >= 0
    P[1:-1, 1:-1] = J
    m = P[1:-1, 1:-1].copy()
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if conn == 8:
        offs += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    for dy, dx in offs:
        np.maximum(m, P[1 + dy:1 + dy + h, 1 + dx:1 + dx + w], out=m)
    return np.minimum(m, np.asarray(I, dtype=np.int16)).astype(np.uint8)


def mr_iterate(marker, mask, conn: int = 8, return_steps: bool = False):
    """Reconstruction by its definition: iterate the elementary geodesic
    dilation from J ^ I until no pixel changes (Sec. 2.1).  Slow; for small
    images."""
    J, I = _u8(marker), _u8(mask)
    cur = np.minimum(J, I)
    steps = 0
    while True:
        nxt = geodesic_dilation(cur, I, conn)
        if np.array_equal(nxt, cur):
            break
        cur = nxt
        steps += 1
    return (cur, steps) if return_steps else cur


# --------------------------------------------------------------------------
# Euclidean distance transform (Sec. 2.2); features (targets) are 0-pixels.

def _edt_call(fn_name: str, binary, conn: int):
    lib = _load()
    B = _u8(binary)
    h, w = B.shape
    sq = np.empty((h, w), dtype=np.int32)
    nr = np.empty((h, w), dtype=np.int32)
    st = np.zeros(3, dtype=np.int64)
    _check(getattr(lib, fn_name)(_ptr(B, ctypes.c_uint8), _ptr(sq, ctypes.c_int32), _ptr(nr, ctypes.c_int32),
                                 h, w, conn, _ptr(st, ctypes.c_int64)), fn_name)
    return sq, nr, st


def edt_rounds(binary, conn: int = 8, return_stats: bool = False):
    """Propagation EDT in level-synchronous rounds with snapshot reads and the
    (squared distance, feature index) tie-break -- the frontier form.

    Returns ``(sqdist, nearest)`` as int32 arrays; ``nearest`` is y*W+x of the
    chosen feature.  Both are -1 everywhere when there is no feature.  With
    ``return_stats`` also a dict: ``rounds``, ``items`` (frontier total,
    Q_ref) and ``initial`` (contour features).
    """
    sq, nr, st = _edt_call("oracle_edt_rounds", binary, conn)
    if return_stats:
        return sq, nr, {"rounds": int(st[0]), "items": int(st[1]), "initial": int(st[2])}
    return sq, nr


def edt_dense(binary, conn: int = 8, return_stats: bool = False):
    """The same rounds as a dense Jacobi operator (every pixel, every round)."""
    sq, nr, st = _edt_call("oracle_edt_dense", binary, conn)
    if return_stats:
        return sq, nr, {"rounds": int(st[0])}
    return sq, nr


def edt_alg3(binary, conn: int = 8, return_stats: bool = False):
    """Algorithm 3 taken literally (one FIFO, in-place, strict comparison)."""
    sq, nr, st = _edt_call("oracle_edt_alg3", binary, conn)
    if return_stats:
        return sq, nr, {"pops": int(st[0])}
    return sq, nr


def edt_exact_bf(binary):
    """Exact EDT by brute force: smallest squared distance to any feature, the
    smallest feature index among ties.  O(pixels x features)."""
    lib = _load()
    B = _u8(binary)
    h, w = B.shape
    sq = np.empty((h, w), dtype=np.int32)
    nr = np.empty((h, w), dtype=np.int32)
    _check(lib.oracle_edt_exact_bf(_ptr(B, ctypes.c_uint8), _ptr(sq, ctypes.c_int32), _ptr(nr, ctypes.c_int32),
                                   h, w), "oracle_edt_exact_bf")
    return sq, nr


def edt_exact_sep(binary) -> np.ndarray:
    """Exact squared EDT by the separable lower-envelope method (int64)."""
    lib = _load()
    B = _u8(binary)
    h, w = B.shape
    sq = np.empty((h, w), dtype=np.int64)
    _check(lib.oracle_edt_exact_sep(_ptr(B, ctypes.c_uint8), _ptr(sq, ctypes.c_int64), h, w),
           "oracle_edt_exact_sep")
    return sq
