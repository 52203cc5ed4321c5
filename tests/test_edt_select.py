"""The EDT kernel picks a pixel's nearest candidate with 32-bit minima: the
smallest squared distance dm, then the smallest feature among candidates at
dm, selected by OR-ing the sign bit of (dm - d) into each feature.  This
checks that identity against the plain lexicographic minimum of
(squared distance, feature) on the packed encoding the kernel uses (features
y << 16 | x with coordinates below 32767, "none" = 0x80008000 whose
saturated distance is 2 * 32767^2), including ties and all-none sets."""
import numpy as np

NONE = 0x80008000


def d2(q, f):
    """Saturating packed 16-bit difference, then the 2-term dot product."""
    def halves(v):
        lo = np.int64(np.int16(np.uint16(v & 0xFFFF)))
        hi = np.int64(np.int16(np.uint16((v >> 16) & 0xFFFF)))
        return lo, hi
    ql, qh = halves(q)
    fl, fh = halves(f)
    el = int(np.clip(ql - fl, -32768, 32767))
    eh = int(np.clip(qh - fh, -32768, 32767))
    return el * el + eh * eh


def select_sign_bit(q, fs):
    d = [d2(q, f) for f in fs]
    dm = min(d)
    return min(f | (((dm - di) & 0xFFFFFFFF) & 0x80000000) for f, di in zip(fs, d))


def select_lex(q, fs):
    return min((d2(q, f), f) for f in fs)[1]


def test_sign_bit_selection_equals_lexicographic_minimum():
    rng = np.random.default_rng(7)
    for _ in range(20000):
        qy, qx = (int(v) for v in rng.integers(0, 32767, 2))
        q = (qy << 16) | qx
        k = int(rng.integers(1, 10))
        fs = []
        for _ in range(k):
            r = rng.random()
            if r < 0.2:
                fs.append(NONE)
            elif r < 0.5:  # near q, so that ties are common
                y = min(32766, max(0, qy + int(rng.integers(-3, 4))))
                x = min(32766, max(0, qx + int(rng.integers(-3, 4))))
                fs.append((y << 16) | x)
            else:
                y, x = (int(v) for v in rng.integers(0, 32767, 2))
                fs.append((y << 16) | x)
        assert select_sign_bit(q, fs) == select_lex(q, fs)


def test_all_none_and_far_corners():
    assert select_sign_bit(0, [NONE, NONE]) == NONE
    far = (32766 << 16) | 32766
    # the farthest real feature still beats "none"
    assert select_sign_bit(0, [NONE, far]) == far
    assert d2(0, far) < d2(0, NONE) < 2 ** 31
    # equidistant features: the smaller packed value wins
    a, b = (1 << 16) | 0, (0 << 16) | 1
    q = 0
    assert d2(q, a) == d2(q, b) and select_sign_bit(q, [a, b]) == min(a, b)
