"""Seeded synthetic inputs shaped like the paper's tissue tiles.

The paper measured on whole-slide brain-tumour tissue images that are not
available; these generators stand in for them.  This module only draws pixels:
it holds none of the reconstruction or distance-transform arithmetic, and both
the GPU library's callers and the CPU oracle's callers consume the same bytes.

Recipes (all drawn from ``numpy.random.default_rng``):

``mr_inputs`` -- grayscale reconstruction (mask I, marker J):
  1. noise ~ uniform integers [0, 255] (uint8), as float32;
  2. Gaussian blur, sigma 4 (scipy ``gaussian_filter``, mode ``reflect``,
     truncate 4), rounded to nearest, clipped to [0, 255], uint8;
  3. ``n_disks`` disks, each drawn as (cx, cy, r, v) in that order: centre
     uniform over the image, integer radius uniform in ``radius``, value
     uniform in [200, 255]; pixels with (x-cx)^2 + (y-cy)^2 <= r^2 are
     overwritten with v (clipped at the border);
  4. marker = max(mask - offset, 0).

``slide_mr_inputs`` -- reconstruction inputs at whole-slide scale (billions
of pixels), block-structured so that drawing them takes seconds (see its
docstring).

``edt_input`` -- binary nucleus-like image (1 = background to measure,
0 = feature/target):
  start from all ones; repeatedly draw a shape -- with probability 1/2 a disk
  of integer radius U[4, 40], else an ellipse with integer semi-axes U[4, 40]
  each and angle U[0, pi) -- centred uniformly, and paint it 0; stop once the
  0-fraction reaches ``coverage``.
"""
from __future__ import annotations

import math

import numpy as np

# Disk density of the 512x512 reconstruction workload: 40 disks per 512^2 px.
MR_DISK_DENSITY = 40.0 / (512 * 512)


def _paint_disk(img: np.ndarray, cx: int, cy: int, r: int, v: int) -> int:
    """Overwrite the disk with value v; return how many pixels changed to v."""
    h, w = img.shape
    y0, y1 = max(cy - r, 0), min(cy + r, h - 1)
    x0, x1 = max(cx - r, 0), min(cx + r, w - 1)
    if y0 > y1 or x0 > x1:
        return 0
    yy = np.arange(y0, y1 + 1, dtype=np.int64)[:, None] - cy
    xx = np.arange(x0, x1 + 1, dtype=np.int64)[None, :] - cx
    inside = yy * yy + xx * xx <= r * r
    sub = img[y0:y1 + 1, x0:x1 + 1]
    changed = int(np.count_nonzero(inside & (sub != v)))
    sub[inside] = v
    return changed


def _paint_ellipse(img: np.ndarray, cx: int, cy: int, a: int, b: int, theta: float, v: int) -> int:
    h, w = img.shape
    r = max(a, b)
    y0, y1 = max(cy - r, 0), min(cy + r, h - 1)
    x0, x1 = max(cx - r, 0), min(cx + r, w - 1)
    if y0 > y1 or x0 > x1:
        return 0
    yy = np.arange(y0, y1 + 1, dtype=np.float64)[:, None] - cy
    xx = np.arange(x0, x1 + 1, dtype=np.float64)[None, :] - cx
    c, s = math.cos(theta), math.sin(theta)
    u = (xx * c + yy * s) / a
    t = (-xx * s + yy * c) / b
    inside = u * u + t * t <= 1.0
    sub = img[y0:y1 + 1, x0:x1 + 1]
    changed = int(np.count_nonzero(inside & (sub != v)))
    sub[inside] = v
    return changed


def mr_inputs(h: int, w: int, seed: int, n_disks: int, radius=(5, 20), offset: int = 32):
    """Return (marker, mask) uint8 arrays of shape (h, w); see module doc."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    noise = rng.integers(0, 256, size=(h, w), dtype=np.uint8).astype(np.float32)
    blurred = gaussian_filter(noise, sigma=4.0, mode="reflect", truncate=4.0)
    del noise
    mask = np.clip(np.rint(blurred), 0, 255).astype(np.uint8)
    del blurred
    lo, hi = radius
    for _ in range(int(n_disks)):
        cx = int(rng.integers(0, w))
        cy = int(rng.integers(0, h))
        r = int(rng.integers(lo, hi + 1))
        v = int(rng.integers(200, 256))
        _paint_disk(mask, cx, cy, r, v)
    marker = np.maximum(mask.astype(np.int16) - int(offset), 0).astype(np.uint8)
    return marker, mask


def edt_input(h: int, w: int, seed: int, coverage: float = 0.30) -> np.ndarray:
    """Return a uint8 (h, w) image: 0 = feature (target), 1 = background."""
    rng = np.random.default_rng(seed)
    img = np.ones((h, w), dtype=np.uint8)
    need = coverage * h * w
    zeros = 0
    while zeros < need:
        if rng.random() < 0.5:
            cx = int(rng.integers(0, w))
            cy = int(rng.integers(0, h))
            r = int(rng.integers(4, 41))
            zeros += _paint_disk(img, cx, cy, r, 0)
        else:
            cx = int(rng.integers(0, w))
            cy = int(rng.integers(0, h))
            a = int(rng.integers(4, 41))
            b = int(rng.integers(4, 41))
            theta = float(rng.uniform(0.0, math.pi))
            zeros += _paint_ellipse(img, cx, cy, a, b, theta, 0)
    return img


def slide_mr_inputs(h: int, w: int, seed: int, block: int = 32, offset: int = 40, seed_frac: float = 0.002):
    """Whole-slide-scale reconstruction inputs that are cheap to draw at
    billions of pixels: a field of ``block`` x ``block`` blocks with levels
    uniform in [0, 219], plus a row ripple 4 * (y mod 7) and a column ripple
    3 * (x mod 5) (so no block is flat); marker = max(mask - offset, 0),
    except in a ``seed_frac`` fraction of the blocks (drawn after the levels),
    where marker = mask.  Returns (marker, mask) uint8 arrays of shape (h, w),
    filled one block row at a time."""
    rng = np.random.default_rng(seed)
    bh, bw = (h + block - 1) // block, (w + block - 1) // block
    levels = rng.integers(0, 220, size=(bh, bw), dtype=np.uint8)
    seeds = rng.random((bh, bw)) < seed_frac
    rowr = ((np.arange(h) % 7) * 4).astype(np.uint8)
    colr = ((np.arange(w) % 5) * 3).astype(np.uint8)
    mask = np.empty((h, w), dtype=np.uint8)
    marker = np.empty((h, w), dtype=np.uint8)
    for by in range(bh):
        rows = slice(by * block, min((by + 1) * block, h))
        lv = np.repeat(levels[by], block)[:w]
        m = lv[None, :] + rowr[rows, None] + colr[None, :]
        mask[rows] = m
        sd = np.repeat(seeds[by], block)[:w]
        marker[rows] = np.where(sd[None, :], m, np.maximum(m.astype(np.int16) - offset, 0).astype(np.uint8))
    return marker, mask


# ---------------------------------------------------------------------------
# Named workloads

def workload_mr_small():
    """512x512 reconstruction, 8-connected: 40 disks of radius 5-20, offset 32, seed 0."""
    return mr_inputs(512, 512, seed=0, n_disks=40, radius=(5, 20), offset=32)


def workload_edt_4k():
    """4096x4096 EDT input, ~30% nucleus-like features, seed 0."""
    return edt_input(4096, 4096, seed=0, coverage=0.30)


def workload_mr_16k():
    """16384x16384 reconstruction: ~20k disks of radius 5-30, offset 48, seed 0."""
    return mr_inputs(16384, 16384, seed=0, n_disks=20000, radius=(5, 30), offset=48)


def batch_tile_spec(i: int) -> dict:
    """Spec of tile i of the 256-tile mixed batch: sides uniform in [512, 4096];
    even i reconstruction (disk density of the 512^2 workload, radius 5-20,
    offset uniform in [16, 64], 8-connected), odd i EDT (coverage uniform in
    [0.10, 0.50], 8-connected).  Content seed is 1000 + i."""
    rng = np.random.default_rng([7, 1000 + i])
    h = int(rng.integers(512, 4097))
    w = int(rng.integers(512, 4097))
    if i % 2 == 0:
        return {"op": "mr", "h": h, "w": w, "seed": 1000 + i, "conn": 8,
                "n_disks": int(round(MR_DISK_DENSITY * h * w)), "offset": int(rng.integers(16, 65))}
    return {"op": "edt", "h": h, "w": w, "seed": 1000 + i, "conn": 8,
            "coverage": float(rng.uniform(0.10, 0.50))}


def tile_inputs(spec: dict):
    """Materialise a spec from ``batch_tile_spec``/``serve_trace``: returns
    (marker, mask) for reconstruction or the binary image for EDT."""
    if spec["op"] == "mr":
        return mr_inputs(spec["h"], spec["w"], spec["seed"], spec["n_disks"], (5, 20), spec["offset"])
    return edt_input(spec["h"], spec["w"], spec["seed"], spec["coverage"])


def serve_trace(rate: float, duration_s: float, seed: int = 0, sigma: float = 0.7):
    """Open-loop request trace: Poisson arrivals at ``rate`` per second for
    ``duration_s``; square tiles with side round(1024 * exp(sigma * Z)) clipped
    to [256, 8192]; 70% reconstruction / 30% EDT, generated as the batch tiles.
    Returns a list of (arrival_time_s, spec)."""
    rng = np.random.default_rng([11, seed, int(rate)])
    out = []
    t = 0.0
    k = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            break
        side = int(np.clip(round(1024.0 * math.exp(sigma * float(rng.standard_normal()))), 256, 8192))
        s = 100000 + seed * 1000003 + k
        if rng.random() < 0.7:
            spec = {"op": "mr", "h": side, "w": side, "seed": s, "conn": 8,
                    "n_disks": int(round(MR_DISK_DENSITY * side * side)), "offset": int(rng.integers(16, 65))}
        else:
            spec = {"op": "edt", "h": side, "w": side, "seed": s, "conn": 8,
                    "coverage": float(rng.uniform(0.10, 0.50))}
        out.append((t, spec))
        k += 1
    return out


def serve_pool(size: int = 64, seed: int = 0, sigma: float = 0.7) -> list:
    """A bounded pool of request inputs drawn like ``serve_trace``'s requests
    (square sides round(1024 * exp(sigma * Z)) clipped to [256, 8192]); exactly
    round(0.7 * size) reconstruction tiles, the rest EDT.  Generating one input
    per request is too slow for long traces, so requests reuse pool items."""
    rng = np.random.default_rng([13, seed])
    n_mr = int(round(0.7 * size))
    out = []
    for k in range(size):
        side = int(np.clip(round(1024.0 * math.exp(sigma * float(rng.standard_normal()))), 256, 8192))
        s = 200000 + seed * 1000003 + k
        if k < n_mr:
            out.append({"op": "mr", "h": side, "w": side, "seed": s, "conn": 8,
                        "n_disks": int(round(MR_DISK_DENSITY * side * side)), "offset": int(rng.integers(16, 65))})
        else:
            out.append({"op": "edt", "h": side, "w": side, "seed": s, "conn": 8,
                        "coverage": float(rng.uniform(0.10, 0.50))})
    return out


def serve_arrivals(rate: float, duration_s: float, pool_size: int, seed: int = 0) -> list:
    """Open-loop Poisson arrivals at ``rate`` per second over ``duration_s``,
    each naming a pool item uniformly at random: a list of (time_s, index)."""
    rng = np.random.default_rng([17, seed, int(rate)])
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            return out
        out.append((t, int(rng.integers(pool_size))))
