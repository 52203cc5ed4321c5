"""Autotuner for the library's launch options.

The options of ``iwpp_options`` change only speed, never results:
  * ``wg_waves`` -- waves per workgroup of the persistent kernels (the
    workgroup size; one wave holds one tile);
  * ``stage_depth`` -- work-list items a wave stages in LDS before one global
    atomic appends them (the depth of the paper's per-block queue);
  * ``mr_seed_strip`` -- tiles per vertical strip of the reconstruction seed
    pass (its tiling: each tile reads the one above it fresh);
  * ``mr_seed_sweeps`` / ``mr_max_sweeps`` -- sweep iterations per seed-pass
    tile and per propagation visit (the number of initial scans that Table 1
    varies);
  * ``persistent_blocks`` -- workgroups of the persistent kernels (the
    paper's blocks-per-multiprocessor knob, Sec. 5.2).
The tuner times a grid of candidates per (operation, connectivity, size
bucket) on synthetic inputs of that bucket -- and, for the "batch" bucket, on
a sample of the mixed 256-tile batch through ``run_batch`` -- checks that every
candidate's output equals the default options' output byte for byte, keeps
the fastest, and caches the choice as JSON keyed by device and library
version.  ``TunedContext`` applies the cached choice before each call,
``run_batch`` and ``batch_graph`` included.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import Context, _lib

DEFAULTS = {"persistent_blocks": 0, "mr_max_sweeps": 0, "mr_seed_sweeps": 0, "mr_list_capacity": 0, "wg_waves": 0,
            "stage_depth": 0, "mr_seed_strip": 0}

# Candidate grids.  0 means the library default (device-filling grid, four
# waves per workgroup, the deepest LDS stage, automatic strips, default sweep
# caps).
GRID = {
    "recon": [{"wg_waves": wg, "stage_depth": sd, "mr_seed_strip": sp, "mr_max_sweeps": ms, "mr_seed_sweeps": ss}
              for wg in (0, 8) for sd in (0, 16) for sp in (0, 4, 16) for ms in (0, 1) for ss in (0, 2)],
    "edt": [{"wg_waves": wg, "stage_depth": sd, "persistent_blocks": pb}
            for wg in (0, 8) for sd in (0, 16) for pb in (0, 512)],
    "batch": [{"wg_waves": wg, "stage_depth": sd, "mr_max_sweeps": ms, "persistent_blocks": pb}
              for wg in (0, 8) for sd in (0, 16) for ms in (0, 1) for pb in (0, 512)],
}


def bucket(op: str, conn: int, pixels: int) -> str:
    """Size bucket of a call: operation, connectivity and the next power of
    two of the pixel count (at least 2^12)."""
    if op not in ("recon", "edt", "batch"):
        raise ValueError(f"unknown op {op!r}")
    k = max(12, math.ceil(math.log2(max(1, pixels))))
    return f"{op}/{conn}/2^{k}"


def bucket_side(key: str) -> tuple:
    """A near-square (h, w) whose pixel count fills the bucket `key`."""
    k = int(key.rsplit("2^", 1)[1])
    h = 1 << (k // 2)
    return h, (1 << k) // h


def default_cache_path(device_name: str) -> str:
    base = os.environ.get("IWPP_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "iwpp")
    safe = "".join(c if c.isalnum() or c in "-_." else "_" for c in device_name)
    return os.path.join(base, f"tune_{safe}.json")


class TuneCache:
    """JSON cache {"version": v, "device": name, "entries": {bucket: {options, ms, default_ms}}}."""

    def __init__(self, path: str, device_name: str, version: int):
        self.path = path
        self.device = device_name
        self.version = version
        self.entries: dict = {}
        if os.path.exists(path):
            try:
                with open(path) as f:
                    d = json.load(f)
                if d.get("version") == version and d.get("device") == device_name:
                    self.entries = dict(d.get("entries", {}))
            except (OSError, ValueError):
                self.entries = {}

    def get(self, key: str):
        e = self.entries.get(key)
        return None if e is None else dict(e["options"])

    def put(self, key: str, options: dict, ms: float, default_ms: float) -> None:
        self.entries[key] = {"options": dict(options), "ms": ms, "default_ms": default_ms}

    def save(self) -> None:
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"version": self.version, "device": self.device, "entries": self.entries}, f, indent=1,
                      sort_keys=True)
        os.replace(tmp, self.path)


def _device_name(device: int) -> str:
    import torch

    p = torch.cuda.get_device_properties(device)
    return getattr(p, "gcnArchName", None) or p.name


def _make_inputs(op: str, h: int, w: int, seed: int):
    from . import synth

    if op == "recon":
        return synth.mr_inputs(h, w, seed=seed, n_disks=max(1, round(synth.MR_DISK_DENSITY * h * w)),
                               radius=(5, 20), offset=32)
    return synth.edt_input(h, w, seed=seed, coverage=0.3)


def _timed(fn, reps: int) -> float:
    import torch

    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def batch_pixels(jobs: list) -> int:
    """Pixels of a batch (the size of its "batch" bucket)."""
    n = 0
    for j in jobs:
        t = j["mask"] if j["op"] in ("recon", "erode") else j["binary"]
        n += t.numel()
    return n


def _job_outputs(jobs: list) -> list:
    return [t for j in jobs for t in ((j["out"],) if j["op"] in ("recon", "erode") else (j["sqdist"], j["nearest"]))]


def tune_jobs(ctx: Context, jobs: list, reps: int = 3) -> tuple:
    """Time every candidate of GRID["batch"] on ``ctx.run_batch(jobs)``.
    Returns (best options, best ms, default ms); raises if a candidate's
    outputs differ from the default options' outputs."""
    import torch

    saved = dict(ctx.options)
    outs = _job_outputs(jobs)
    fn = lambda: ctx.run_batch(jobs)
    try:
        ctx.set_options(**DEFAULTS)
        default_ms = _timed(fn, reps)
        ref = [o.clone() for o in outs]
        best, best_ms = dict(DEFAULTS), default_ms
        for cand in GRID["batch"]:
            opts = dict(DEFAULTS, **cand)
            ctx.set_options(**opts)
            ms = _timed(fn, reps)
            if not all(torch.equal(o, r) for o, r in zip(outs, ref)):
                raise RuntimeError(f"tuning candidate {opts} changed a batch result")
            if ms < best_ms:
                best, best_ms = opts, ms
        return best, best_ms, default_ms
    finally:
        ctx.set_options(**saved)


def _batch_sample(pixels: int, device) -> list:
    """Tiles of the mixed batch (synth.batch_tile_spec) in order until they
    hold at least `pixels` pixels, as device jobs with outputs."""
    import torch

    from . import synth

    jobs, n, i = [], 0, 0
    while n < pixels:
        spec = synth.batch_tile_spec(i)
        x = synth.tile_inputs(spec)
        h, w = spec["h"], spec["w"]
        if spec["op"] == "mr":
            jobs.append({"op": "recon", "conn": spec["conn"], "marker": torch.from_numpy(x[0]).to(device),
                         "mask": torch.from_numpy(x[1]).to(device),
                         "out": torch.empty((h, w), dtype=torch.uint8, device=device)})
        else:
            jobs.append({"op": "edt", "conn": spec["conn"], "binary": torch.from_numpy(x).to(device),
                         "sqdist": torch.empty((h, w), dtype=torch.int32, device=device),
                         "nearest": torch.empty((h, w), dtype=torch.int32, device=device)})
        n += h * w
        i += 1
    return jobs


def tune_bucket(ctx: Context, op: str, conn: int, key: str, reps: int = 3, seed: int = 0) -> tuple:
    """Time every candidate of GRID[op] on a synthetic image of bucket `key`.
    Returns (best options, best ms, default ms).  Raises if any candidate's
    output differs from the default options' output."""
    import torch

    dev = torch.device("cuda", ctx.device)
    if op == "batch":
        return tune_jobs(ctx, _batch_sample(1 << int(key.rsplit("2^", 1)[1]) - 1, dev), reps)
    h, w = bucket_side(key)
    saved = dict(ctx.options)
    x = _make_inputs(op, h, w, seed)
    if op == "recon":
        J, I = (torch.from_numpy(a).to(dev) for a in x)
        out = torch.empty_like(I)
        fn = lambda: ctx.morph_recon(J, I, conn, out=out)
        outs = [out]
    else:
        B = torch.from_numpy(x).to(dev)
        sq = torch.empty(B.shape, dtype=torch.int32, device=dev)
        nr = torch.empty_like(sq)
        fn = lambda: ctx.edt(B, conn, out=(sq, nr))
        outs = [sq, nr]
    try:
        ctx.set_options(**DEFAULTS)
        default_ms = _timed(fn, reps)
        ref = [o.clone() for o in outs]
        best, best_ms = dict(DEFAULTS), default_ms
        for cand in GRID[op]:
            opts = dict(DEFAULTS, **cand)
            ctx.set_options(**opts)
            ms = _timed(fn, reps)
            if not all(torch.equal(o, r) for o, r in zip(outs, ref)):
                raise RuntimeError(f"tuning candidate {opts} changed the result of {key}")
            if ms < best_ms:
                best, best_ms = opts, ms
        return best, best_ms, default_ms
    finally:
        ctx.set_options(**saved)


def autotune(buckets, device: int = 0, cache_path: str | None = None, reps: int = 3, force: bool = False) -> TuneCache:
    """Tune every (op, conn, pixels) of `buckets` that the cache lacks (all of
    them with `force`) and save the cache."""
    name = _device_name(device)
    cache = TuneCache(cache_path or default_cache_path(name), name, _lib.load().iwpp_version())
    ctx = Context(device)
    try:
        for op, conn, pixels in buckets:
            key = bucket(op, conn, pixels)
            if not force and cache.get(key) is not None:
                continue
            t = time.time()
            opts, ms, dms = tune_bucket(ctx, op, conn, key, reps)
            cache.put(key, opts, ms, dms)
            print(f"[tune] {key}: {opts} {ms:.3f} ms (default {dms:.3f} ms, {time.time() - t:.1f}s)", flush=True)
        cache.save()
    finally:
        ctx.close()
    return cache


class TunedContext(Context):
    """A Context that sets the cached options of each call's bucket before the
    call (the default options where the cache has no entry)."""

    def __init__(self, device: int = 0, cache: TuneCache | None = None, **kw):
        super().__init__(device, **kw)
        if cache is None:
            name = _device_name(device)
            cache = TuneCache(default_cache_path(name), name, self._lib.iwpp_version())
        self.cache = cache

    def _apply(self, op: str, conn: int, pixels: int) -> None:
        want = dict(DEFAULTS, **(self.cache.get(bucket(op, conn, pixels)) or {}))
        if any(self.options.get(k) != v for k, v in want.items()):
            self.set_options(**want)

    def morph_recon(self, marker, mask, conn: int = 8, out=None):
        self._apply("recon", conn, mask.numel())
        return super().morph_recon(marker, mask, conn, out)

    def edt(self, binary, conn: int = 8, out=None):
        self._apply("edt", conn, binary.numel())
        return super().edt(binary, conn, out)

    def morph_recon_erode(self, marker, mask, conn: int = 8, out=None):
        self._apply("recon", conn, mask.numel())
        return super().morph_recon_erode(marker, mask, conn, out)

    def run_batch(self, jobs: list) -> None:
        self._apply("batch", 0, batch_pixels(jobs))
        return super().run_batch(jobs)

    def batch_graph(self, jobs: list):
        # the options are read when the graph is captured
        self._apply("batch", 0, batch_pixels(jobs))
        return super().batch_graph(jobs)


def main(argv=None) -> int:
    """Tune buckets given as op:conn:pixels and write the cache, e.g.

        python -m paper_1209_3314_amd.tune --out paper_1209_3314_amd/tuned/gfx950.json --reps 5 \\
            recon:8:268435456 recon:4:268435456 edt:8:16777216
    """
    import argparse

    ap = argparse.ArgumentParser(description=main.__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("buckets", nargs="+", help="op:conn:pixels (op = recon, edt or batch)")
    ap.add_argument("--out", default=None, help="cache file (default: the per-user cache)")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    todo = []
    for b in args.buckets:
        op, conn, px = b.split(":")
        todo.append((op, int(conn), int(px)))
    autotune(todo, cache_path=args.out, reps=args.reps, force=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
