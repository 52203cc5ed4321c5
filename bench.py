#!/usr/bin/env python
"""Throughput benchmark of the IWPP hot path on one MI355X.

One step = the whole path over one batch of synthetic input, inputs already
resident in HBM:
  * grayscale reconstruction by dilation of the 16384 x 16384 whole-slide-tile
    workload, 8-connected and 4-connected (seed pass, seed detection,
    persistent propagation);
  * propagation EDT of the 4096 x 4096 nucleus-like workload, 8-connected
    (initialisation, rounds, finalisation).
`value` is pixels processed per second over the timed steps (Mpixel/s).

The roofline object describes the kernel that takes the most time per step:
its algorithmic bytes per launch (the paper's work model, with the oracle's
work counts) divided by its average launch time from HIP events recorded
around each launch on the benchmark's stream.  `traffic` is the measured HBM
traffic of that kernel from the committed rocprofv3 counter summary when it
was taken on the current kernel sources, else null.

The CPU baseline runs the oracle (single-threaded C) over one full step and
doubles as the bit-exactness check of the GPU outputs.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s morph-recon & EDT (bit-exact) + batched p50/p99 tile latency vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# Launch options per operation chosen by the library's autotuner on its own
# synthetic inputs of each size bucket (python -m paper_1209_3314_amd.tune);
# results never depend on them.
TUNED_FILE = os.path.join(ROOT, "paper_1209_3314_amd", "tuned", "gfx950.json")
# The paper's own end-to-end speedups (context only: other hardware, other
# images, several devices).
PAPER_CONTEXT = {
    "reconstruction": "50x over one CPU core, 96K x 96K image, 3 NVIDIA M2090 GPUs + 12 Xeon X5660 cores (Sec. 5.3)",
    "edt": "85.6x over one CPU core, 64K x 64K image, same machine (Sec. 5.3)",
}
CSRC = os.path.join(ROOT, "paper_1209_3314_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """Hash of the sources that decide what the measured step runs: every
    HIP source and header of the library except the serving loop's, which
    the step does not use."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")) and name != "iwpp_server.hip":
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(part: str, kernel: str, n: int, q_ref: int, conn: int) -> float:
    """Bytes the method itself moves, attributed to the kernel that does that
    part of the work.  Reconstruction (one persistent kernel whose round 0 is
    the seed pass): the raster and anti-raster passes read I and J and write J
    (6 B/px) and every queue item moves 10 + 2*conn bytes.  EDT:
    initialisation reads the input and writes the state (5 B/px); the rounds
    move 24 + 4*conn bytes per frontier item and the finalisation reads the
    state and writes two int32 maps (12 B/px)."""
    if part.startswith("mr"):
        if kernel == "mr_propagate":
            return 6.0 * n + float(10 + 2 * conn) * q_ref
        return 0.0
    if kernel == "edt_init":
        return 5.0 * n
    if kernel == "edt_rounds":
        return 12.0 * n + float(24 + 4 * conn) * q_ref
    return 0.0


def _gen_tile(i):
    from paper_1209_3314_amd import synth

    return synth.tile_inputs(synth.batch_tile_spec(i))


def _oracle_tile(args):
    import numpy as np

    import oracle

    spec, x, got = args
    if spec["op"] == "mr":
        return bool(np.array_equal(oracle.mr_fh(x[0], x[1], spec["conn"]), got[0]))
    s, n = oracle.edt_rounds(x, spec["conn"])
    return bool(np.array_equal(s, got[0]) and np.array_equal(n, got[1]))


SERVE_POOL = 512


def _gen_serve(i):
    from paper_1209_3314_amd import synth

    return synth.tile_inputs(synth.serve_pool(SERVE_POOL)[i])


def serve_leg(ctx, iw, torch, np, gen, rates, seconds: float, burst: int) -> dict:
    """Serving (iwpp_server_*): requests with host buffers (pinned), admitted
    by a 64 GiB device budget, continuous batching ("batched") against the
    same loop launching one job at a time ("plain").  Per rate: open-loop
    Poisson arrivals for `seconds`, each request one of a pool of SERVE_POOL
    tiles (square sides lognormal around 1024, clipped to [256, 8192], 70%
    reconstruction, 30% EDT, conn 8); latency = end of the output download
    minus the scheduled arrival.  Capacity: `burst` requests submitted at
    once, pixels over the time until the last completes.  Every output is
    compared with a plain single-image call of the same tile.  The capacity
    burst runs again on a resident server (inputs already in HBM, outputs
    per request on the device): the same loop without the PCIe copies."""
    from paper_1209_3314_amd import synth

    specs = synth.serve_pool(SERVE_POOL)
    host = gen.get()
    dev = torch.device("cuda", 0)
    jobs, ref, npx = [], [], []
    for spec, x in zip(specs, host):
        h, w = spec["h"], spec["w"]
        npx.append(h * w)
        if spec["op"] == "mr":
            j = {"op": "recon", "conn": spec["conn"], "marker": torch.from_numpy(x[0]).pin_memory(),
                 "mask": torch.from_numpy(x[1]).pin_memory(), "out": torch.empty((h, w), dtype=torch.uint8).pin_memory()}
            ref.append([ctx.morph_recon(j["marker"].to(dev), j["mask"].to(dev), j["conn"]).cpu()])
        else:
            j = {"op": "edt", "conn": spec["conn"], "binary": torch.from_numpy(x).pin_memory(),
                 "sqdist": torch.empty((h, w), dtype=torch.int32).pin_memory(),
                 "nearest": torch.empty((h, w), dtype=torch.int32).pin_memory()}
            sq, nr = ctx.edt(j["binary"].to(dev), j["conn"])
            ref.append([sq.cpu(), nr.cpu()])
        jobs.append(j)
    outs = lambda j: [j["out"]] if j["op"] == "recon" else [j["sqdist"], j["nearest"]]

    def clear():
        for j in jobs:
            for o in outs(j):
                o.fill_(-7 if o.dtype == torch.int32 else 7)

    def run(max_batch, arrivals):
        """Submit (time_s, index) on schedule; returns per-request latency (ms),
        makespan (s) and server statistics."""
        clear()
        with iw.Server(ctx, hbm_budget_bytes=64 << 30, max_batch=max_batch) as srv:
            for j in jobs[:8]:  # warm-up
                srv.submit(j)
            srv.drain(timeout_ms=120000)
            t0 = time.monotonic_ns() + 20_000_000
            tickets = []
            for t, idx in arrivals:
                at = t0 + int(t * 1e9)
                while True:
                    now = time.monotonic_ns()
                    if now >= at:
                        break
                    if at - now > 300_000:
                        time.sleep((at - now - 200_000) / 1e9)
                tickets.append((srv.submit(jobs[idx], arrival_ns=at), at))
            srv.drain(timeout_ms=600000)
            lat = np.array([srv.poll(tk)[1] for tk, _ in tickets])
            st = srv.stats()
        end = max(at + l * 1e6 for (_, at), l in zip(tickets, lat))
        used = sorted(set(i for _, i in arrivals))
        exact = all(torch.equal(o, r) for i in used for o, r in zip(outs(jobs[i]), ref[i]))
        return lat, (end - t0) / 1e9, st, exact

    def summary(arrivals, lat, span, st, exact):
        px = sum(npx[i] for _, i in arrivals)
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "req_s": round(len(arrivals) / span, 1),
                "mpix_s": round(px / span / 1e6, 1), "batches": st["batches"], "max_batch_jobs": st["max_batch_jobs"],
                "peak_gib": round(st["peak_bytes"] / 2**30, 2), "failed": st["failed"], "equal_to_plain_calls": exact}

    res = {"workload": f"{SERVE_POOL}-tile pool: square sides lognormal(median 1024, sigma 0.7) clipped [256, 8192], "
                       "70% reconstruction / 30% EDT, conn 8; Poisson arrivals; host buffers pinned; 64 GiB budget; "
                       "every request uploads its inputs to fresh device memory, so pool reuse gives no cache reuse",
           "pool_mpix": round(sum(npx) / 1e6, 1), "rates": []}
    # Each rate runs batched, plain, plain, batched (seconds / 2 each, two
    # arrival traces), so neither mode always runs first; a mode's figures pool
    # its two runs.
    for rate in rates:
        arrs = [synth.serve_arrivals(rate, seconds / 2, SERVE_POOL, seed=k) for k in (0, 1)]
        row = {"rate_req_s": rate, "seconds": seconds, "requests": sum(len(a) for a in arrs), "order": "ABBA"}
        got = {"batched": [], "plain": []}
        for mode, k in (("batched", 0), ("plain", 0), ("plain", 1), ("batched", 1)):
            got[mode].append((arrs[k], run(0 if mode == "batched" else 1, arrs[k])))
        for mode in ("batched", "plain"):
            (a0, (l0, s0, st0, e0)), (a1, (l1, s1, st1, e1)) = got[mode]
            st = {"batches": st0["batches"] + st1["batches"], "max_batch_jobs": max(st0["max_batch_jobs"], st1["max_batch_jobs"]),
                  "peak_bytes": max(st0["peak_bytes"], st1["peak_bytes"]), "failed": st0["failed"] + st1["failed"]}
            row[mode] = summary(a0 + a1, np.concatenate([l0, l1]), s0 + s1, st, e0 and e1)
            log(f"serve rate {rate} {mode}: {row[mode]}")
        row["p99_plain_over_batched"] = round(row["plain"]["p99_ms"] / max(row["batched"]["p99_ms"], 1e-9), 3)
        res["rates"].append(row)
    if burst:
        arr = [(0.0, i % SERVE_POOL) for i in range(burst)]
        cap = {"requests": burst}
        for mode, mb in (("batched", 0), ("plain", 1)):
            cap[mode] = summary(arr, *run(mb, arr))
            log(f"serve burst {mode}: {cap[mode]}")
        cap["throughput_batched_over_plain"] = round(cap["batched"]["mpix_s"] / max(cap["plain"]["mpix_s"], 1e-9), 3)
        # The host-buffer burst moves every input up and every output down
        # over PCIe: its bytes per second beside what plain pinned copies reach.
        up = sum(npx[i] * (2 if specs[i]["op"] == "mr" else 1) for _, i in arr)
        down = sum(npx[i] * (1 if specs[i]["op"] == "mr" else 8) for _, i in arr)
        span_b = sum(npx[i] for _, i in arr) / (cap["batched"]["mpix_s"] * 1e6)
        cap["pcie"] = {"bytes_up": up, "bytes_down": down, "batched_gb_s": round((up + down) / span_b / 1e9, 2),
                       "pinned_copy_gb_s": pinned_copy_rates(torch)}
        log(f"serve burst PCIe: {cap['pcie']}")
        res["capacity"] = cap
        # Device-resident serving: the pool's inputs uploaded once, every request with
        # device outputs of its own, no copies in the loop.
        dinp = []
        for j in jobs:
            if j["op"] == "recon":
                dinp.append({"op": "recon", "conn": j["conn"], "marker": j["marker"].to(dev), "mask": j["mask"].to(dev)})
            else:
                dinp.append({"op": "edt", "conn": j["conn"], "binary": j["binary"].to(dev)})

        def run_resident(max_batch):
            reqs = []
            for _, idx in arr:
                b = dinp[idx]
                if b["op"] == "recon":
                    reqs.append(dict(b, out=torch.empty_like(b["mask"])))
                else:
                    z = torch.empty(b["binary"].shape, dtype=torch.int32, device=dev)
                    reqs.append(dict(b, sqdist=z, nearest=torch.empty_like(z)))
            with iw.Server(ctx, hbm_budget_bytes=64 << 30, max_batch=max_batch, resident=True) as srv:
                for r in reqs[:8]:  # warm-up
                    srv.submit(r)
                srv.drain(timeout_ms=120000)
                torch.cuda.synchronize()
                t0 = time.monotonic_ns()
                tickets = [srv.submit(r, arrival_ns=t0) for r in reqs]
                srv.drain(timeout_ms=600000)
                lat = np.array([srv.poll(tk)[1] for tk in tickets])
                st = srv.stats()
            span = lat.max() / 1e3
            exact = all(torch.equal(o.cpu(), rr) for r, (_, idx) in zip(reqs, arr)
                        for o, rr in zip(outs(r), ref[idx]))
            return lat, span, st, exact

        rcap = {"requests": burst, "inputs": "device-resident (uploaded once), outputs per request on the device"}
        for mode, mb in (("batched", 0), ("plain", 1)):
            rcap[mode] = summary(arr, *run_resident(mb))
            log(f"serve resident burst {mode}: {rcap[mode]}")
        rcap["throughput_batched_over_plain"] = round(rcap["batched"]["mpix_s"] / max(rcap["plain"]["mpix_s"], 1e-9), 3)
        res["capacity_resident"] = rcap
    return res


def slide_leg(ctx, torch, np) -> dict:
    """A whole slide in one call: reconstruction by dilation, 8-connected, of
    a 65536 x 65600 image (4.3 G pixels, above 2^32), generated block-wise
    (32 x 32 blocks of uniform level plus row and column ripples; marker =
    mask - 40 except in 0.2% of the blocks).  Inputs resident in HBM; device
    time of one call after one warm-up.  Bit-exactness at this size is checked
    by the GPU tests against the oracle (about 100 s of CPU), not here."""
    from paper_1209_3314_amd import synth

    h, w = 65536, 65600
    t = time.time()
    J, I = synth.slide_mr_inputs(h, w, seed=11)
    gen_s = time.time() - t
    dev = torch.device("cuda", 0)
    Id = torch.from_numpy(I).to(dev)
    Jd = torch.from_numpy(J).to(dev)
    del J, I
    out = torch.empty_like(Id)
    ctx.morph_recon(Jd, Id, 8, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.morph_recon(Jd, Id, 8, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = ctx.stats()
    del Id, Jd, out
    torch.cuda.empty_cache()
    res = {"workload": f"reconstruction by dilation, conn 8, {h}x{w} whole slide (block field, seed 11)",
           "pixels": h * w, "ms": round(ms, 2), "mpix_s": round(h * w / (ms * 1e-3) / 1e6, 1),
           "status": st["status"], "rounds": st["rounds"], "tile_visits": st["items"],
           "input_generation_s": round(gen_s, 1)}
    log(f"slide: {res}")
    return res


def pinned_copy_rates(torch) -> dict:
    """Host<->device rates of plain 256 MiB copies from and to pinned memory,
    each direction alone and both at once (GB/s, best of 3)."""
    n = 256 << 20
    h1 = torch.empty(n, dtype=torch.uint8).pin_memory()
    h2 = torch.empty(n, dtype=torch.uint8).pin_memory()
    d1 = torch.empty(n, dtype=torch.uint8, device="cuda")
    d2 = torch.empty(n, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def best(fn):
        b = float("inf")
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            b = min(b, time.perf_counter() - t)
        return b

    up = best(lambda: d1.copy_(h1, non_blocking=True))
    down = best(lambda: h2.copy_(d2, non_blocking=True))

    def both():
        with torch.cuda.stream(s1):
            d1.copy_(h1, non_blocking=True)
        with torch.cuda.stream(s2):
            h2.copy_(d2, non_blocking=True)

    bi = best(both)
    return {"h2d": round(n / up / 1e9, 1), "d2h": round(n / down / 1e9, 1), "both": round(2 * n / bi / 1e9, 1)}


def pool_workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0)) - 1))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_child(conn, core: int, reps: int) -> None:
    """The CPU baseline: the oracle (single-threaded C) over one full step,
    pinned to one core, `reps` times.  Sends the run times, the work counts
    and digests of the outputs (the parent compares the GPU's outputs with
    them)."""
    import hashlib

    import numpy as np

    import oracle
    from paper_1209_3314_amd import synth

    try:
        os.sched_setaffinity(0, {core})
        Jm, Im = synth.workload_mr_16k()
        Be = synth.workload_edt_4k()
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            r8, s8 = oracle.mr_fh(Jm, Im, 8, return_stats=True)
            r4, s4 = oracle.mr_fh(Jm, Im, 4, return_stats=True)
            es, en, se = oracle.edt_rounds(Be, 8, return_stats=True)
            times.append(time.perf_counter() - t)
        dig = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
        conn.send({"times": times, "q_ref": {"mr16k_conn8": s8["pops"], "mr16k_conn4": s4["pops"],
                                             "edt4k_conn8": se["items"]},
                   "digests": [dig(r8), dig(r4), dig(es), dig(en)]})
    except Exception as e:  # reported by the parent
        conn.send({"error": repr(e)})
    conn.close()


def batch_leg(ctx, torch, np, pool, gen, ntiles: int, check: bool) -> dict:
    """The mixed batch of `ntiles` tiles (sides uniform in [512, 4096], even
    tiles reconstruction, odd tiles EDT, all 8-connected): one plain call per
    tile on one stream, against one batched call and against one replay of the
    batch captured as a HIP graph.  All tiles are submitted together at t = 0;
    a tile's latency is the time from t = 0 until its result is complete (plain:
    its call's end on the stream; batched: the end of the batch).  Inputs are
    resident in HBM; outputs of the three runs are compared with each other on
    the device and, with `check`, with the oracle (`pool`, forked before the
    process touched the GPU; `gen` is the pending generation of the tiles)."""
    from paper_1209_3314_amd import synth

    specs = [synth.batch_tile_spec(i) for i in range(ntiles)]
    t = time.time()
    host = gen.get()
    log(f"batch: tiles ready after {time.time() - t:.1f}s more")
    dev = torch.device("cuda", 0)
    jobs = []
    px = 0
    for spec, x in zip(specs, host):
        h, w = spec["h"], spec["w"]
        px += h * w
        if spec["op"] == "mr":
            jobs.append({"op": "recon", "conn": spec["conn"], "marker": torch.from_numpy(x[0]).to(dev),
                         "mask": torch.from_numpy(x[1]).to(dev),
                         "out": torch.empty((h, w), dtype=torch.uint8, device=dev)})
        else:
            jobs.append({"op": "edt", "conn": spec["conn"], "binary": torch.from_numpy(x).to(dev),
                         "sqdist": torch.empty((h, w), dtype=torch.int32, device=dev),
                         "nearest": torch.empty((h, w), dtype=torch.int32, device=dev)})
    outs = lambda j: [j["out"]] if j["op"] == "recon" else [j["sqdist"], j["nearest"]]

    def plain():
        for j in jobs:
            if j["op"] == "recon":
                ctx.morph_recon(j["marker"], j["mask"], j["conn"], out=j["out"])
            else:
                ctx.edt(j["binary"], j["conn"], out=(j["sqdist"], j["nearest"]))

    # warm up each form once
    plain()
    ctx.run_batch(jobs)
    g = ctx.batch_graph(jobs)
    g.launch()
    torch.cuda.synchronize()
    ctx.profile_read()

    # plain: an event after every tile gives each tile's completion time
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(ntiles + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i, j in enumerate(jobs):
        if j["op"] == "recon":
            ctx.morph_recon(j["marker"], j["mask"], j["conn"], out=j["out"])
        else:
            ctx.edt(j["binary"], j["conn"], out=(j["sqdist"], j["nearest"]))
        ev[i + 1].record()
    torch.cuda.synchronize()
    done_plain = np.array([ev[0].elapsed_time(e) for e in ev[1:]])
    ref = [[o.clone() for o in outs(j)] for j in jobs]

    def timed(fn):
        for j in jobs:
            for o in outs(j):
                o.fill_(-3 if o.dtype == torch.int32 else 3)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        same = all(torch.equal(o, r) for j, rr in zip(jobs, ref) for o, r in zip(outs(j), rr))
        return a.elapsed_time(b), same

    batch_ms, batch_same = timed(lambda: ctx.run_batch(jobs))
    bstats = ctx.stats()
    graph_ms, graph_same = timed(lambda: g.launch())
    gstats = g.stats()
    g.close()
    ctx.profile_read()
    # Tuned: the autotuner's batch grid on this batch (tune_jobs checks every
    # candidate's outputs against the default options' outputs), then the
    # batch and a graph captured under the chosen options.
    from paper_1209_3314_amd import tune

    t = time.time()
    saved = dict(ctx.options)
    best, _, _ = tune.tune_jobs(ctx, jobs, reps=2)
    tune_s = time.time() - t
    ctx.set_options(**best)
    tbatch_ms, tbatch_same = timed(lambda: ctx.run_batch(jobs))
    gt = ctx.batch_graph(jobs)
    gt.launch()
    torch.cuda.synchronize()
    tgraph_ms, tgraph_same = timed(lambda: gt.launch())
    tgstats = gt.stats()
    gt.close()
    ctx.set_options(**saved)
    ctx.profile_read()
    plain_ms = float(done_plain[-1])
    res = {
        "tiles": ntiles, "pixels": px, "workload": "256-tile mixed batch: sides U[512,4096], even tiles reconstruction "
        "(disk density of the 512^2 workload, offset U[16,64]), odd tiles EDT (coverage U[0.1,0.5]), conn 8, seeds 1000+i",
        "plain_ms": round(plain_ms, 3), "batch_ms": round(batch_ms, 3), "graph_ms": round(graph_ms, 3),
        "plain_mpix_s": round(px / plain_ms / 1e3, 1), "batch_mpix_s": round(px / batch_ms / 1e3, 1),
        "graph_mpix_s": round(px / graph_ms / 1e3, 1),
        "speedup_batch": round(plain_ms / batch_ms, 3), "speedup_graph": round(plain_ms / graph_ms, 3),
        "latency_ms": {"plain_p50": round(float(np.percentile(done_plain, 50)), 3),
                       "plain_p99": round(float(np.percentile(done_plain, 99)), 3),
                       "batch_p50": round(batch_ms, 3), "batch_p99": round(batch_ms, 3),
                       "graph_p50": round(graph_ms, 3), "graph_p99": round(graph_ms, 3)},
        "plain_tile_ms": {"p50": round(float(np.percentile(np.diff(done_plain, prepend=0.0), 50)), 3),
                          "p99": round(float(np.percentile(np.diff(done_plain, prepend=0.0), 99)), 3)},
        "batch_equals_plain": bool(batch_same), "graph_equals_plain": bool(graph_same),
        "batch_status": bstats["status"], "graph_status": gstats["status"],
        "tuned": {"options": {k: v for k, v in best.items() if v}, "tuning_s": round(tune_s, 1),
                  "batch_ms": round(tbatch_ms, 3), "graph_ms": round(tgraph_ms, 3),
                  "speedup_batch": round(plain_ms / tbatch_ms, 3), "speedup_graph": round(plain_ms / tgraph_ms, 3),
                  "batch_equals_plain": bool(tbatch_same), "graph_equals_plain": bool(tgraph_same),
                  "graph_status": tgstats["status"]},
        "bit_exact": None, "cpu_baseline": None,
    }
    if check:
        got = [[r.cpu().numpy() for r in rr] for rr in ref]
        nw = pool_workers()
        t = time.perf_counter()
        ok = pool.map(_oracle_tile, list(zip(specs, host, got)), chunksize=1)
        cpu_s = time.perf_counter() - t
        res["bit_exact"] = bool(all(ok))
        res["cpu_baseline"] = {"value": round(px / cpu_s / 1e6, 2), "unit": "Mpixel/s", "cores": nw, "kind": "oracle",
                               "sample": f"all {ntiles} tiles, oracle in a pool of {nw} processes ({cpu_s:.1f} s)"}
    log(f"batch: {res}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle run (then no bit-exactness check and no work counts)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-tile batched leg")
    ap.add_argument("--batch-tiles", type=int, default=256, help="tiles in the batched leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-slide", action="store_true", help="skip the whole-slide reconstruction leg")
    ap.add_argument("--options", choices=("tuned", "default"), default="tuned",
                    help="launch options of the step: the autotuner's per-operation choice or the library defaults")
    ap.add_argument("--serve-rates", default="200,800,2000", help="comma-separated request rates (per second)")
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="trace length per rate")
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle runs of the CPU baseline (median reported)")
    ap.add_argument("--serve-burst", type=int, default=256, help="requests of the capacity burst (0 = none)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (reference for rocprofv3 byte counters)")
    ap.add_argument("--copy-first", action="store_true",
                    help="run the 1 GiB reference copy 3 times before the workload (same process, for counter runs)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        a = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": 1 << 30, "bytes_written_per_launch": 1 << 30,
                          "launches": 3}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (independent tiles would "
              "shard one per GPU, one image in horizontal bands). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    # The CPU baseline runs in a child pinned to one core (the paper's
    # single-core baseline, median of 3 runs); this process and the tile
    # generators keep off that core.  Forked before the GPU is initialised.
    oracle_rx = oracle_proc = None
    cores = sorted(os.sched_getaffinity(0))
    if not args.no_cpu_baseline:
        from multiprocessing import Pipe, get_context

        oracle_rx, tx = Pipe(duplex=False)
        oracle_proc = get_context("fork").Process(target=_oracle_child, args=(tx, cores[0], args.cpu_reps))
        oracle_proc.start()
        tx.close()
        if len(cores) > 1:
            os.sched_setaffinity(0, set(cores[1:]))
    pool = gen = None
    if not args.no_batch:
        # Workers are forked before this process initialises the GPU; the batch
        # tiles are generated while the single-image part runs.
        from multiprocessing import get_context

        pool = get_context("fork").Pool(pool_workers())
        gen = pool.map_async(_gen_tile, range(args.batch_tiles), chunksize=1)
    serve_gen = None
    if not args.no_serve:
        from multiprocessing import get_context

        if pool is None:
            pool = get_context("fork").Pool(pool_workers())
        serve_gen = pool.map_async(_gen_serve, range(SERVE_POOL), chunksize=1)

    import numpy as np
    import torch

    import paper_1209_3314_amd as iw
    from paper_1209_3314_amd import synth

    dev = torch.device("cuda", 0)
    if args.copy_first:
        ca = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        cb = torch.empty_like(ca)
        for _ in range(3):
            cb.copy_(ca)
        torch.cuda.synchronize()
        del ca, cb
        log("reference copy: 3 x 1 GiB device-to-device")
    t = time.time()
    Jm, Im = synth.workload_mr_16k()
    Be = synth.workload_edt_4k()
    log(f"generated inputs in {time.time() - t:.1f}s")
    n_mr, n_edt = Jm.size, Be.size
    Jd, Id, Bd = torch.from_numpy(Jm).to(dev), torch.from_numpy(Im).to(dev), torch.from_numpy(Be).to(dev)
    o8, o4 = torch.empty_like(Id), torch.empty_like(Id)
    sq = torch.empty(Be.shape, dtype=torch.int32, device=dev)
    nr = torch.empty(Be.shape, dtype=torch.int32, device=dev)
    ctx = iw.Context(0, profile=True)
    parts = [("mr16k_conn8", 8), ("mr16k_conn4", 4), ("edt4k_conn8", 8)]
    # Options per part: the autotuner's choice for the part's size bucket, or
    # the library defaults (--options default).
    from paper_1209_3314_amd import tune

    opts = {name: dict(tune.DEFAULTS) for name, _ in parts}
    if args.options == "tuned":
        cache = tune.TuneCache(TUNED_FILE, tune._device_name(0), ctx._lib.iwpp_version())
        for name, conn in parts:
            op, npx = ("recon", n_mr) if name.startswith("mr") else ("edt", n_edt)
            opts[name].update(cache.get(tune.bucket(op, conn, npx)) or {})
    used = {name: {k: v for k, v in o.items() if v != tune.DEFAULTS[k]} for name, o in opts.items()}
    log(f"launch options per part ({args.options}): {used}")

    def call(name, conn):
        ctx.set_options(**opts[name])
        if name.startswith("mr"):
            ctx.morph_recon(Jd, Id, conn, out=o8 if conn == 8 else o4)
        else:
            ctx.edt(Bd, conn, out=(sq, nr))

    def step():
        for name, conn in parts:
            call(name, conn)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    gpu_stats = {}
    for name, conn in parts:  # counters of one call each (not timed)
        call(name, conn)
        gpu_stats[name] = ctx.stats()
        assert gpu_stats[name]["status"] == 0, gpu_stats[name]
    ctx.profile_read()  # drop the warm-up records

    # ---- timed region ----
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - w0) * 1e3
    dev_ms = e0.elapsed_time(e1)
    ms_per_step = dev_ms / args.steps
    records = ctx.profile_read()

    # Per-kernel averages, by part of the step (launch order within a step).
    per_call = []
    for name, conn in parts:
        names = ["reset", "mr_propagate"] if name.startswith("mr") else ["reset", "edt_init", "edt_rounds"]
        per_call.append((name, conn, names))
    launches_per_step = sum(len(c[2]) for c in per_call)
    assert len(records) == launches_per_step * args.steps, (len(records), launches_per_step)
    kern_ms = {}
    i = 0
    for _ in range(args.steps):
        for name, conn, names in per_call:
            for kn in names:
                rk, ms = records[i]
                assert rk == kn, (rk, kn)
                kern_ms.setdefault((name, kn), []).append(ms)
                i += 1
    kernels = {f"{p}/{k}": sum(v) / len(v) for (p, k), v in kern_ms.items()}

    # ---- oracle: CPU baseline + bit-exactness + work counts ----
    q_ref, cpu = {}, None
    bit_exact = None
    edt_vs_exact = None
    if not args.no_cpu_baseline:
        import hashlib

        import oracle

        g8, g4 = o8.cpu().numpy(), o4.cpu().numpy()
        gs, gn = sq.cpu().numpy(), nr.cpu().numpy()
        res = oracle_rx.recv()
        oracle_proc.join()
        if "error" in res:
            raise RuntimeError(f"oracle child failed: {res['error']}")
        dig = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
        bit_exact = [dig(g8), dig(g4), dig(gs), dig(gn)] == res["digests"]
        q_ref = res["q_ref"]
        cpu_s = float(np.median(res["times"]))
        cpu = {"value": round((2 * n_mr + n_edt) / cpu_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
               "sample": "one full step (16384^2 reconstruction conn 8 and conn 4, 4096^2 EDT conn 8), "
                         f"median of {len(res['times'])} runs pinned to one core: {cpu_s:.1f} s single-threaded C",
               "runs_s": [round(x, 2) for x in res["times"]], "cpu_model": cpu_model(),
               "host_cores_allowed": len(cores), "host_cpu_count": os.cpu_count()}
        log(f"oracle step median {cpu_s:.1f}s bit_exact={bit_exact} q_ref={q_ref}")
        # The propagation EDT against the exact EDT, on the timed output.
        ex = oracle.edt_exact_sep(Be)
        diff = gs.astype(np.int64) != ex
        err = np.abs(np.sqrt(gs.astype(np.float64)) - np.sqrt(ex.astype(np.float64)))
        edt_vs_exact = {"pixels_differing": int(diff.sum()), "fraction": float(diff.mean()),
                        "max_distance_error_px": float(err.max()), "tolerance": {"fraction": 1e-4, "max_px": 1.0}}
        log(f"EDT vs exact: {edt_vs_exact}")

    # ---- roofline of the dominant kernel ----
    dom_key = max(kernels, key=kernels.get)
    dom_part, dom_kernel = dom_key.split("/")
    dom_conn = dict(parts)[dom_part]
    dom_n = n_edt if dom_part.startswith("edt") else n_mr
    roofline = None
    op_roofline = {}
    if q_ref:
        ab = algorithmic_bytes(dom_part, dom_kernel, dom_n, q_ref[dom_part], dom_conn)
        achieved = ab / (kernels[dom_key] * 1e-3) / 1e9
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            with open(TRAFFIC_FILE) as f:
                tr = json.load(f)
            ent = tr.get("kernels", {}).get(dom_key)
            if ent and tr.get("kernel_source_sha") == kernel_source_sha():
                traffic = ent["hbm_bytes_per_launch"]
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom_key,
                    "algorithmic_bytes": ab, "avg_ms": round(kernels[dom_key], 4)}
        for name, conn in parts:
            n = n_edt if name.startswith("edt") else n_mr
            ks = [k for k in kernels if k.startswith(name + "/")]
            ms = sum(kernels[k] for k in ks)
            b = sum(algorithmic_bytes(name, k.split("/")[1], n, q_ref[name], conn) for k in ks)
            op_roofline[name] = {"ms": round(ms, 4), "algorithmic_GB": round(b / 1e9, 4),
                                 "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "mpix_s": round(n / (ms * 1e-3) / 1e6, 1)}

    ctx.set_options(**tune.DEFAULTS)  # the other legs run with the defaults (the batch leg tunes its own)
    slide = None
    if not args.no_slide:
        slide = slide_leg(ctx, torch, np)
    batch = None
    if not args.no_batch:
        batch = batch_leg(ctx, torch, np, pool, gen, args.batch_tiles, check=not args.no_cpu_baseline)
    serve = None
    if not args.no_serve:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        serve = serve_leg(ctx, iw, torch, np, serve_gen, rates, args.serve_seconds, args.serve_burst)
    if pool is not None:
        pool.close()
        pool.join()
    # Release the library's device memory and event records before the
    # interpreter tears the process down.
    torch.cuda.synchronize()
    ctx.close()

    px = 2 * n_mr + n_edt
    value = px / (ms_per_step * 1e-3) / 1e6
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8/int32", "data": "synthetic",
        "config": {"workload": "morph-recon 16384x16384 uint8 conn 8 + conn 4 (20k disks r5-30, offset 48, seed 0) "
                               "+ EDT 4096x4096 conn 8 (30% nucleus-like features, seed 0)",
                   "pixels_per_step": px},
        "bit_exact": bit_exact, "roofline": roofline, "cpu_baseline": cpu,
        "per_op": op_roofline, "kernels_ms": {k: round(v, 4) for k, v in kernels.items()},
        "wall_ms_per_step": round(wall_ms / args.steps, 4),
        "work": {"q_ref": q_ref, "gpu": gpu_stats},
        "launch_options": {"mode": args.options, "per_part": used,
                           "source": "autotuner cache paper_1209_3314_amd/tuned/gfx950.json" if args.options == "tuned"
                           else "library defaults"},
        "edt_vs_exact": edt_vs_exact,
        "paper_context": PAPER_CONTEXT,
        "batch": batch,
        "slide": slide,
        "serve": serve,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
