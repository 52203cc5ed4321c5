"""Queue-design comparison on one GPU, after the paper's Table 1 (Sec. 5.2.1)
and its queue-overflow cost (Sec. 5.2.4).

Workload: reconstruction by dilation, 4-connected (as in Table 1), of a
4096 x 4096 tile built like the 16384 x 16384 workload (blurred noise plus
bright disks at the same density, radius 5-30, marker = mask - 48, seed 0).

Rows:
  * the pixel-queue reconstruction (iwpp_morph_recon_queue_u8) for each way
    of appending to a round's queue (one global atomic per item, one per wave
    with ballot offsets, LDS staging with one per flush) and each number of
    seed-pass sweep iterations (the analogue of Table 1's number of initial
    raster scans): device time, initial queue, queue pops, successful atomic
    raises, rounds;
  * the tile design (iwpp_morph_recon_u8) for the same sweep counts;
  * the overflow cost: the staged queue with capacities that force one and
    two rebuilds, and the tile design's bounded list likewise, against the
    unconstrained run.

Every output is compared with the unconstrained tile design's (all schedules
give rho_I(J), byte for byte).

    python -m paper_1209_3314_amd.ablation [--side 4096] [--reps 5] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _time(torch, fn, reps: int) -> float:
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


def run(side: int = 4096, reps: int = 5, sweeps=(1, 2, 4, 8), conn: int = 4) -> dict:
    import torch

    from . import Context, synth

    d = torch.device("cuda", 0)
    J, I = synth.mr_inputs(side, side, seed=0, n_disks=int(round(20000 * (side / 16384) ** 2)), radius=(5, 30),
                           offset=48)
    Jd, Id = torch.from_numpy(J).to(d), torch.from_numpy(I).to(d)
    out = torch.empty_like(Id)
    ctx = Context(0)
    rows = []
    try:
        ref = ctx.morph_recon(Jd, Id, conn).clone()
        torch.cuda.synchronize()

        def row(design, mode, s, ms, st, exact, **extra):
            r = {"design": design, "append": mode, "seed_sweeps": s, "ms": round(ms, 4), "exact": exact,
                 "initial_items": st["seeds"], "pops": st["items"], "atomic_raises": st["updates"],
                 "rounds": st["rounds"], "restarts": st["overflow_restarts"]}
            r.update(extra)
            rows.append(r)
            print(json.dumps(r), flush=True)

        for s in sweeps:
            ctx.set_options(mr_seed_sweeps=s)
            ms = _time(torch, lambda: ctx.morph_recon(Jd, Id, conn, out=out), reps)
            st = ctx.stats()
            row("tile", "-", s, ms, st, bool(torch.equal(out, ref)))
            for mode in ("naive", "ballot", "staged"):
                ms = _time(torch, lambda: ctx.morph_recon_queue(Jd, Id, conn, mode=mode, seed_sweeps=s, out=out), reps)
                st = ctx.stats()
                row("pixel queue", mode, s, ms, st, bool(torch.equal(out, ref)))
        ctx.set_options(mr_seed_sweeps=0)

        # Overflow cost: capacities below what the queues need, chosen from the
        # unconstrained run's initial queue, until one and two rebuilds occur.
        over = []
        ctx.morph_recon_queue(Jd, Id, conn, mode="staged", out=out)
        torch.cuda.synchronize()
        init = max(1, ctx.stats()["seeds"])
        base_ms = _time(torch, lambda: ctx.morph_recon_queue(Jd, Id, conn, mode="staged", out=out), reps)
        over.append({"design": "pixel queue", "capacity": 0, "restarts": 0, "ms": round(base_ms, 4), "ratio": 1.0})
        found = set()
        for f in (1.1, 1.0, 0.9, 0.75, 0.6, 0.5, 0.4, 0.3, 0.2):
            cap = int(init * f)
            ms = _time(torch, lambda: ctx.morph_recon_queue(Jd, Id, conn, mode="staged", capacity=cap, out=out), reps)
            st = ctx.stats()
            k = st["overflow_restarts"]
            if k in (1, 2) and k not in found:
                found.add(k)
                over.append({"design": "pixel queue", "capacity": cap, "capacity_over_initial": f, "restarts": k,
                             "ms": round(ms, 4), "ratio": round(ms / base_ms, 3), "exact": bool(torch.equal(out, ref))})
                print(json.dumps(over[-1]), flush=True)
            if found == {1, 2}:
                break
        tiles = ((side + 63) // 64) ** 2
        base_t = _time(torch, lambda: ctx.morph_recon(Jd, Id, conn, out=out), reps)
        over.append({"design": "tile", "capacity": 0, "restarts": 0, "ms": round(base_t, 4), "ratio": 1.0})
        found = set()
        for f in (0.999, 0.99, 0.97, 0.95, 0.9, 0.7, 0.5, 0.3, 0.2, 0.1, 0.05):
            cap = max(1, int(tiles * f))
            ctx.set_options(mr_list_capacity=cap)
            ms = _time(torch, lambda: ctx.morph_recon(Jd, Id, conn, out=out), reps)
            st = ctx.stats()
            k = st["overflow_restarts"]
            if k in (1, 2) and k not in found:
                found.add(k)
                over.append({"design": "tile", "capacity": cap, "capacity_over_tiles": f, "restarts": k,
                             "ms": round(ms, 4), "ratio": round(ms / base_t, 3), "exact": bool(torch.equal(out, ref))})
                print(json.dumps(over[-1]), flush=True)
            if found == {1, 2}:
                break
        ctx.set_options(mr_list_capacity=0)
    finally:
        torch.cuda.synchronize()
        ctx.close()
    return {"workload": f"reconstruction by dilation, {conn}-connected, {side}x{side} (blurred noise + disks, "
                        "offset 48, seed 0)", "rows": rows, "overflow": over}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--side", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--json", default=None, help="write the result here as JSON")
    args = ap.parse_args(argv)
    t = time.time()
    res = run(args.side, args.reps)
    res["seconds"] = round(time.time() - t, 1)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({"done": True, "seconds": res["seconds"]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
