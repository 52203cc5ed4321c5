"""Serving loop: jobs with host buffers, admitted by memory budget, run in
continuous batches.  Each result is the same bytes alone (a plain call) and in
the mix, and equals the oracle; admission respects the budget; the plain
one-job-per-launch mode gives the same bytes."""
import time

import numpy as np
import pytest

import oracle
from paper_1209_3314_amd import _lib, synth
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, iw = require_gpu()
    ctx = iw.Context(0)
    yield torch, iw, ctx
    ctx.close()


def host_jobs(torch, rng, n, sizes=(1, 400)):
    jobs, ref = [], []
    for i in range(n):
        h, w = (int(v) for v in rng.integers(sizes[0], sizes[1], 2))
        conn = int(rng.choice([4, 8]))
        pin = lambda a: torch.from_numpy(a).pin_memory()
        if rng.random() < 0.7:
            J, I = synth.mr_inputs(h, w, seed=int(rng.integers(1 << 30)), n_disks=max(1, h * w // 8000),
                                   radius=(3, 12), offset=int(rng.integers(16, 65)))
            jobs.append({"op": "recon", "conn": conn, "marker": pin(J), "mask": pin(I),
                         "out": torch.empty((h, w), dtype=torch.uint8).pin_memory()})
            ref.append(("recon", conn, J, I))
        else:
            B = synth.edt_input(h, w, seed=int(rng.integers(1 << 30)), coverage=float(rng.uniform(0.05, 0.5)))
            jobs.append({"op": "edt", "conn": conn, "binary": pin(B),
                         "sqdist": torch.empty((h, w), dtype=torch.int32).pin_memory(),
                         "nearest": torch.empty((h, w), dtype=torch.int32).pin_memory()})
            ref.append(("edt", conn, B, None))
    return jobs, ref


def outputs(j):
    return [j["out"].numpy().copy()] if j["op"] == "recon" else [j["sqdist"].numpy().copy(), j["nearest"].numpy().copy()]


def alone(torch, ctx, j):
    """The same job as a plain single-image call on the device."""
    d = torch.device("cuda", 0)
    if j["op"] == "recon":
        return [ctx.morph_recon(j["marker"].to(d), j["mask"].to(d), j["conn"]).cpu().numpy()]
    s, n = ctx.edt(j["binary"].to(d), j["conn"])
    return [s.cpu().numpy(), n.cpu().numpy()]


def check_oracle(got, r):
    op, conn, a, b = r
    if op == "recon":
        assert np.array_equal(got[0], oracle.mr_fh(a, b, conn))
    else:
        s, n = oracle.edt_rounds(a, conn)
        assert np.array_equal(got[0], s) and np.array_equal(got[1], n)


def run_server(iw, ctx, jobs, stagger_s=0.0, **opts):
    srv = iw.Server(ctx, **opts)
    try:
        tickets = []
        for j in jobs:
            tickets.append(srv.submit(j))
            if stagger_s:
                time.sleep(stagger_s)
        srv.drain(timeout_ms=60000)
        states = [srv.poll(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.stop()
    assert all(s == _lib.JOB_DONE for s, _ in states), states
    assert all(lat >= 0 for _, lat in states)
    return st


@pytest.mark.parametrize("seed,n,max_batch", [(41, 30, 8), (42, 12, 0)])
def test_mix_equals_alone_and_oracle(env, seed, n, max_batch):
    torch, iw, ctx = env
    jobs, ref = host_jobs(torch, np.random.default_rng(seed), n)
    announce("serve mix", seed, n, max_batch)
    st = run_server(iw, ctx, jobs, hbm_budget_bytes=256 << 20, max_batch=max_batch)
    assert st["completed"] == n and st["failed"] == 0
    if max_batch:
        assert st["max_batch_jobs"] <= max_batch and st["batches"] >= (n + max_batch - 1) // max_batch
    mixed = [outputs(j) for j in jobs]
    for j, m, r in zip(jobs, mixed, ref):
        a = alone(torch, ctx, j)
        assert all(np.array_equal(x, y) for x, y in zip(m, a))
        check_oracle(m, r)


def test_staggered_arrivals(env):
    torch, iw, ctx = env
    jobs, ref = host_jobs(torch, np.random.default_rng(43), 24, sizes=(100, 500))
    announce("serve staggered")
    st = run_server(iw, ctx, jobs, stagger_s=0.002, hbm_budget_bytes=256 << 20)
    assert st["completed"] == 24
    for j, r in zip(jobs, ref):
        check_oracle(outputs(j), r)


def test_tight_budget_admission(env):
    torch, iw, ctx = env
    jobs, ref = host_jobs(torch, np.random.default_rng(44), 16, sizes=(300, 600))
    budget = 16 << 20
    announce("serve tight budget")
    st = run_server(iw, ctx, jobs, hbm_budget_bytes=budget, scratch_bytes=8 << 20, max_inflight=3)
    assert st["completed"] == 16 and st["peak_bytes"] <= budget
    assert st["batches"] >= 6  # at most 3 jobs admitted at a time
    for j, r in zip(jobs, ref):
        check_oracle(outputs(j), r)


def test_one_job_per_launch_mode(env):
    torch, iw, ctx = env
    jobs, ref = host_jobs(torch, np.random.default_rng(45), 10)
    announce("serve plain mode")
    st = run_server(iw, ctx, jobs, hbm_budget_bytes=128 << 20, max_batch=1)
    assert st["batches"] == 10 and st["max_batch_jobs"] == 1
    for j, r in zip(jobs, ref):
        check_oracle(outputs(j), r)


def test_busy_context_and_oversize_job(env):
    torch, iw, ctx = env
    srv = iw.Server(ctx, hbm_budget_bytes=16 << 20, scratch_bytes=4 << 20)
    try:
        d = torch.device("cuda", 0)
        a = torch.zeros((8, 8), dtype=torch.uint8, device=d)
        with pytest.raises(iw.IwppError):
            ctx.morph_recon(a, a.clone(), 8)
        big = torch.zeros((4096, 4096), dtype=torch.uint8)
        with pytest.raises(iw.IwppError):
            srv.submit({"op": "recon", "conn": 8, "marker": big, "mask": big.clone(), "out": big.clone()})
        with pytest.raises(ValueError):
            srv.submit({"op": "recon", "conn": 8, "marker": a, "mask": a, "out": a})  # device tensors
    finally:
        srv.stop()
    # usable again after stop
    a = torch.zeros((8, 8), dtype=torch.uint8, device=torch.device("cuda", 0))
    assert int(ctx.morph_recon(a, a.clone(), 8).sum()) == 0


def device_jobs(torch, rng, n, sizes=(1, 400)):
    """Jobs of a resident server: every job on device tensors of its own."""
    hjobs, ref = host_jobs(torch, rng, n, sizes)
    d = torch.device("cuda", 0)
    djobs = []
    for j in hjobs:
        djobs.append({k: (v.to(d) if hasattr(v, "to") else v) for k, v in j.items()})
    return djobs, ref


def dev_outputs(j):
    return [j["out"].cpu().numpy()] if j["op"] == "recon" else [j["sqdist"].cpu().numpy(), j["nearest"].cpu().numpy()]


@pytest.mark.parametrize("seed,n,max_batch", [(51, 30, 0), (52, 10, 1)])
def test_resident_mix_equals_alone_and_oracle(env, seed, n, max_batch):
    torch, iw, ctx = env
    jobs, ref = device_jobs(torch, np.random.default_rng(seed), n)
    announce("serve resident", seed, n, max_batch)
    srv = iw.Server(ctx, hbm_budget_bytes=256 << 20, max_batch=max_batch, resident=True)
    try:
        tickets = [srv.submit(j) for j in jobs]
        srv.drain(timeout_ms=60000)
        states = [srv.poll(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.stop()
    assert all(s == _lib.JOB_DONE for s, _ in states), states
    assert st["completed"] == n and st["failed"] == 0
    if max_batch == 1:
        assert st["batches"] == n
    torch.cuda.synchronize()
    for j, r in zip(jobs, ref):
        got = dev_outputs(j)
        check_oracle(got, r)
        a = alone(torch, ctx, j)
        assert all(np.array_equal(x, y) for x, y in zip(got, a))


def test_resident_rejects_host_buffers(env):
    torch, iw, ctx = env
    srv = iw.Server(ctx, hbm_budget_bytes=64 << 20, resident=True)
    try:
        h = torch.zeros((16, 16), dtype=torch.uint8).pin_memory()
        with pytest.raises(ValueError):
            srv.submit({"op": "recon", "conn": 8, "marker": h, "mask": h.clone(), "out": h.clone()})
        # the library's own check, below the binding: host pointers are refused
        m, o = h.clone().pin_memory(), h.clone().pin_memory()
        j = _lib.Job(_lib.IWPP_OP_RECON, 8, 16, 16, h.data_ptr(), m.data_ptr(), o.data_ptr(), None)
        import ctypes
        t = ctypes.c_uint64()
        assert srv._lib.iwpp_server_submit(srv._h, ctypes.byref(j), 0, None, ctypes.byref(t)) == _lib.IWPP_EINVAL
    finally:
        srv.stop()


def test_resident_job_waits_for_the_callers_stream(env):
    """Inputs written by kernels still queued on a side stream, and an output
    buffer that a queued kernel still writes, are submitted with no
    synchronisation: the job's batch waits for the side stream's work queued
    before the submit, so the result equals the oracle."""
    torch, iw, ctx = env
    d = torch.device("cuda", 0)
    h, w = 700, 900
    J, I = synth.mr_inputs(h, w, seed=61, n_disks=60, radius=(3, 12), offset=40)
    expect = oracle.mr_fh(J, I, 8)
    hJ, hI = torch.from_numpy(J).pin_memory(), torch.from_numpy(I).pin_memory()
    side = torch.cuda.Stream(d)
    srv = iw.Server(ctx, hbm_budget_bytes=256 << 20, resident=True)
    try:
        with torch.cuda.stream(side):
            big = torch.randn((6144, 6144), device=d)
            marker = torch.zeros((h, w), dtype=torch.uint8, device=d)
            mask = torch.zeros((h, w), dtype=torch.uint8, device=d)
            out = torch.empty((h, w), dtype=torch.uint8, device=d)
            for _ in range(8):  # keep the side stream busy well past the submit
                big = big @ big
                big = big / big.abs().max()
            marker.copy_(hJ, non_blocking=True)
            mask.copy_(hI, non_blocking=True)
            out.fill_(9)  # a queued writer of the output buffer
            announce("serve resident stream order")
            t = srv.submit({"op": "recon", "conn": 8, "marker": marker, "mask": mask, "out": out}, stream=side)
        srv.drain(timeout_ms=60000)
        state, _ = srv.poll(t)
    finally:
        srv.stop()
    assert state == _lib.JOB_DONE
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), expect)
