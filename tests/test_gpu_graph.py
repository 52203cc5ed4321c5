"""Batches captured into a HIP graph: every replay is bit-exact with the oracle,
with eager library work and synchronisations between the replays, and a replay
after the inputs were rewritten in place computes the new inputs' results."""
import numpy as np
import pytest

from tests.gpu_util import announce, require_gpu
from tests.test_gpu_batch import check, make_jobs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, iw = require_gpu()
    ctx = iw.Context(0)
    yield torch, iw, ctx
    ctx.close()


def scramble(torch, jobs):
    for j in jobs:
        if j["op"] == "recon":
            j["out"].fill_(77)
        else:
            j["sqdist"].fill_(-5)
            j["nearest"].fill_(12345)


@pytest.mark.parametrize("seed,n", [(21, 1), (22, 12)])
def test_graph_replays_match_oracle(env, seed, n):
    torch, iw, ctx = env
    jobs, ref = make_jobs(torch, np.random.default_rng(seed), n, sizes=(1, 260))
    other, other_ref = make_jobs(torch, np.random.default_rng(seed + 100), 5, sizes=(20, 200))
    announce("graph create", seed, n)
    g = ctx.batch_graph(jobs)
    try:
        for rep in range(4):
            scramble(torch, jobs)
            torch.cuda.synchronize()
            announce("graph replay", seed, n, rep)
            g.launch()
            torch.cuda.synchronize()
            assert g.stats()["status"] == 0
            check(jobs, ref)
            # eager work of the same context between replays
            scramble(torch, other)
            ctx.run_batch(other)
            torch.cuda.synchronize()
            check(other, other_ref)
    finally:
        g.close()


def test_graph_reads_inputs_at_each_replay(env):
    torch, iw, ctx = env
    rng = np.random.default_rng(31)
    jobs, ref = make_jobs(torch, rng, 6, sizes=(40, 300))
    announce("graph new inputs")
    g = ctx.batch_graph(jobs)
    try:
        g.launch()
        torch.cuda.synchronize()
        check(jobs, ref)
        # rewrite every input in place with fresh images of the same shapes
        from paper_1209_3314_amd import synth

        new_ref = []
        for j, (op, conn, a, _) in zip(jobs, ref):
            h, w = a.shape
            if op == "recon":
                J, I = synth.mr_inputs(h, w, seed=int(rng.integers(1 << 30)), n_disks=4, radius=(3, 10), offset=40)
                j["marker"].copy_(torch.from_numpy(J))
                j["mask"].copy_(torch.from_numpy(I))
                new_ref.append((op, conn, J, I))
            else:
                B = synth.edt_input(h, w, seed=int(rng.integers(1 << 30)), coverage=0.2)
                j["binary"].copy_(torch.from_numpy(B))
                new_ref.append((op, conn, B, None))
        scramble(torch, jobs)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        check(jobs, new_ref)
    finally:
        g.close()


def test_graph_rejects_bad_batches(env):
    torch, iw, ctx = env
    d = torch.device("cuda", 0)
    a = torch.zeros((8, 8), dtype=torch.uint8, device=d)
    with pytest.raises(iw.IwppError):
        ctx.batch_graph([{"op": "recon", "conn": 8, "marker": a, "mask": a, "out": a}])


def test_graph_round_times(env):
    """The graph's own timeline: empty before a replay, one phase per grid
    barrier of its last persistent kernel after one."""
    torch, iw, ctx = env
    jobs, ref = make_jobs(torch, np.random.default_rng(41), 4, sizes=(100, 400))
    announce("graph round times")
    g = ctx.batch_graph(jobs)
    try:
        assert g.round_times() == []
        g.launch()
        torch.cuda.synchronize()
        check(jobs, ref)
        rt = g.round_times()
        assert len(rt) >= 1 and all(t >= 0.0 for t in rt)
    finally:
        g.close()
