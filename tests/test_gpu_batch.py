"""Batched launches (many images, both operations, mixed sizes): every image's
result is bit-exact with the oracle and with its own single-image call."""
import numpy as np
import pytest

import oracle
from paper_1209_3314_amd import synth
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, iw = require_gpu()
    ctx = iw.Context(0)
    yield torch, iw, ctx
    ctx.close()


def make_jobs(torch, rng, n, sizes=(1, 300)):
    d = torch.device("cuda", 0)
    jobs, ref = [], []
    for i in range(n):
        h, w = (int(v) for v in rng.integers(sizes[0], sizes[1], 2))
        conn = int(rng.choice([4, 8]))
        if i % 2 == 0:
            J, I = synth.mr_inputs(h, w, seed=int(rng.integers(1 << 30)), n_disks=max(1, h * w // 8000),
                                   radius=(3, 12), offset=int(rng.integers(16, 65)))
            jobs.append({"op": "recon", "conn": conn, "marker": torch.from_numpy(J).to(d),
                         "mask": torch.from_numpy(I).to(d), "out": torch.empty((h, w), dtype=torch.uint8, device=d)})
            ref.append(("recon", conn, J, I))
        else:
            B = synth.edt_input(h, w, seed=int(rng.integers(1 << 30)), coverage=float(rng.uniform(0.05, 0.5)))
            jobs.append({"op": "edt", "conn": conn, "binary": torch.from_numpy(B).to(d),
                         "sqdist": torch.empty((h, w), dtype=torch.int32, device=d),
                         "nearest": torch.empty((h, w), dtype=torch.int32, device=d)})
            ref.append(("edt", conn, B, None))
    return jobs, ref


def check(jobs, ref):
    for j, (op, conn, a, b) in zip(jobs, ref):
        if op == "recon":
            assert np.array_equal(j["out"].cpu().numpy(), oracle.mr_fh(a, b, conn))
        else:
            s, n = oracle.edt_rounds(a, conn)
            assert np.array_equal(j["sqdist"].cpu().numpy(), s) and np.array_equal(j["nearest"].cpu().numpy(), n)


@pytest.mark.parametrize("seed,n", [(1, 2), (2, 9), (3, 24)])
def test_mixed_batch_matches_oracle(env, seed, n):
    torch, iw, ctx = env
    jobs, ref = make_jobs(torch, np.random.default_rng(seed), n)
    announce("batch", seed, n)
    ctx.run_batch(jobs)
    torch.cuda.synchronize()
    assert ctx.stats()["status"] == 0
    check(jobs, ref)


def test_batch_with_tiny_images_and_ragged_sizes(env):
    torch, iw, ctx = env
    jobs, ref = make_jobs(torch, np.random.default_rng(7), 16, sizes=(1, 70))
    announce("batch tiny")
    ctx.run_batch(jobs)
    torch.cuda.synchronize()
    check(jobs, ref)


def test_batch_with_forced_overflow(env):
    torch, iw, _ = env
    jobs, ref = make_jobs(torch, np.random.default_rng(11), 8, sizes=(100, 400))
    c = iw.Context(0, mr_list_capacity=3)
    try:
        announce("batch overflow")
        c.run_batch(jobs)
        torch.cuda.synchronize()
        assert c.stats()["overflow_restarts"] >= 1
    finally:
        c.close()
    check(jobs, ref)


def test_batch_rejects_overlapping_outputs(env):
    torch, iw, ctx = env
    d = torch.device("cuda", 0)
    I = torch.zeros((8, 8), dtype=torch.uint8, device=d)
    out = torch.empty_like(I)
    jobs = [{"op": "recon", "marker": I, "mask": I.clone(), "out": out},
            {"op": "recon", "marker": I.clone(), "mask": I.clone(), "out": out}]
    with pytest.raises(iw.IwppError):
        ctx.run_batch(jobs)
