"""The pixel-queue reconstruction (the paper's queue design, kept for the
queue-design comparison): bit-exact with the oracle for every append mode,
with forced queue overflows (drop, flag, rebuild from the partial result) and
with different numbers of seed-pass sweeps."""
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


def _run(env, J, I, conn, **kw):
    torch, iw, ctx = env
    d = torch.device("cuda", 0)
    out = ctx.morph_recon_queue(torch.from_numpy(J).to(d), torch.from_numpy(I).to(d), conn, **kw)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["status"] == 0, st
    return out.cpu().numpy(), st


@pytest.mark.parametrize("mode", ["naive", "ballot", "staged"])
@pytest.mark.parametrize("conn", [4, 8])
def test_queue_modes_match_oracle(env, mode, conn):
    J, I = synth.mr_inputs(700, 531, seed=50 + conn, n_disks=40, radius=(5, 20), offset=48)
    announce("queue", mode, conn)
    got, st = _run(env, J, I, conn, mode=mode)
    assert np.array_equal(got, oracle.mr_fh(J, I, conn))
    assert st["overflow_restarts"] == 0 and st["items"] > 0


@pytest.mark.parametrize("h,w", [(1, 1), (1, 300), (300, 1), (65, 63)])
def test_queue_degenerate_shapes(env, h, w):
    rng = np.random.default_rng(h * 1000 + w)
    I = rng.integers(0, 256, (h, w)).astype(np.uint8)
    J = rng.integers(0, 256, (h, w)).astype(np.uint8)
    announce("queue shape", h, w)
    got, _ = _run(env, J, I, 8, mode="ballot")
    assert np.array_equal(got, oracle.mr_fh(J, I, 8))


@pytest.mark.parametrize("cap", [1, 7, 500])
@pytest.mark.parametrize("mode", ["naive", "staged"])
def test_queue_overflow_restarts_are_exact(env, cap, mode):
    """A tiny queue drops most appends; every drop is recovered by rebuilding
    the queue from the partial result once the queues drain."""
    J, I = synth.mr_inputs(200, 230, seed=60, n_disks=6, radius=(5, 20), offset=48)
    announce("queue overflow", cap, mode)
    got, st = _run(env, J, I, 4, mode=mode, capacity=cap)
    assert np.array_equal(got, oracle.mr_fh(J, I, 4))
    assert st["overflow_restarts"] >= 1


@pytest.mark.parametrize("sweeps", [1, 2, 4])
def test_queue_seed_sweeps(env, sweeps):
    """More seed-pass sweeps leave fewer queue items; the result is the same."""
    J, I = synth.mr_inputs(512, 512, seed=0, n_disks=40, radius=(5, 20), offset=32)
    announce("queue seed sweeps", sweeps)
    got, st = _run(env, J, I, 4, mode="staged", seed_sweeps=sweeps)
    assert np.array_equal(got, oracle.mr_fh(J, I, 4))
