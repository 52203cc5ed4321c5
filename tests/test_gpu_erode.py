"""Reconstruction by erosion on the GPU (the dilation kernels on complemented
bytes), bit-exact against the oracle's erosion (pinned to its own
definition, the threshold decomposition and the duality identity)."""
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


def erode_inputs(h, w, seed, offset=40):
    """Dark nuclei on a blurred background (the reconstruction workload
    complemented) with the marker above the mask."""
    Jd, Id = synth.mr_inputs(h, w, seed=seed, n_disks=max(2, h * w // 6500), radius=(5, 20), offset=offset)
    return (255 - Jd).astype(np.uint8), (255 - Id).astype(np.uint8)


@pytest.mark.parametrize("h,w,conn,seed", [(1, 1, 8, 1), (1, 333, 4, 2), (257, 1, 8, 3), (63, 65, 8, 4),
                                           (300, 257, 4, 5), (513, 770, 8, 6), (1000, 1000, 4, 7)])
def test_erode_matches_oracle(env, h, w, conn, seed):
    torch, iw, ctx = env
    J, I = erode_inputs(h, w, seed)
    d = torch.device("cuda", 0)
    announce("erode", h, w, conn)
    got = ctx.morph_recon_erode(torch.from_numpy(J).to(d), torch.from_numpy(I).to(d), conn)
    torch.cuda.synchronize()
    assert ctx.stats()["status"] == 0
    assert np.array_equal(got.cpu().numpy(), oracle.mr_erode(J, I, conn))


def test_erode_marker_below_mask_and_in_place(env):
    """A marker below the mask is raised to it first; out may alias the marker."""
    torch, iw, ctx = env
    rng = np.random.default_rng(8)
    I = rng.integers(0, 256, (200, 300)).astype(np.uint8)
    J = rng.integers(0, 256, (200, 300)).astype(np.uint8)  # above and below the mask
    d = torch.device("cuda", 0)
    Jd = torch.from_numpy(J).to(d)
    announce("erode in place")
    ctx.morph_recon_erode(Jd, torch.from_numpy(I).to(d), 8, out=Jd)
    torch.cuda.synchronize()
    assert np.array_equal(Jd.cpu().numpy(), oracle.mr_erode(J, I, 8))


def test_erode_and_dilate_in_one_batch(env):
    """Erosion and dilation jobs of one connectivity share the launches of
    one group; every result equals its oracle."""
    torch, iw, ctx = env
    d = torch.device("cuda", 0)
    jobs, want = [], []
    for k in range(6):
        h, w = 150 + 97 * k, 400 - 41 * k
        if k % 2:
            J, I = erode_inputs(h, w, 30 + k)
            jobs.append({"op": "erode", "conn": 8, "marker": torch.from_numpy(J).to(d),
                         "mask": torch.from_numpy(I).to(d), "out": torch.empty((h, w), dtype=torch.uint8, device=d)})
            want.append(oracle.mr_erode(J, I, 8))
        else:
            J, I = synth.mr_inputs(h, w, seed=30 + k, n_disks=8, radius=(5, 20), offset=32)
            jobs.append({"op": "recon", "conn": 8, "marker": torch.from_numpy(J).to(d),
                         "mask": torch.from_numpy(I).to(d), "out": torch.empty((h, w), dtype=torch.uint8, device=d)})
            want.append(oracle.mr_fh(J, I, 8))
    announce("erode + dilate batch")
    ctx.run_batch(jobs)
    torch.cuda.synchronize()
    assert ctx.stats()["status"] == 0
    for j, r in zip(jobs, want):
        assert np.array_equal(j["out"].cpu().numpy(), r)


@pytest.mark.timeout(300)
def test_erode_whole_slide_tile(env):
    """16384 x 16384, 4-connected: the complemented reconstruction workload."""
    torch, iw, ctx = env
    Jd, Id = synth.workload_mr_16k()
    J, I = (255 - Jd).astype(np.uint8), (255 - Id).astype(np.uint8)
    d = torch.device("cuda", 0)
    announce("erode 16384^2 conn 4")
    got = ctx.morph_recon_erode(torch.from_numpy(J).to(d), torch.from_numpy(I).to(d), 4)
    torch.cuda.synchronize()
    assert ctx.stats()["status"] == 0
    assert np.array_equal(got.cpu().numpy(), oracle.mr_erode(J, I, 4))


def test_erode_served(env):
    """Erosion jobs through the serving loop equal the single-image call."""
    torch, iw, ctx = env
    J, I = erode_inputs(700, 500, 40)
    out = torch.empty((700, 500), dtype=torch.uint8).pin_memory()
    announce("erode served")
    with iw.Server(ctx, hbm_budget_bytes=1 << 30) as srv:
        t = srv.submit({"op": "erode", "conn": 8, "marker": torch.from_numpy(J).pin_memory(),
                        "mask": torch.from_numpy(I).pin_memory(), "out": out})
        srv.drain(timeout_ms=60000)
        assert srv.poll(t)[0] == 3  # done
    assert np.array_equal(out.numpy(), oracle.mr_erode(J, I, 8))
