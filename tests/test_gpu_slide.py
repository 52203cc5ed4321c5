"""Whole-slide images on one GPU (the paper's large-image setting, Sec. 4 and
Sec. 5.3): a reconstruction image beyond 2^32 pixels and distance transforms
wider than the 15-bit coordinate fields of the ordinary path, each bit-exact
with the oracle."""
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


@pytest.mark.timeout(900)
def test_mr_slide_beyond_2_32_pixels(env):
    """65536 x 65600 = 4,299,161,600 pixels (above 2^32), 8-connected; the
    flood crosses the pixel index 2^32 (row 65472) like every other row."""
    torch, iw, ctx = env
    h, w = 65536, 65600
    assert h * w > 2**32
    announce("slide mr generate", h, w)
    J, I = synth.slide_mr_inputs(h, w, seed=11)
    d = torch.device("cuda", 0)
    Id = torch.from_numpy(I).to(d)
    out = torch.from_numpy(J).to(d)  # in place: out aliases the marker
    announce("slide mr gpu", h, w)
    ctx.morph_recon(out, Id, 8, out=out)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["status"] == 0, st
    del Id
    got = out.cpu().numpy()
    del out
    torch.cuda.empty_cache()
    announce("slide mr oracle", h, w)
    ref = oracle.mr_fh(J, I, 8)
    assert np.array_equal(got, ref)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("h,w,cov,seed,conn", [
    (2048, 40000, 0.30, 3, 8),   # nucleus-like strip wider than 32767
    (40000, 512, 0.30, 4, 4),    # taller than 32767, 4-connected
    (300, 46000, 0.00002, 5, 8),  # few features: distances near the int32 limit
])
def test_edt_wide_strips(env, h, w, cov, seed, conn):
    torch, iw, ctx = env
    announce("slide edt generate", h, w, conn)
    B = synth.edt_input(h, w, seed=seed, coverage=cov)
    d = torch.device("cuda", 0)
    announce("slide edt gpu", h, w, conn)
    sq, nr = ctx.edt(torch.from_numpy(B).to(d), conn)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["status"] == 0, st
    announce("slide edt oracle", h, w, conn)
    so, no = oracle.edt_rounds(B, conn)
    assert np.array_equal(sq.cpu().numpy(), so)
    assert np.array_equal(nr.cpu().numpy(), no)


def test_edt_small_images_in_a_wide_group(env):
    """A batch whose EDT group holds one wide image runs every image of the
    group with the wide coordinate fields; the small ones must still equal the
    oracle."""
    torch, iw, ctx = env
    d = torch.device("cuda", 0)
    rng = np.random.default_rng(9)
    imgs = [synth.edt_input(64, 33000, seed=21, coverage=0.2)]
    imgs += [synth.edt_input(int(rng.integers(1, 300)), int(rng.integers(1, 300)), seed=30 + k, coverage=0.2)
             for k in range(6)]
    jobs = []
    for B in imgs:
        h, w = B.shape
        jobs.append({"op": "edt", "conn": 8, "binary": torch.from_numpy(B).to(d),
                     "sqdist": torch.empty((h, w), dtype=torch.int32, device=d),
                     "nearest": torch.empty((h, w), dtype=torch.int32, device=d)})
    announce("slide edt wide group")
    ctx.run_batch(jobs)
    torch.cuda.synchronize()
    assert ctx.stats()["status"] == 0
    for B, j in zip(imgs, jobs):
        so, no = oracle.edt_rounds(B, 8)
        assert np.array_equal(j["sqdist"].cpu().numpy(), so)
        assert np.array_equal(j["nearest"].cpu().numpy(), no)


def test_edt_rejects_sides_beyond_the_int32_distance_limit(env):
    torch, iw, ctx = env
    d = torch.device("cuda", 0)
    announce("slide edt limits")
    B = torch.ones((2, 46341), dtype=torch.uint8, device=d)  # a side above 46340
    with pytest.raises(iw.IwppError):
        ctx.edt(B, 8)
    B = torch.ones((33000, 33000), dtype=torch.uint8, device=d)  # 32999^2 * 2 > 2^31 - 1
    with pytest.raises(iw.IwppError):
        ctx.edt(B, 8)
