"""Propagation EDT on the GPU, through the C ABI, against the oracle's round
semantics: squared distances and nearest-feature indices bit-exact."""
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


def run(env, B, conn, ctx=None):
    torch, iw, c = env
    c = ctx or c
    sq, nr = c.edt(torch.from_numpy(B).to(torch.device("cuda", 0)), conn)
    torch.cuda.synchronize()
    st = c.stats()
    assert st["status"] == 0, st
    return sq.cpu().numpy(), nr.cpu().numpy(), st


def check(env, B, conn, ctx=None):
    s, n, st = run(env, B, conn, ctx)
    so, no, ost = oracle.edt_rounds(B, conn, return_stats=True)
    assert np.array_equal(s, so) and np.array_equal(n, no)
    assert st["rounds"] == ost["rounds"] and st["items"] == ost["items"]
    return st


SHAPES = [(1, 1), (1, 300), (300, 1), (2, 2), (63, 65), (64, 64), (129, 257), (301, 199)]


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape", SHAPES)
def test_random_images(env, shape, conn):
    h, w = shape
    rng = np.random.default_rng(h * 7 + w + conn)
    for d in (0.003, 0.05, 0.5):
        B = (rng.random((h, w)) >= d).astype(np.uint8)
        announce("edt random", h, w, conn, d)
        check(env, B, conn)


@pytest.mark.parametrize("conn", [4, 8])
def test_generator_images(env, conn):
    for h, w, cov in [(256, 256, 0.1), (500, 333, 0.3), (129, 700, 0.5)]:
        B = synth.edt_input(h, w, seed=h + w, coverage=cov)
        announce("edt synth", h, w, conn, cov)
        check(env, B, conn)


def test_degenerate(env):
    for conn in (4, 8):
        announce("edt no feature", conn)
        s, n, _ = run(env, np.ones((40, 50), np.uint8), conn)
        assert (s == -1).all() and (n == -1).all()
        announce("edt all features", conn)
        s, n, _ = run(env, np.zeros((40, 50), np.uint8), conn)
        assert (s == 0).all() and np.array_equal(n, np.arange(2000).reshape(40, 50))
        B = np.ones((37, 41), np.uint8)
        B[36, 40] = 0
        announce("edt single corner feature", conn)
        check(env, B, conn)


def test_widest_allowed_row(env):
    B = np.ones((2, 32767), np.uint8)
    B[0, 0] = 0
    B[1, 32766] = 0
    announce("edt 2 x 32767")
    check(env, B, 8)


def test_first_wide_row(env):
    """Width 32768: the first size that takes the wide coordinate fields."""
    B = np.ones((2, 32768), np.uint8)
    B[0, 0] = 0
    B[1, 32767] = 0
    announce("edt 2 x 32768")
    check(env, B, 8)


def test_rejects_oversize(env):
    torch, iw, ctx = env
    announce("edt oversize")
    with pytest.raises(iw.IwppError):
        ctx.edt(torch.ones((1, 46341), dtype=torch.uint8, device="cuda"), 8)


@pytest.mark.parametrize("pb", [1, 3, 64])
def test_grid_size_does_not_change_bytes(env, pb):
    torch, iw, _ = env
    B = synth.edt_input(300, 400, seed=4, coverage=0.2)
    ctx = iw.Context(0, persistent_blocks=pb)
    try:
        announce("edt blocks", pb)
        check(env, B, 8, ctx)
    finally:
        ctx.close()


@pytest.mark.parametrize("conn,opts", [(8, dict(wg_waves=8)), (8, dict(stage_depth=1)), (4, dict(wg_waves=8, stage_depth=16))])
def test_launch_options_do_not_change_bytes(env, conn, opts):
    """Eight-wave workgroups and LDS stages of 1 and 16 items on a few hundred
    26x26 tiles with ragged edges."""
    torch, iw, _ = env
    B = synth.edt_input(700, 533, seed=12, coverage=0.25)
    ctx = iw.Context(0, **opts)
    try:
        announce("edt options", conn, opts)
        check(env, B, conn, ctx)
    finally:
        ctx.close()


def test_repeatable(env):
    B = synth.edt_input(600, 500, seed=8, coverage=0.3)
    announce("edt repeat")
    s0, n0, _ = run(env, B, 8)
    for _ in range(5):
        s, n, _ = run(env, B, 8)
        assert np.array_equal(s, s0) and np.array_equal(n, n0)


def test_4k_workload(env):
    """The 4096^2 nucleus-like workload in the benchmark's configuration,
    every pixel, plus the tolerance against the exact EDT."""
    B = synth.workload_edt_4k()
    announce("edt 4096^2")
    st = check(env, B, 8)
    s, _, _ = run(env, B, 8)
    ex = oracle.edt_exact_sep(B)
    assert float((s != ex).mean()) <= 1e-4
    assert float(np.abs(np.sqrt(s.astype(np.float64)) - np.sqrt(ex.astype(np.float64))).max()) <= 1.0
    assert st["seeds"] > 0


def test_4k_workload_conn4(env):
    """The same workload with 4-connected propagation, every pixel."""
    B = synth.workload_edt_4k()
    announce("edt 4096^2 conn 4")
    check(env, B, 4)


@pytest.mark.parametrize("conn", [4, 8])
def test_few_features_long_fronts(env, conn):
    """Three far-apart features: hundreds of rounds of thin fronts crossing
    tiles, where every step depends on the change records of the step before."""
    B = np.ones((900, 1100), np.uint8)
    for y, x in [(450, 0), (0, 1099), (899, 555)]:
        B[y, x] = 0
    announce("edt few features", conn)
    check(env, B, conn)
