"""Autotuner host logic: size buckets, cache round trip and invalidation, and
(on the GPU) that tuned options never change results."""
import json

import numpy as np
import pytest

from paper_1209_3314_amd import tune


def test_bucket_keys():
    assert tune.bucket("recon", 8, 1) == "recon/8/2^12"
    assert tune.bucket("recon", 8, 4096) == "recon/8/2^12"
    assert tune.bucket("recon", 8, 4097) == "recon/8/2^13"
    assert tune.bucket("edt", 4, 4096 * 4096) == "edt/4/2^24"
    with pytest.raises(ValueError):
        tune.bucket("nope", 8, 10)


@pytest.mark.parametrize("k", [12, 13, 20, 25, 28])
def test_bucket_side_fills_bucket(k):
    h, w = tune.bucket_side(f"recon/8/2^{k}")
    assert h * w == 1 << k and abs(h - w) <= w
    assert tune.bucket("recon", 8, h * w) == f"recon/8/2^{k}"


def test_cache_round_trip_and_invalidation(tmp_path):
    p = str(tmp_path / "c" / "t.json")
    c = tune.TuneCache(p, "gfx950", 3)
    assert c.get("recon/8/2^20") is None
    c.put("recon/8/2^20", {"persistent_blocks": 256}, 1.0, 2.0)
    c.save()
    assert tune.TuneCache(p, "gfx950", 3).get("recon/8/2^20") == {"persistent_blocks": 256}
    assert tune.TuneCache(p, "gfx950", 4).get("recon/8/2^20") is None  # other library version
    assert tune.TuneCache(p, "gfx942", 3).get("recon/8/2^20") is None  # other device
    with open(p, "w") as f:
        f.write("{not json")
    assert tune.TuneCache(p, "gfx950", 3).entries == {}


def test_grid_uses_known_options():
    for cands in tune.GRID.values():
        for c in cands:
            assert set(c) <= set(tune.DEFAULTS)
            assert all(isinstance(v, int) and v >= 0 for v in c.values())


@pytest.mark.gpu
def test_tuning_never_changes_results(tmp_path):
    from tests.gpu_util import announce, require_gpu

    torch, iw = require_gpu()
    announce("autotune small buckets")
    cache = tune.autotune([("recon", 8, 300 * 300), ("recon", 4, 300 * 300), ("edt", 8, 300 * 300)],
                          cache_path=str(tmp_path / "t.json"), reps=1)
    assert len(cache.entries) == 3
    with open(tmp_path / "t.json") as f:
        assert len(json.load(f)["entries"]) == 3
    import oracle
    from paper_1209_3314_amd import synth

    ctx = tune.TunedContext(0, cache=cache)
    d = torch.device("cuda", 0)
    J, I = synth.mr_inputs(250, 333, seed=5, n_disks=8, radius=(5, 20), offset=32)
    got = ctx.morph_recon(torch.from_numpy(J).to(d), torch.from_numpy(I).to(d), 8)
    assert np.array_equal(got.cpu().numpy(), oracle.mr_fh(J, I, 8))
    B = synth.edt_input(260, 301, seed=6, coverage=0.3)
    s, n = ctx.edt(torch.from_numpy(B).to(d), 8)
    es, en = oracle.edt_rounds(B, 8)
    assert np.array_equal(s.cpu().numpy(), es) and np.array_equal(n.cpu().numpy(), en)
    ctx.close()


def test_batch_bucket_and_grid():
    assert tune.bucket("batch", 0, 1 << 20) == "batch/0/2^20"
    assert "batch" in tune.GRID and len(tune.GRID["batch"]) >= 8
    # every knob the survey names is tuned: workgroup size, LDS stage depth, seed tiling
    knobs = set().union(*[set(c) for c in tune.GRID["recon"]])
    assert {"wg_waves", "stage_depth", "mr_seed_strip"} <= knobs


@pytest.mark.gpu
def test_tuned_batch_never_changes_results(tmp_path):
    from tests.gpu_util import announce, require_gpu

    torch, iw = require_gpu()
    import oracle
    from paper_1209_3314_amd import synth

    announce("autotune batch bucket")
    pixels = 1 << 22
    cache = tune.autotune([("batch", 0, pixels)], cache_path=str(tmp_path / "t.json"), reps=1)
    key = tune.bucket("batch", 0, pixels)
    assert cache.get(key) is not None
    d = torch.device("cuda", 0)
    jobs = tune._batch_sample(pixels // 2, d)
    ctx = tune.TunedContext(0, cache=cache)
    cache.put(tune.bucket("batch", 0, tune.batch_pixels(jobs)), cache.get(key), 1.0, 1.0)
    ctx.run_batch(jobs)
    torch.cuda.synchronize()
    for i, j in enumerate(jobs):
        spec = synth.batch_tile_spec(i)
        x = synth.tile_inputs(spec)
        if j["op"] == "recon":
            assert np.array_equal(j["out"].cpu().numpy(), oracle.mr_fh(x[0], x[1], 8))
        else:
            s, n = oracle.edt_rounds(x, 8)
            assert np.array_equal(j["sqdist"].cpu().numpy(), s) and np.array_equal(j["nearest"].cpu().numpy(), n)
    g = ctx.batch_graph(jobs)
    g.launch()
    torch.cuda.synchronize()
    assert g.stats()["status"] == 0
    g.close()
    ctx.close()


def test_command_line_parses_buckets(monkeypatch, tmp_path):
    """`python -m paper_1209_3314_amd.tune op:conn:pixels ...` tunes exactly the
    named buckets into the given file (the tuning itself is stubbed: no GPU)."""
    seen = {}

    def fake_autotune(buckets, device=0, cache_path=None, reps=3, force=False):
        seen.update(buckets=list(buckets), cache_path=cache_path, reps=reps, force=force)

    monkeypatch.setattr(tune, "autotune", fake_autotune)
    out = str(tmp_path / "c.json")
    assert tune.main(["--out", out, "--reps", "5", "recon:8:268435456", "edt:8:16777216"]) == 0
    assert seen == {"buckets": [("recon", 8, 268435456), ("edt", 8, 16777216)], "cache_path": out, "reps": 5,
                    "force": True}


def test_committed_cache_names_known_options():
    """The cache the benchmark reads holds option sets the library accepts,
    keyed by buckets of the benchmark's sizes."""
    import os

    path = os.path.join(os.path.dirname(tune.__file__), "tuned", "gfx950.json")
    with open(path) as f:
        d = json.load(f)
    keys = {tune.bucket("recon", 8, 16384 * 16384), tune.bucket("recon", 4, 16384 * 16384),
            tune.bucket("edt", 8, 4096 * 4096)}
    assert keys <= set(d["entries"])
    for e in d["entries"].values():
        assert set(e["options"]) <= set(tune.DEFAULTS)
        assert e["ms"] <= e["default_ms"]
