"""The seeded generators: deterministic bytes, shapes, and the recipe's
stated properties (marker = max(mask - offset, 0); EDT coverage reached)."""
import numpy as np

from paper_1209_3314_amd import synth


def test_mr_inputs_deterministic_and_recipe():
    J1, I1 = synth.mr_inputs(96, 80, seed=4, n_disks=5, radius=(5, 20), offset=32)
    J2, I2 = synth.mr_inputs(96, 80, seed=4, n_disks=5, radius=(5, 20), offset=32)
    assert J1.dtype == np.uint8 and I1.shape == (96, 80)
    assert np.array_equal(J1, J2) and np.array_equal(I1, I2)
    assert np.array_equal(J1, np.maximum(I1.astype(int) - 32, 0).astype(np.uint8))
    assert (I1 >= 200).any()  # disks painted
    J3, _ = synth.mr_inputs(96, 80, seed=5, n_disks=5)
    assert not np.array_equal(J1, J3)


def test_edt_input_coverage():
    for cov in (0.1, 0.3, 0.5):
        B = synth.edt_input(200, 150, seed=1, coverage=cov)
        assert B.dtype == np.uint8 and set(np.unique(B)) <= {0, 1}
        assert (B == 0).mean() >= cov
    assert np.array_equal(synth.edt_input(64, 64, 2), synth.edt_input(64, 64, 2))


def test_batch_specs():
    specs = [synth.batch_tile_spec(i) for i in range(256)]
    assert all(512 <= s["h"] <= 4096 and 512 <= s["w"] <= 4096 for s in specs)
    assert [s["op"] for s in specs[:4]] == ["mr", "edt", "mr", "edt"]
    assert specs[10] == synth.batch_tile_spec(10)


def test_serve_trace():
    tr = synth.serve_trace(200.0, 2.0, seed=0)
    assert 250 < len(tr) < 550
    times = [t for t, _ in tr]
    assert times == sorted(times)
    assert all(256 <= s["h"] <= 8192 for _, s in tr)


def test_serve_pool_and_arrivals():
    pool = synth.serve_pool(40, seed=1)
    assert sum(p["op"] == "mr" for p in pool) == 28
    assert all(256 <= p["h"] == p["w"] <= 8192 for p in pool)
    arr = synth.serve_arrivals(500.0, 2.0, 40, seed=1)
    assert 800 < len(arr) < 1200
    assert [t for t, _ in arr] == sorted(t for t, _ in arr)
    assert all(0 <= i < 40 for _, i in arr)
    assert arr == synth.serve_arrivals(500.0, 2.0, 40, seed=1)
