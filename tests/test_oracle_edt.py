"""Pins for the distance-transform oracle (Sec. 2.2).

The round (level-synchronous) reading of Algorithms 3/6 is computed twice --
frontier form and dense Jacobi form, written independently -- and the two must
agree bit for bit.  Both are pinned from outside: exact results where the
propagation is provably exact (one row or column, a single feature, whose
round count is the Chebyshev or Manhattan radius), never below the exact EDT,
and the exact EDTs (brute force, separable, scipy) agree with each other.
Algorithm 3 taken literally reproduces the error of Fig. 3 (170 for 169).
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy import ndimage

import oracle
from paper_1209_3314_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rand_binary(rng, h, w, density):
    return (rng.random((h, w)) >= density).astype(np.uint8)


bins = st.tuples(st.integers(1, 24), st.integers(1, 24), st.sampled_from([0.01, 0.05, 0.2, 0.5, 0.9]),
                 st.integers(0, 2**31 - 1))


@settings(max_examples=200, deadline=None)
@given(bins, st.sampled_from([4, 8]))
def test_frontier_form_equals_dense_form(spec, conn):
    h, w, d, seed = spec
    B = rand_binary(np.random.default_rng(seed), h, w, d)
    s1, n1, st1 = oracle.edt_rounds(B, conn, return_stats=True)
    s2, n2, st2 = oracle.edt_dense(B, conn, return_stats=True)
    assert np.array_equal(s1, s2) and np.array_equal(n1, n2)
    assert st1["rounds"] == st2["rounds"]


@settings(max_examples=100, deadline=None)
@given(bins, st.sampled_from([4, 8]))
def test_consistency_and_lower_bound(spec, conn):
    h, w, d, seed = spec
    B = rand_binary(np.random.default_rng(seed), h, w, d)
    sq, nr = oracle.edt_rounds(B, conn)
    ex, _ = oracle.edt_exact_bf(B)
    if (B != 0).all():
        assert (sq == -1).all() and (nr == -1).all()
        return
    ys, xs = np.divmod(nr, w)
    yy, xx = np.mgrid[0:h, 0:w]
    assert np.array_equal(sq, (yy - ys) ** 2 + (xx - xs) ** 2)  # sqdist is the distance to the carried feature
    assert (B.flat[nr.ravel()] == 0).all()  # the carried pixel is a feature
    assert np.array_equal(sq == 0, B == 0)
    assert (sq >= ex).all()  # never better than the exact EDT


def test_exact_references_agree():
    rng = np.random.default_rng(4)
    for h, w, d in [(1, 1, 0.5), (13, 29, 0.05), (40, 33, 0.01), (64, 64, 0.3)]:
        B = rand_binary(rng, h, w, d)
        if (B != 0).all():
            B[0, 0] = 0
        bf, _ = oracle.edt_exact_bf(B)
        sep = oracle.edt_exact_sep(B)
        sci = np.rint(ndimage.distance_transform_edt(B) ** 2).astype(np.int64)
        assert np.array_equal(bf, sep) and np.array_equal(sep, sci)


@pytest.mark.parametrize("conn", [4, 8])
def test_one_row_and_column_are_exact(conn):
    """On a line every Voronoi cell is an interval, so propagation is exact,
    including the smallest-index choice among equidistant features."""
    rng = np.random.default_rng(9)
    for n in (1, 2, 5, 64):
        for d in (0.1, 0.5):
            B = rand_binary(rng, 1, n, d)
            for img in (B, B.T.copy()):
                s, nr = oracle.edt_rounds(img, conn)
                es, en = oracle.edt_exact_bf(img)
                assert np.array_equal(s, es) and np.array_equal(nr, en)
    B = np.ones((1, 9), np.uint8)
    B[0, 0] = B[0, 8] = 0
    s, nr = oracle.edt_rounds(B, conn)
    assert nr[0, 4] == 0  # tie at distance 4: the smaller feature index wins


@pytest.mark.parametrize("conn", [4, 8])
def test_single_feature_rounds_are_the_radius(conn):
    rng = np.random.default_rng(10)
    for _ in range(10):
        h, w = rng.integers(1, 30, 2)
        fy, fx = rng.integers(0, h), rng.integers(0, w)
        B = np.ones((h, w), np.uint8)
        B[fy, fx] = 0
        s, nr, st_ = oracle.edt_rounds(B, conn, return_stats=True)
        yy, xx = np.mgrid[0:h, 0:w]
        assert np.array_equal(s, (yy - fy) ** 2 + (xx - fx) ** 2)
        assert (nr == fy * w + fx).all()
        dy, dx = np.abs(yy - fy), np.abs(xx - fx)
        radius = int(np.maximum(dy, dx).max()) if conn == 8 else int((dy + dx).max())
        assert st_["rounds"] == radius  # a wave advances one step of N_G per round


def test_no_feature_and_all_features():
    for conn in (4, 8):
        s, nr = oracle.edt_rounds(np.ones((5, 6), np.uint8), conn)
        assert (s == -1).all() and (nr == -1).all()
        s, nr, st_ = oracle.edt_rounds(np.zeros((5, 6), np.uint8), conn, return_stats=True)
        assert (s == 0).all() and np.array_equal(nr, np.arange(30).reshape(5, 6)) and st_["rounds"] == 0


def test_fig3_error_of_algorithm3():
    """Sec. 2.2, Fig. 3: 8-connected propagation can leave a pixel with
    sqrt(170) although its nearest feature is at sqrt(169)."""
    with open(os.path.join(GOLDEN, "fig3_alg3.json")) as f:
        fx = json.load(f)
    B = np.ones((fx["height"], fx["width"]), np.uint8)
    for y, x in fx["features"]:
        B[y, x] = 0
    qy, qx = fx["pixel"]
    a, _ = oracle.edt_alg3(B, fx["conn"])
    ex = oracle.edt_exact_sep(B)
    assert a[qy, qx] == fx["alg3_sqdist"] == 170
    assert ex[qy, qx] == fx["exact_sqdist"] == 169


@pytest.mark.parametrize("conn", [4, 8])
def test_alg3_and_rounds_differ_only_where_inexact(conn):
    rng = np.random.default_rng(13)
    for _ in range(20):
        B = rand_binary(rng, 48, 48, 0.01)
        s, _ = oracle.edt_rounds(B, conn)
        a, _ = oracle.edt_alg3(B, conn)
        ex = oracle.edt_exact_sep(B)
        diff = s != a
        assert ((s[diff] != ex[diff]) | (a[diff] != ex[diff])).all()


def test_four_connected_propagation_is_an_approximation():
    """The oracle computes the propagation approximation, not the exact EDT."""
    B = synth.edt_input(256, 256, seed=3, coverage=0.3)
    s, _ = oracle.edt_rounds(B, 4)
    assert (s != oracle.edt_exact_sep(B)).any()


@pytest.mark.slow
def test_tolerance_against_exact_on_4k_workload():
    """The 4096^2 nucleus-like workload: at most 1e-4 of the pixels may differ
    from the exact EDT, by at most one pixel of distance."""
    B = synth.workload_edt_4k()
    s, _, st_ = oracle.edt_rounds(B, 8, return_stats=True)
    ex = oracle.edt_exact_sep(B)
    frac = float((s != ex).mean())
    err = float((np.sqrt(s.astype(np.float64)) - np.sqrt(ex.astype(np.float64))).max())
    assert frac <= 1e-4 and err <= 1.0
    assert st_["rounds"] > 0 and st_["items"] > B.size // 2
