"""Pins for the reconstruction oracle (Sec. 2.1).

The oracle's Fast Hybrid routine (Algorithm 2) and its brute-force definition
(iterated elementary geodesic dilation) are checked against each other and,
independently of both, against the threshold-decomposition closed form
computed with scipy's connected-component labelling, plus invariants and
special cases with closed-form answers.  A dropped neighbour, a wrong
raster/anti-raster neighbour set or a wrong propagation condition each fail one
of these.  (The explicit clamp J <- J ^ I has no observable effect: the first
raster scan clamps every pixel anyway.)
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy import ndimage

import oracle
from paper_1209_3314_amd import synth


def threshold_reconstruction(J, I, conn):
    """rho_I(J)(p) = max{t : p lies in a connected component of {I >= t} that
    meets {J ^ I >= t}} -- the grayscale reconstruction as a stack of binary
    reconstructions (each level extracts the mask components hit by the
    marker, Sec. 2.1), with components from scipy.ndimage.label."""
    Jc = np.minimum(J, I)
    struct = ndimage.generate_binary_structure(2, 2 if conn == 8 else 1)
    R = np.zeros(I.shape, np.int32)
    for t in range(1, int(I.max()) + 1):
        lab, _ = ndimage.label(I >= t, structure=struct)
        hit = np.unique(lab[(Jc >= t) & (lab > 0)])
        R += np.isin(lab, hit[hit > 0])
    return R.astype(np.uint8)


def random_pair(rng, h, w, levels):
    I = rng.integers(0, levels, (h, w)).astype(np.uint8)
    J = rng.integers(0, levels, (h, w)).astype(np.uint8)
    return J, I


images = st.tuples(st.integers(1, 20), st.integers(1, 20), st.sampled_from([2, 4, 256]), st.integers(0, 2**31 - 1))


@settings(max_examples=150, deadline=None)
@given(images, st.sampled_from([4, 8]))
def test_fh_equals_definition(spec, conn):
    h, w, levels, seed = spec
    J, I = random_pair(np.random.default_rng(seed), h, w, levels)
    assert np.array_equal(oracle.mr_fh(J, I, conn), oracle.mr_iterate(J, I, conn))


@settings(max_examples=60, deadline=None)
@given(images, st.sampled_from([4, 8]))
def test_definition_equals_threshold_decomposition(spec, conn):
    h, w, levels, seed = spec
    J, I = random_pair(np.random.default_rng(seed), h, w, min(levels, 16))
    assert np.array_equal(oracle.mr_iterate(J, I, conn), threshold_reconstruction(J, I, conn))


def test_full_range_threshold_decomposition():
    rng = np.random.default_rng(3)
    for conn in (4, 8):
        J, I = random_pair(rng, 24, 31, 256)
        assert np.array_equal(oracle.mr_fh(J, I, conn), threshold_reconstruction(J, I, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_small_workload_matches_definition(conn):
    J, I = synth.workload_mr_small()
    R = oracle.mr_fh(J, I, conn)
    assert np.array_equal(R, oracle.mr_iterate(J, I, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_invariants(conn):
    rng = np.random.default_rng(11)
    J, I = random_pair(rng, 40, 37, 256)
    R = oracle.mr_fh(J, I, conn)
    assert (np.minimum(J, I) <= R).all() and (R <= I).all()  # J ^ I <= R <= I
    assert np.array_equal(oracle.mr_fh(R, I, conn), R)  # idempotent
    assert np.array_equal(oracle.geodesic_dilation(R, I, conn), R)  # stable under delta_I
    J2 = np.maximum(J, rng.integers(0, 256, J.shape).astype(np.uint8))
    assert (oracle.mr_fh(J2, I, conn) >= R).all()  # monotone in the marker
    I2 = np.maximum(I, rng.integers(0, 256, I.shape).astype(np.uint8))
    assert (oracle.mr_fh(J, I2, conn) >= R).all()  # monotone in the mask


def test_4_below_8():
    rng = np.random.default_rng(12)
    J, I = random_pair(rng, 33, 41, 256)
    assert (oracle.mr_fh(J, I, 4) <= oracle.mr_fh(J, I, 8)).all()


@pytest.mark.parametrize("conn", [4, 8])
def test_special_cases(conn):
    rng = np.random.default_rng(5)
    I = rng.integers(0, 256, (17, 23)).astype(np.uint8)
    assert np.array_equal(oracle.mr_fh(I, I, conn), I)  # J = I
    assert np.array_equal(oracle.mr_fh(np.zeros_like(I), I, conn), np.zeros_like(I))  # J = 0
    J = rng.integers(0, 256, I.shape).astype(np.uint8)
    c = np.full(I.shape, 100, np.uint8)  # constant mask: everything floods to min(max J, c)
    assert (oracle.mr_fh(J, c, conn) == min(int(J.max()), 100)).all()


def one_dim_closed_form(J, I):
    """R(x) = max over y of min(J^I(y), min of I on [x, y]): on a line the only
    paths are intervals."""
    Jc = np.minimum(J, I).astype(int)
    n = len(I)
    R = np.zeros(n, int)
    for x in range(n):
        best = 0
        for y in range(n):
            lo, hi = min(x, y), max(x, y)
            best = max(best, min(Jc[y], int(I[lo:hi + 1].min())))
        R[x] = best
    return R.astype(np.uint8)


@pytest.mark.parametrize("conn", [4, 8])
def test_one_row_and_one_column(conn):
    rng = np.random.default_rng(8)
    for n in (1, 2, 7, 50):
        J, I = random_pair(rng, 1, n, 256)
        assert np.array_equal(oracle.mr_fh(J, I, conn)[0], one_dim_closed_form(J[0], I[0]))
        assert np.array_equal(oracle.mr_fh(J.T, I.T, conn)[:, 0], one_dim_closed_form(J[0], I[0]))


@pytest.mark.parametrize("conn", [4, 8])
def test_binary_reconstruction_extracts_marked_components(conn):
    """Binary case (Sec. 2.1, Fig. 1): the result is the union of the mask's
    connected components that contain a marker pixel."""
    rng = np.random.default_rng(21)
    I = (rng.random((40, 40)) < 0.55).astype(np.uint8)
    J = ((rng.random((40, 40)) < 0.02) & (I > 0)).astype(np.uint8)
    struct = ndimage.generate_binary_structure(2, 2 if conn == 8 else 1)
    lab, _ = ndimage.label(I, structure=struct)
    keep = np.unique(lab[J > 0])
    expect = np.isin(lab, keep[keep > 0]).astype(np.uint8)
    assert np.array_equal(oracle.mr_fh(J, I, conn), expect)


def test_marker_above_mask_is_clamped():
    rng = np.random.default_rng(2)
    J, I = random_pair(rng, 19, 13, 256)
    assert np.array_equal(oracle.mr_fh(J, I, 8), oracle.mr_fh(np.minimum(J, I), I, 8))


def test_stats_are_counts():
    J, I = synth.workload_mr_small()
    _, st8 = oracle.mr_fh(J, I, 8, return_stats=True)
    assert st8["pops"] == st8["initial"] + st8["pushes"]  # every queued pixel is popped once
    assert st8["depth"] >= 1


@pytest.mark.parametrize("conn", [4, 8])
def test_scans_do_monotone_work(conn):
    """A raster scan carries a marker at the top-left corner through a flat
    mask in one pass, and the anti-raster scan carries one from the bottom-right
    corner, so Algorithm 2 queues nothing (Q_ref = 0) -- this pins the N+/N-
    neighbour sets of the two scans, which the result alone cannot."""
    I = np.full((9, 13), 255, np.uint8)
    for corner in [(0, 0), (8, 12)]:
        J = np.zeros_like(I)
        J[corner] = 200
        R, stt = oracle.mr_fh(J, I, conn, return_stats=True)
        assert (R == 200).all()
        assert stt["initial"] == 0 and stt["pops"] == 0


# ---- reconstruction by erosion (the dual instance) -----------------------------

def threshold_reconstruction_erode(J, I, conn):
    """rho*_I(J)(p) = min{t : p lies in a connected component of {I <= t}
    that meets {J v I <= t}} -- erosion-reconstruction as a stack of binary
    reconstructions of the lower level sets, with scipy's labelling."""
    Jc = np.maximum(J, I)
    struct = ndimage.generate_binary_structure(2, 2 if conn == 8 else 1)
    R = np.full(I.shape, 255, np.int32)
    for t in range(254, int(I.min()) - 1, -1):
        lab, _ = ndimage.label(I <= t, structure=struct)
        hit = np.unique(lab[(Jc <= t) & (lab > 0)])
        R -= np.isin(lab, hit[hit > 0])
    return R.astype(np.uint8)


@settings(max_examples=120, deadline=None)
@given(images, st.sampled_from([4, 8]))
def test_erode_equals_its_definition(spec, conn):
    h, w, levels, seed = spec
    J, I = random_pair(np.random.default_rng(seed), h, w, levels)
    assert np.array_equal(oracle.mr_erode(J, I, conn), oracle.mr_erode_iterate(J, I, conn))


@settings(max_examples=40, deadline=None)
@given(images, st.sampled_from([4, 8]))
def test_erode_definition_equals_threshold_decomposition(spec, conn):
    h, w, levels, seed = spec
    rng = np.random.default_rng(seed)
    J, I = random_pair(rng, h, w, min(levels, 16))
    J, I = (255 - J).astype(np.uint8), (255 - I).astype(np.uint8)  # levels near the top of the range
    assert np.array_equal(oracle.mr_erode_iterate(J, I, conn), threshold_reconstruction_erode(J, I, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_erode_is_the_dual_of_dilate(conn):
    """rho*_I(J) = 255 - rho_{255-I}(255-J) (complementing swaps the order)."""
    rng = np.random.default_rng(21)
    for _ in range(5):
        J, I = random_pair(rng, 37, 41, 256)
        got = oracle.mr_erode(J, I, conn)
        assert np.array_equal(got, 255 - oracle.mr_fh(255 - J, 255 - I, conn))
    J, I = synth.workload_mr_small()
    Jd = np.minimum(I.astype(np.int16) + 32, 255).astype(np.uint8)  # a marker above the mask
    assert np.array_equal(oracle.mr_erode(Jd, I, conn), 255 - oracle.mr_fh(255 - Jd, 255 - I, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_erode_invariants(conn):
    rng = np.random.default_rng(12)
    J, I = random_pair(rng, 33, 29, 256)
    R = oracle.mr_erode(J, I, conn)
    assert (I <= R).all() and (R <= np.maximum(J, I)).all()
    assert np.array_equal(oracle.mr_erode(R, I, conn), R)  # idempotent
    assert np.array_equal(oracle.geodesic_erosion(R, I, conn), R)  # stable under one more erosion
    assert np.array_equal(oracle.mr_erode(I, I, conn), I)  # marker = mask
    assert np.array_equal(oracle.mr_erode(np.full_like(I, 255), I, conn), np.full_like(I, 255))  # nothing to descend from
