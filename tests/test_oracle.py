"""Pins for the CPU oracle (CPU only).

The oracle is checked against references that do not flood-fill: boolean
transitive closure on every tiny image, closed forms, invariants,
``scipy.ndimage.label`` and a stored worked example.
"""
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_1708_08180_amd import workloads as wl
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("conn", [4, 8])
def test_exhaustive_small_shapes(conn):
    # every binary image with h*w <= 12, plus all 2^16 images of 4x4, 2x8, 8x2
    for (H, W) in pins.shapes_upto(12):
        pins.check_exhaustive(oracle.label, H, W, conn)
    for (H, W) in ((4, 4), (2, 8), (8, 2)):
        pins.check_exhaustive(oracle.label, H, W, conn)


@pytest.mark.parametrize("conn", [4, 8])
def test_foreground_value_does_not_matter(conn):
    # any nonzero value is foreground (1 and 255 give identical labels)
    pins.check_exhaustive(oracle.label, 3, 4, conn, fg=255)
    img = wl.bernoulli(40, 50, 0.5, 7)
    assert np.array_equal(oracle.label(img, conn), oracle.label(img * 255, conn))


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 16), st.integers(1, 16), st.floats(0.0, 1.0), st.integers(0, 2**31 - 1),
       st.sampled_from([4, 8]))
def test_random_vs_closure(H, W, p, seed, conn):
    img = wl.bernoulli(H, W, p, seed)
    want = pins.closure_labels(img[None], conn)[0]
    assert np.array_equal(oracle.label(img, conn), want)


def test_closed_forms():
    pins.check_closed_forms(oracle.label)


def test_pitch_is_not_the_raster_stride():
    pins.check_pitch(oracle.label, oracle.label)


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("conn", [4, 8])
def test_scipy_cross_check_256(seed, conn):
    img = wl.bernoulli(256, 256, 0.5, seed)
    lab = oracle.label(img, conn)
    assert np.array_equal(lab, pins.scipy_canonical(img, conn))
    pins.check_invariants(img, lab)
    pins.check_neighbour_consistency(img, lab, conn)


@pytest.mark.parametrize("p,g", [(0.5, 1), (0.3, 4), (0.9, 16)])
@pytest.mark.parametrize("conn", [4, 8])
def test_scipy_cross_check_sweep_cells(p, g, conn):
    # a few cells of the 4096^2 density x granularity sweep, cropped to 1024^2 for time
    img = wl.bernoulli(4096, 4096, p, wl.sweep_seed(p, g), g)[:1024, :1024].copy()
    assert np.array_equal(oracle.label(img, conn), pins.scipy_canonical(img, conn))


def test_scipy_cross_check_smoothed():
    img = wl.smoothed_noise(512, 640, 4.0, 30001)
    for conn in (4, 8):
        lab = oracle.label(img, conn)
        assert np.array_equal(lab, pins.scipy_canonical(img, conn))
        pins.check_invariants(img, lab)


def test_component_count_matches_scipy():
    from scipy import ndimage

    img = wl.bernoulli(300, 200, 0.45, 11)
    for conn in (4, 8):
        st_ = ndimage.generate_binary_structure(2, 1 if conn == 4 else 2)
        _, n = ndimage.label(img, structure=st_)
        assert pins.component_count(oracle.label(img, conn)) == n


def _read_golden(path):
    blocks, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                blocks[cur] = []
                continue
            blocks[cur].append([int(v) for v in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def test_golden_worked_example():
    g = _read_golden(os.path.join(GOLDEN, "worked_8x8.txt"))
    img = g["image"].astype(np.uint8)
    assert np.array_equal(oracle.label(img, 4), g["labels_conn4"].astype(np.uint32))
    assert np.array_equal(oracle.label(img, 8), g["labels_conn8"].astype(np.uint32))


def test_equal_value_variant_vs_closure():
    # literal "same property" semantics: every value class is labeled, background too
    for conn in (4, 8):
        for (H, W) in ((3, 3), (2, 5), (4, 3)):
            imgs = pins.all_images(H, W)
            want = pins.closure_labels(imgs, conn, mode="equal")
            for k in range(imgs.shape[0]):
                assert np.array_equal(oracle.label_equal(imgs[k], conn), want[k])
        rng = wl.rng_for(3)
        imgs = rng.integers(0, 3, size=(200, 5, 6)).astype(np.uint8)
        want = pins.closure_labels(imgs, conn, mode="equal")
        for k in range(imgs.shape[0]):
            assert np.array_equal(oracle.label_equal(imgs[k], conn), want[k])


def test_rejects_bad_arguments():
    img = np.zeros((4, 4), np.uint8)
    with pytest.raises(ValueError):
        oracle.label(img, 6)
    with pytest.raises(ValueError):
        oracle.label(np.zeros((2, 2, 2), np.uint8), 4)
