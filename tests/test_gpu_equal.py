"""GPU parity of equal-value labeling (every value class, background
included) against the oracle's equal-value flood fill, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import workloads as wl
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

EQ_CONFIGS = [(64, 4), (64, 8), (32, 2), (32, 8), (16, 4)]


def gpu_label_equal(img, conn, config=None, pad=0):
    import torch
    from paper_1708_08180_amd import binding

    d = to_dev(img, pad)
    out = binding.label_equal(d, conn, config=config)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def _cmp(img, conn, config=None, pad=0, what=""):
    say("equal %s %dx%d conn=%d config=%s pad=%d" % (what, img.shape[0], img.shape[1], conn, config, pad))
    got = gpu_label_equal(img, conn, config, pad)
    want = oracle.label_equal(img, conn)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d mismatches, first at (%d,%d): got %d want %d"
                             % (what, len(bad), y, x, got[y, x], want[y, x]))


def levels(H, W, k, seed, g=1):
    """k-valued field, each g x g block one uniform value."""
    rng = wl.rng_for(seed)
    f = rng.integers(0, k, size=(-(-H // g), -(-W // g)), dtype=np.uint8)
    return np.ascontiguousarray(np.repeat(np.repeat(f, g, 0), g, 1)[:H, :W])


@pytest.mark.parametrize("config", EQ_CONFIGS)
@pytest.mark.parametrize("conn", [8, 4])
def test_equal_levels_every_config(config, conn):
    for seed, (H, W, k, g) in enumerate(((256, 256, 3, 1), (200, 333, 2, 1), (65, 129, 4, 2),
                                         (130, 70, 256, 1), (97, 191, 3, 5))):
        _cmp(levels(H, W, k, 700 + seed, g), conn, config, what="levels k=%d g=%d" % (k, g))


@pytest.mark.parametrize("conn", [8, 4])
def test_equal_binary_images_label_background_too(conn):
    img = wl.bernoulli(300, 257, 0.5, 41)
    _cmp(img, conn, what="binary")
    got = gpu_label_equal(img, conn)
    assert (got > 0).all()


@pytest.mark.parametrize("conn", [8, 4])
def test_equal_closed_forms(conn):
    H, W = 70, 130
    const = np.full((H, W), 9, np.uint8)
    assert (gpu_label_equal(const, conn) == 1).all()
    cb = wl.checkerboard(H, W, 0, fg=5)
    got = gpu_label_equal(cb, conn)
    if conn == 4:   # every pixel its own component
        assert np.array_equal(got, np.arange(1, H * W + 1, dtype=np.uint32).reshape(H, W))
    else:           # two diagonal classes: pixel 0 and pixel 1
        want = np.where(((np.indices((H, W)).sum(0)) % 2) == 0, 1, 2).astype(np.uint32)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("config", EQ_CONFIGS)
def test_equal_checkerboard_every_config(config):
    # 4-connectivity: every pixel is its own component, so every edge cell of
    # every tile is a root that the link pass resolves in the global forest
    # (the most such roots a link wavefront resolves: a 64-cell top row
    # plus the side cells of its rows, more than one lane round)
    H, W = 200, 300
    cb = wl.checkerboard(H, W, 0, fg=5)
    say("equal checkerboard %dx%d config=%s" % (H, W, config))
    got = gpu_label_equal(cb, 4, config=config)
    assert np.array_equal(got, np.arange(1, H * W + 1, dtype=np.uint32).reshape(H, W))
    _cmp(cb, 8, config, what="checkerboard")


@pytest.mark.parametrize("config", EQ_CONFIGS)
def test_equal_antidiagonals_many_boundary_pairs(config):
    # value 1 + (x + y) mod 4: under 8-connectivity every anti-diagonal is its
    # own component, so every top- and left-edge cell of a tile pairs with a
    # different component across the edge -- more distinct merge requests
    # than one wavefront holds at once (the dedupe runs in several rounds)
    H, W = 200, 300
    yy, xx = np.indices((H, W))
    img = (1 + (xx + yy) % 4).astype(np.uint8)
    _cmp(img, 8, config, what="antidiagonals")
    _cmp(img, 4, config, what="antidiagonals")


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (3, 70000 // 64), (129, 65), (64, 64)])
def test_equal_ragged_and_pitch(shape):
    H, W = shape
    img = levels(H, W, 3, H * 1000 + W)
    for conn in (8, 4):
        _cmp(img, conn, what="ragged")
        _cmp(img, conn, pad=13, what="ragged pitched")


def test_equal_full_size_quantized_noise():
    # 4096^2: smoothed noise quantized to 4 levels (large equal-valued regions
    # of every class), and 3-level pixel noise
    from scipy import ndimage

    rng = wl.rng_for(31001)
    z = ndimage.gaussian_filter(rng.standard_normal((4096, 4096), dtype=np.float32), 4.0)
    q = np.digitize(z, np.quantile(z, [0.25, 0.5, 0.75])).astype(np.uint8)
    for conn in (8, 4):
        _cmp(q, conn, what="quantized smooth 4096")
    _cmp(levels(4096, 4096, 3, 31002), 8, what="levels3 4096")
