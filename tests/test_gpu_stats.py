"""GPU parity of the per-component statistics (ccl_component_stats over the
library's own labels) against the oracle's statistics, field by field."""
import numpy as np
import pytest

import oracle
from paper_1708_08180_amd import workloads as wl
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

FIELDS = ("label", "area", "x_min", "y_min", "x_max", "y_max", "sum_x", "sum_y")


def gpu_stats(img, conn, equal=False, capacity=None):
    import torch
    from paper_1708_08180_amd import binding

    d = to_dev(img)
    lab = binding.label_equal(d, conn) if equal else binding.label(d, conn)
    rec = binding.component_stats(lab, capacity=capacity)
    torch.cuda.synchronize()
    return rec


def _cmp(img, conn, equal=False, what=""):
    say("stats %s %dx%d conn=%d equal=%s" % (what, img.shape[0], img.shape[1], conn, equal))
    got = gpu_stats(img, conn, equal)
    want = oracle.stats(img, conn, equal=equal)
    assert len(got) == len(want), "%s: %d components, want %d" % (what, len(got), len(want))
    for f in FIELDS:
        if not np.array_equal(got[f].astype(np.uint64), want[f].astype(np.uint64)):
            k = int(np.argmax(got[f].astype(np.uint64) != want[f].astype(np.uint64)))
            raise AssertionError("%s: field %s differs first at record %d (label %d): got %d want %d"
                                 % (what, f, k, want["label"][k], got[f][k], want[f][k]))


@pytest.mark.parametrize("conn", [8, 4])
def test_stats_small_and_ragged(conn):
    for seed, (H, W, p, g) in enumerate(((256, 256, 0.5, 1), (300, 257, 0.45, 1), (1, 1, 1.0, 1),
                                         (3, 1000, 0.5, 1), (129, 65, 0.6, 3), (70, 70, 0.2, 1))):
        _cmp(wl.bernoulli(H, W, p, 1200 + seed, g), conn, what="bern p=%.2f g=%d" % (p, g))


@pytest.mark.parametrize("conn", [8, 4])
def test_stats_closed_forms(conn):
    _cmp(np.zeros((50, 70), np.uint8), conn, what="empty")
    _cmp(np.ones((50, 70), np.uint8), conn, what="full")
    _cmp(wl.checkerboard(130, 190, 0), conn, what="checkerboard")   # 4-conn: every pixel alone
    _cmp(wl.rings(97, 131), conn, what="rings")
    _cmp(wl.serpentine(128, 200), conn, what="serpentine")


@pytest.mark.parametrize("conn", [8, 4])
def test_stats_equal_value(conn):
    rng = wl.rng_for(1301)
    img = rng.integers(0, 3, size=(300, 257), dtype=np.uint8)
    _cmp(img, conn, equal=True, what="3-valued")


def test_stats_full_size():
    # a percolating component spread over every block, and many small ones
    _cmp(wl.bernoulli(4096, 4096, 0.5, wl.sweep_seed(0.5, 1)), 8, what="bern 4096")
    _cmp(wl.smoothed_noise(2048, 2048, 4.0, 1302), 4, what="smoothed 2048")


def test_stats_capacity():
    img = wl.bernoulli(200, 300, 0.4, 1303)
    want = oracle.stats(img, 8)
    assert len(want) > 20
    got = gpu_stats(img, 8, capacity=10)
    assert len(got) == 10
    for f in FIELDS:
        assert np.array_equal(got[f].astype(np.uint64), want[f][:10].astype(np.uint64))
