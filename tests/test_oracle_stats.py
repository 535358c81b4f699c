"""Pins of the oracle's per-component statistics (area, inclusive bounding
box, sums of column and row indices; records in increasing label order).

Independent references: scipy.ndimage's own labeling and per-label
reductions, statistics counted from transitive-closure labels on tiny
images, and closed forms of hand-built patterns."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1708_08180_amd import workloads as wl
from tests import pins


def scipy_stats(img: np.ndarray, conn: int, equal: bool = False) -> np.ndarray:
    """The same records from scipy.ndimage (its labeling, its reductions),
    ordered by each component's smallest raster index."""
    H, W = img.shape
    st = ndimage.generate_binary_structure(2, 2 if conn == 8 else 1)
    if equal:
        lab = np.zeros((H, W), np.int64)
        nxt = 0
        for v in np.unique(img):
            l, k = ndimage.label(img == v, structure=st)
            lab[l > 0] = l[l > 0] + nxt
            nxt += k
        n = nxt
    else:
        lab, n = ndimage.label(img != 0, structure=st)
    if n == 0:
        return np.zeros(0, oracle.STATS_DTYPE)
    idx = np.arange(1, n + 1)
    yy, xx = np.indices((H, W))
    raster = (yy * W + xx).astype(np.int64)
    out = np.zeros(n, oracle.STATS_DTYPE)
    out["label"] = ndimage.minimum(raster, lab, idx).astype(np.int64) + 1
    out["area"] = ndimage.sum_labels(np.ones((H, W)), lab, idx)
    boxes = ndimage.find_objects(lab)
    out["y_min"] = [b[0].start for b in boxes]
    out["y_max"] = [b[0].stop - 1 for b in boxes]
    out["x_min"] = [b[1].start for b in boxes]
    out["x_max"] = [b[1].stop - 1 for b in boxes]
    out["sum_x"] = np.rint(ndimage.sum_labels(xx.astype(np.float64), lab, idx)).astype(np.uint64)
    out["sum_y"] = np.rint(ndimage.sum_labels(yy.astype(np.float64), lab, idx)).astype(np.uint64)
    return np.sort(out, order="label")


def closure_stats(img: np.ndarray, conn: int, mode: str) -> np.ndarray:
    """Records counted pixel by pixel from transitive-closure labels."""
    lab = pins.closure_labels(img[None], conn, mode)[0]
    H, W = img.shape
    recs = {}
    for y in range(H):
        for x in range(W):
            L = int(lab[y, x])
            if L == 0:
                continue
            r = recs.setdefault(L, [L, 0, x, y, x, y, 0, 0])
            r[1] += 1
            r[2], r[3] = min(r[2], x), min(r[3], y)
            r[4], r[5] = max(r[4], x), max(r[5], y)
            r[6] += x
            r[7] += y
    return np.array([tuple(recs[k]) for k in sorted(recs)], dtype=oracle.STATS_DTYPE)


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("seed", range(4))
def test_stats_match_scipy(conn, seed):
    for H, W, p, g in ((64, 70, 0.5, 1), (101, 37, 0.3, 2), (50, 50, 0.7, 1)):
        img = wl.bernoulli(H, W, p, 900 + seed, g)
        assert np.array_equal(oracle.stats(img, conn), scipy_stats(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_equal_value_stats_match_scipy(conn):
    rng = wl.rng_for(77)
    img = rng.integers(0, 3, size=(40, 53), dtype=np.uint8)
    assert np.array_equal(oracle.stats(img, conn, equal=True), scipy_stats(img, conn, equal=True))


@pytest.mark.parametrize("conn", [4, 8])
def test_stats_brute_force_tiny(conn):
    rng = wl.rng_for(5)
    for _ in range(60):
        H, W = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        img = (rng.random((H, W)) < 0.5).astype(np.uint8)
        assert np.array_equal(oracle.stats(img, conn), closure_stats(img, conn, "binary"))
        img3 = rng.integers(0, 3, size=(H, W), dtype=np.uint8)
        assert np.array_equal(oracle.stats(img3, conn, equal=True), closure_stats(img3, conn, "equal"))


def test_stats_closed_forms():
    H, W = 21, 33
    # all foreground: one component covering the image
    s = oracle.stats(np.ones((H, W), np.uint8), 8)
    assert len(s) == 1
    assert tuple(s[0]) == (1, H * W, 0, 0, W - 1, H - 1, H * W * (W - 1) // 2, W * H * (H - 1) // 2)
    # empty image: no records
    assert len(oracle.stats(np.zeros((H, W), np.uint8), 8)) == 0
    # 4-connected checkerboard: every foreground pixel alone
    cb = wl.checkerboard(H, W, 0)
    s = oracle.stats(cb, 4)
    ys, xs = np.nonzero(cb)
    assert len(s) == len(ys)
    assert np.array_equal(s["label"], ys * W + xs + 1)
    assert (s["area"] == 1).all() and np.array_equal(s["x_min"], xs) and np.array_equal(s["y_max"], ys)
    # nested rings: ring t spans [t, H-1-t] x [t, W-1-t]
    s = oracle.stats(wl.rings(H, W), 8)
    corners = wl.ring_corners(H, W)
    assert len(s) == len(corners)
    for rec, (t, _) in zip(s, corners):
        top, left, bottom, right = t, t, H - 1 - t, W - 1 - t
        h, w = bottom - top + 1, right - left + 1
        area = w * h if h <= 2 or w <= 2 else 2 * w + 2 * (h - 2)
        assert tuple(rec)[:6] == (t * W + t + 1, area, left, top, right, bottom)
        # symmetric rings: centroid at the centre
        assert 2 * int(rec["sum_x"]) == area * (left + right)
        assert 2 * int(rec["sum_y"]) == area * (top + bottom)


def test_stats_agree_with_labels():
    # one record per distinct label, areas are the label counts
    img = wl.bernoulli(300, 257, 0.45, 12)
    for conn in (4, 8):
        lab = oracle.label(img, conn)
        s = oracle.stats(img, conn)
        labs, counts = np.unique(lab[lab > 0], return_counts=True)
        assert np.array_equal(s["label"], labs) and np.array_equal(s["area"], counts)
